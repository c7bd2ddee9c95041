"""Plain FP64 CPU oracle for the LGDM hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call anything in this package.
It shares no code with the HIP path (paper_2301_06503_amd/) and imports
nothing from it; the only common input is the seeded problem definitions in
lgdm_workloads.

Every function cites the passage of the paper it follows.  Readings of
passages that are silent, ambiguous or garbled are listed in the module
docstring of oracle.lgdm.

Parity status: every function here is pinned by the not-gpu tests in
tests/test_oracle_pins.py, tests/test_oracle_fe.py, tests/test_oracle_coupling.py
(the Eq. 2 coupling variant) and tests/test_oracle_mixed.py (the mixed-order
elements of oracle.mixed_order), except the full load-displacement curve
shapes, which the paper only shows in figures (parity unpinned for the curve
shapes).
"""
from .lgdm import *  # noqa: F401,F403
from .mixed_order import *  # noqa: F401,F403
