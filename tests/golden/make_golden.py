"""Writes the stored expected values of the GPU parity tests.  Runs the FP64
oracle only (tests/golden/ holds its outputs; nothing here comes from the
HIP path).

  c3p_oracle_path.npz   the 64 x 16 x 8 beam (the parity subsample of the
                        256 x 64 x 32 workload), first N_INC increments of
                        its load path, Newton to ||R||/||F|| < 1e-10 with
                        direct solves: damage and kappa per Gauss point and
                        the reaction after each increment

Usage: python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lgdm_workloads as W  # noqa: E402
from oracle.lgdm import Oracle  # noqa: E402

N_INC = 4


def c3p_path():
    prob = W.config("c3p")
    o = Oracle(prob)
    D, kappa, reaction, iters = [], [], [], []
    for n in range(1, N_INC + 1):
        t0 = time.time()
        r = o.solve_increment(tol=1e-10, max_iter=40)
        assert r["converged"], n
        D.append(o.D_n.copy())
        kappa.append(o.kappa_n.copy())
        reaction.append(r["reaction"])
        iters.append(r["iters"])
        print("increment %d: %d Newton iterations, max D %.4f (%.0f s)" % (n, r["iters"], o.D_n.max(),
                                                                          time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "c3p_oracle_path.npz"), D=np.array(D), kappa=np.array(kappa),
                        reaction=np.array(reaction), newton=np.array(iters), tol_newton=1e-10)


if __name__ == "__main__":
    c3p_path()
