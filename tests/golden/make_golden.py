"""Writes the stored expected values of the GPU parity tests.  Runs the FP64
oracle only (tests/golden/ holds its outputs; nothing here comes from the
HIP path).

Each file is one load path of Algorithm 2 run by the oracle with Newton to
||R||/||F|| < 1e-10 per field and direct solves, uniform load steps and no
step cutting:

  c3p_path.npz   the 64 x 16 x 8 beam (the parity subsample of the
                 256 x 64 x 32 workload) through its load peak and on into
                 the softening branch, until POST increments after the peak
                 or until the oracle's Newton iteration fails
  c1_path.npz    the 200 x 100 notched plate, every increment of its path
                 (or until the oracle's Newton iteration fails)

Contents: `reaction[n]`, `newton[n]` (Newton iterations of increment n+1),
`max_D[n]`, and the damage of every Gauss point after every committed
increment, stored sparsely: the history variable is a running maximum
(Eq. A.2) and D is nondecreasing in it (Eq. A.1), so a Gauss point damaged
at some increment stays damaged after it; `idx` lists the Gauss points
damaged at the last stored increment and `D[n]` their damage after increment
n+1 (every other Gauss point has D = 0 throughout); with --kappa, `kappa[n]`
holds their history variable after increment n+1 (to tell a history-band
tie, reading A18, from a damage error; stored for c3p, left out of the
larger c1 file).  `stopped` is the first
increment the oracle could not converge (0 if none), `peak` the increment of
the largest |reaction|.

Each increment is also written to a part file in --parts, so a run can be
stopped and resumed; `pack` builds the stored file from the parts.

Usage:
  python tests/golden/make_golden.py run c3p [--post 12] [--parts DIR]
  python tests/golden/make_golden.py run c1 [--parts DIR]
  python tests/golden/make_golden.py pack c3p --kappa [--parts DIR]
  python tests/golden/make_golden.py pack c1 [--parts DIR]
"""
import argparse
import glob
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lgdm_workloads as W  # noqa: E402
from oracle.lgdm import Oracle  # noqa: E402

TOL = 1e-10
MAX_NEWTON = 40


def _part(parts, name, n):
    return os.path.join(parts, "%s_%04d.npz" % (name, n))


def _load_parts(parts, name):
    files = sorted(glob.glob(os.path.join(parts, name + "_[0-9][0-9][0-9][0-9].npz")))
    return [dict(np.load(f)) for f in files]


def run(name, parts, post, max_inc):
    os.makedirs(parts, exist_ok=True)
    prob = W.config(name)
    o = Oracle(prob)
    done = _load_parts(parts, name)
    if done:
        last = done[-1]
        o.x = last["x"].copy()
        o.kappa_n = last["kappa"].copy()
        o.D_n = last["D"].copy()
        o.increment = int(last["n"])
        if int(last["failed"]):
            print("%s: stopped at increment %d (resume refused)" % (name, o.increment), flush=True)
            return
    n_inc = min(prob.n_increments, max_inc)
    reactions = [abs(float(p["reaction"])) for p in done if not int(p["failed"])]
    while o.increment < n_inc:
        n = o.increment + 1
        t0 = time.time()
        r = o.solve_increment(tol=TOL, max_iter=MAX_NEWTON)
        if not r["converged"]:
            h = r["history"][-1]
            np.savez(_part(parts, name, n), n=n, failed=1, x=o.x, kappa=o.kappa_n, D=o.D_n,
                     reaction=0.0, newton=r["iters"], res_u=h["res_u"] / max(h["ref_u"], 1e-300),
                     res_e=h["res_e"] / max(h["ref_e"], 1e-300))
            print("%s increment %d: Newton did not converge in %d iterations (last |R_u|/|F_u| %.3e, "
                  "|R_e|/|F_e| %.3e)" % (name, n, r["iters"], h["res_u"] / max(h["ref_u"], 1e-300),
                                        h["res_e"] / max(h["ref_e"], 1e-300)), flush=True)
            return
        np.savez(_part(parts, name, n), n=n, failed=0, x=o.x, kappa=o.kappa_n, D=o.D_n,
                 reaction=r["reaction"], newton=r["iters"], res_u=0.0, res_e=0.0)
        reactions.append(abs(r["reaction"]))
        peak = int(np.argmax(reactions)) + 1
        print("%s increment %d: %d Newton iterations, reaction %.6g, max D %.6f, peak so far %d (%.0f s)"
              % (name, n, r["iters"], r["reaction"], float(o.D_n.max()), peak, time.time() - t0),
              flush=True)
        if post is not None and n - peak >= post and reactions[-1] < 0.98 * reactions[peak - 1]:
            return


def pack(name, parts, with_kappa):
    ps = _load_parts(parts, name)
    ok = [p for p in ps if not int(p["failed"])]
    stopped = next((int(p["n"]) for p in ps if int(p["failed"])), 0)
    assert ok and [int(p["n"]) for p in ok] == list(range(1, len(ok) + 1))
    Dlast = ok[-1]["D"]
    idx = np.flatnonzero(Dlast > 0).astype(np.int32)
    D = np.stack([p["D"][idx] for p in ok])
    extra = {"kappa": np.stack([p["kappa"][idx] for p in ok])} if with_kappa else {}
    for p in ok:
        assert not np.any(np.delete(p["D"], idx) != 0.0)
    reaction = np.array([float(p["reaction"]) for p in ok])
    np.savez_compressed(os.path.join(HERE, "%s_path.npz" % name), idx=idx, D=D, reaction=reaction,
                        newton=np.array([int(p["newton"]) for p in ok]),
                        max_D=np.array([float(p["D"].max()) for p in ok]),
                        n_gauss=len(Dlast), tol_newton=TOL, max_newton=MAX_NEWTON, stopped=stopped,
                        peak=int(np.argmax(np.abs(reaction))) + 1, **extra)
    print("%s: %d increments, %d damaged Gauss points of %d, peak at %d, stopped %d" %
          (name, len(ok), len(idx), len(Dlast), int(np.argmax(np.abs(reaction))) + 1, stopped))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["run", "pack"])
    ap.add_argument("name", choices=["c3p", "c1"])
    ap.add_argument("--parts", default=os.path.join(HERE, "parts"))
    ap.add_argument("--post", type=int, default=None, help="stop this many increments after the peak")
    ap.add_argument("--max-inc", type=int, default=10 ** 9)
    ap.add_argument("--kappa", action="store_true", help="pack: also store the history variable")
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.name, a.parts, a.post if a.post is not None else (12 if a.name == "c3p" else None), a.max_inc)
    else:
        pack(a.name, a.parts, a.kappa)
