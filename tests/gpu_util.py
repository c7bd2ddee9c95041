"""Helpers shared by the GPU parity tests: run a problem through the C ABI
and compare against the oracle."""
import numpy as np

import lgdm_workloads as W


def context(prob, precision=0):
    from paper_2301_06503_amd import binding
    ctx = binding.Context(device=0, precision=precision)
    ctx.setup_problem(prob)
    return ctx


def block_masks(row_ptr, col_idx, nd):
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    re = (rows % nd) == nd - 1
    ce = (col_idx % nd) == nd - 1
    return {"uu": ~re & ~ce, "ue": ~re & ce, "eu": re & ~ce, "ee": re & ce}


def blockwise_error(a, b, row_ptr, col_idx, nd):
    """max |a - b| / max |b| per block type (uu, ue, eu, ee)."""
    out = {}
    for k, m in block_masks(row_ptr, col_idx, nd).items():
        if not m.any():
            continue
        scale = np.abs(b[m]).max()
        err = np.abs(a[m] - b[m]).max()
        out[k] = err / scale if scale > 0 else err
    return out


def fieldwise_error(a, b, nd):
    out = {}
    for name, sl in (("u", np.arange(len(a)) % nd != nd - 1), ("e", np.arange(len(a)) % nd == nd - 1)):
        scale = np.abs(b[sl]).max()
        err = np.abs(a[sl] - b[sl]).max()
        out[name] = err / scale if scale > 0 else err
    return out


def tiny_problems():
    """Small problems the oracle finishes in well under a second, spanning
    several assembly workgroups and ragged tails."""
    m_ps = W.base_material()
    m_pe = W.base_material(plane=1)
    out = {
        "bar1d_37": W.bar1d(nx=37, lx=37.0, u_end=0.01, weak_elem=18, n_increments=30,
                            material=W.base_material(beta=25.0)),
        "sen2d_13x7_ps": W.sen2d(nx=13, ny=7, lx=26.0, ly=14.0, notch_len=4, u_top=0.006,
                                 n_increments=30, material=m_ps),
        "sen2d_13x7_pe": W.sen2d(nx=13, ny=7, lx=26.0, ly=14.0, notch_len=4, u_top=0.006,
                                 n_increments=30, material=m_pe),
        "beam3d_10x4x3": W.beam3d(nx=10, ny=4, nz=3, lx=40.0, ly=16.0, lz=12.0, u_load=-0.02,
                                  n_increments=20),
        "beam3d_24x8x6": W.beam3d(nx=24, ny=8, nz=6, lx=96.0, ly=32.0, lz=24.0, u_load=-0.04,
                                  n_increments=20),
    }
    d = W.beam3d(nx=6, ny=4, nz=3, lx=24.0, ly=16.0, lz=12.0, u_load=-0.02, n_increments=20)
    d.coords = W.perturbed_coords(d, seed=3, amp=0.2)
    d.name = "beam3d_6x4x3_distorted"
    out[d.name] = d
    q = W.sen2d(nx=9, ny=6, lx=18.0, ly=12.0, notch_len=3, u_top=0.02, n_increments=20)
    q.coords = W.perturbed_coords(q, seed=5, amp=0.25)
    q.name = "sen2d_9x6_distorted"
    out[q.name] = q
    return out
