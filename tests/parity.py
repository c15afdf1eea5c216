"""Shared helpers for the GPU parity tests: run a batch through the HIP
decoder (via the C-ABI) and through the oracle, and compare."""

from __future__ import annotations

import numpy as np

import oracle
import synth

NP_DT = {"f32": np.float32, "i16": np.int16, "i8": np.int8}
REL_TOL = 1e-5  # metric tolerance for float32 (|dPM| <= 1e-5 |PM|)


def gpu_decode(code, L, llr_np, dtype, spc_max=4, mode=0, plan=None):
    import torch

    import paper_1505_01466_amd as pk

    if plan is None:
        plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, L, dtype, spc_max, mode)
    llr = torch.from_numpy(np.ascontiguousarray(llr_np)).to("cuda")
    u, ok, pm = plan.decode(llr)
    torch.cuda.synchronize()
    return u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()


def oracle_decode(code, L, llr_np, dtype, spc_max=4, mode=0):
    return oracle.decode_tree(code.N, code.K, code.frozen, code.poly, code.r, L, llr_np, dtype,
                              spc_max=spc_max, mode=mode)


def compare(gpu, ref, dtype, what=""):
    """Integer dtypes: identical bits, CRC flags and metrics on every frame.
    float32: identical decisions and CRC flags, metrics within REL_TOL, on
    every frame the oracle did not flag as a metric near-tie.  Returns the
    number of frames that are bit-identical in every output."""
    u_g, ok_g, pm_g = gpu
    u_o, ok_o, pm_o, nt = ref
    F = u_o.shape[0]
    assert u_g.shape == u_o.shape, what
    same_u = (u_g == u_o).all(axis=1)
    same_ok = ok_g == ok_o
    if dtype == "f32":
        pm_g = pm_g.astype(np.float64)
        close = np.abs(pm_g - pm_o) <= REL_TOL * np.abs(pm_o) + 1e-6
        good = same_u & same_ok & close
        bad = np.flatnonzero(~good & (nt == 0))
        assert bad.size == 0, (
            f"{what}: {bad.size}/{F} frames differ without a near-tie, first {bad[:8]}; "
            f"pm gpu {pm_g[bad[:4]]} oracle {pm_o[bad[:4]]}")
        exact = same_u & same_ok & (pm_g == pm_o)
        return int(exact.sum())
    pm_g = pm_g.astype(np.int64)
    bad = np.flatnonzero(~(same_u & same_ok & (pm_g == pm_o.astype(np.int64))))
    assert bad.size == 0, (f"{what}: {bad.size}/{F} frames differ, first {bad[:8]}; "
                           f"pm gpu {pm_g[bad[:4]]} oracle {pm_o[bad[:4]]}")
    return F


def batch(N, K, r, poly, design, F, ebn0, seed, dtype):
    code = synth.make_code(N, K, r, poly, design)
    return code, synth.make_batch(code, F, ebn0, seed, dtype)
