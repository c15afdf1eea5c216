"""Lists of 64 and 128 paths (Sec. VII-B compares CRC lengths at L = 128):
parity with the oracle on the paper's (1024,860) polar-CRC codes, on small
and degenerate codes, on selections with up to 1024 candidates, and across
launch shapes and mixed launches."""

import sys

import numpy as np
import pytest

import synth

from parity import batch, compare, gpu_decode, oracle_decode

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pk():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_01466_amd as pk

    return pk


def _random_code(rng, N):
    K = int(rng.integers(1, N + 1))
    frozen = np.ones(N, np.uint8)
    frozen[rng.choice(N, K, replace=False)] = 0
    r = int(rng.integers(0, min(K - 1, 8) + 1))
    poly = {0: 0, 1: 0x1, 2: 0x3, 3: 0x3, 4: 0x3, 5: 0x5, 6: 0x3, 7: 0x9, 8: 0x07}[r]
    return synth.PolarCode(N=N, K=K, r=r, poly=poly, design_ebn0_db=0.0, frozen=frozen)


@pytest.mark.parametrize("dtype", ["i8", "i16", "f32"])
@pytest.mark.parametrize("N", [8, 32, 128])
def test_small_codes_large_lists(pk, dtype, N):
    rng = np.random.default_rng(5000 + N)
    for trial in range(4):
        code = _random_code(rng, N)
        for L in (64, 128):
            for mode, spc_max in ((0, 4), (0, N), (1, 4)):
                _say(f"N={N} K={code.K} r={code.r} L={L} mode={mode} spc={spc_max} {dtype}")
                b = synth.make_batch(code, 37, 1.0, (N, trial, L, 7), dtype)
                g = gpu_decode(code, L, b.llr, dtype, spc_max, mode)
                o = oracle_decode(code, L, b.llr, dtype, spc_max, mode)
                compare(g, o, dtype, f"N={N} L={L} mode={mode}")


# The CRC-length comparison: 860 payload bits with an 8- or a 32-bit CRC,
# the polar code's dimension raised by the CRC length.
@pytest.mark.parametrize("dtype", ["f32", "i16", "i8"])
@pytest.mark.parametrize("r,poly", [(8, synth.CRC8_POLY), (32, synth.CRC32_POLY)])
@pytest.mark.parametrize("L", [64, 128])
def test_1024_860_crc_lengths(pk, dtype, r, poly, L):
    for ebn0 in (2.5, 3.5):
        code, b = batch(1024, 860 + r, r, poly, 4.0, 200, ebn0, (9, r, L, int(ebn0 * 2)), dtype)
        _say(f"(1024,{860 + r}) CRC-{r} L={L} {dtype} {ebn0} dB")
        g = gpu_decode(code, L, b.llr, dtype)
        o = oracle_decode(code, L, b.llr, dtype)
        compare(g, o, dtype, f"(1024,{860 + r}) L={L} {ebn0} dB")


@pytest.mark.parametrize("dtype", ["f32", "i8"])
@pytest.mark.parametrize("L", [64, 128])
def test_wide_selections(pk, dtype, L):
    """Long SPC nodes (8 candidates each) in deep noise: up to 8 L = 1024
    candidates per selection, most of them above the rank-0 threshold."""
    code, b = batch(512, 256, 8, synth.CRC8_POLY, 2.0, 120, -1.0, (10, L), dtype)
    _say(f"(512,256) SPC-{512} L={L} {dtype} -1 dB")
    g = gpu_decode(code, L, b.llr, dtype, spc_max=512)
    o = oracle_decode(code, L, b.llr, dtype, spc_max=512)
    compare(g, o, dtype, f"(512,256) L={L} wide")


@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_headline_code_at_L128(pk, dtype):
    code, b = batch(2048, 1723, 32, synth.CRC32_POLY, 4.0, 96, 3.5, (11,), dtype)
    _say(f"(2048,1723) L=128 {dtype}")
    g = gpu_decode(code, 128, b.llr, dtype)
    o = oracle_decode(code, 128, b.llr, dtype)
    compare(g, o, dtype, "(2048,1723) L=128")


@pytest.mark.parametrize("L,threads,budget", [(64, 64, 0), (64, 128, 0), (64, 256, 32768),
                                              (128, 128, 0), (128, 256, 0), (128, 512, 65536),
                                              (128, 128, 4096), (128, 1024, 0), (64, 1024, 0),
                                              (32, 1024, 0)])
def test_launch_shapes(pk, L, threads, budget):
    """Including a budget below the path tables' own size: every tree level
    then lives in the workspace."""
    import torch

    code, b = batch(1024, 892, 32, synth.CRC32_POLY, 4.0, 150, 3.0, (12, L, threads), "i16")
    _say(f"(1024,892) L={L} threads={threads} budget={budget} i16")
    plan = pk.Plan(1024, 892, code.frozen, code.poly, 32, L, "i16", threads=threads,
                   lds_budget=budget)
    if budget == 4096:
        assert plan.info()["first_global_stage"] == 0
    g = gpu_decode(code, L, b.llr, "i16", plan=plan)
    o = oracle_decode(code, L, b.llr, "i16")
    compare(g, o, "i16", f"L={L} threads={threads}")
    plan.close()
    torch.cuda.synchronize()


def test_plan_rejects_one_wavefront_for_128_paths(pk):
    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.0)
    with pytest.raises(pk.PsclError):
        pk.Plan(256, 128, code.frozen, code.poly, 8, 128, "i8", threads=64)


def test_mixed_launch_with_large_lists(pk):
    """A launch mixing L = 128, 64 and 8 plans (int8: the group raises its
    workgroups to 128 threads for the 128-path plan)."""
    import torch

    specs = [(1024, 868, 8, synth.CRC8_POLY, 128, 3.0), (256, 128, 8, synth.CRC8_POLY, 64, 1.5),
             (512, 430, 32, synth.CRC32_POLY, 8, 3.5)]
    plans, work, refs = [], [], []
    for i, (N, K, r, poly, L, e) in enumerate(specs):
        code, b = batch(N, K, r, poly, 2.5 if K <= N // 2 else 4.0, 70 + 13 * i, e, (13, i), "i8")
        plans.append(pk.Plan(N, K, code.frozen, poly, r, L, "i8"))
        work.append((i, torch.from_numpy(b.llr).cuda()))
        refs.append((code, L, b))
    outs = pk.decode_mixed(plans, work)
    torch.cuda.synchronize()
    for (code, L, b), (u, ok, pm) in zip(refs, outs):
        _say(f"mixed ({code.N},{code.K}) L={L}")
        o = oracle_decode(code, L, b.llr, "i8")
        compare((u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()), o, "i8", f"mixed L={L}")


@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_largest_code_and_ragged_batches_at_L128(pk, dtype):
    """N = 4096 at L = 128, and batches of 0, 1 and 3 frames."""
    import torch

    code, b = batch(4096, 3441, 32, synth.CRC32_POLY, 4.0, 24, 3.5, (14,), dtype)
    _say(f"(4096,3441) L=128 {dtype}")
    g = gpu_decode(code, 128, b.llr, dtype)
    o = oracle_decode(code, 128, b.llr, dtype)
    compare(g, o, dtype, "(4096,3441) L=128")
    plan = pk.Plan(4096, 3441, code.frozen, code.poly, 32, 128, dtype)
    for F in (0, 1, 3):
        u, ok, pm = plan.decode(torch.from_numpy(np.ascontiguousarray(b.llr[:F])).cuda())
        torch.cuda.synchronize()
        assert u.shape == (F, 3441)
        if F:
            compare((u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()),
                    tuple(x[:F] for x in o), dtype, f"ragged F={F}")
    plan.close()
