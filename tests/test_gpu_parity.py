"""Parity of the HIP decoder with the CPU oracle, element by element, on
seeded synthetic frames (BPSK-AWGN, random payloads, CRC inside K).

Integer LLRs must match bit for bit (decisions, CRC flags, path metrics);
float32 must match decisions and CRC flags with metrics within 1e-5
relative, except on frames the oracle reports as metric near-ties."""

import sys

import numpy as np
import pytest

import synth

from parity import batch, compare, gpu_decode, oracle_decode

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_01466_amd  # noqa: F401  (fails loudly without the library)


# ---------------------------------------------------------------------------
# Small and degenerate codes: every node class at the root and below, every
# list size, both tree modes, SPC-4 and longer SPC nodes.
# ---------------------------------------------------------------------------

def _random_code(rng, N):
    K = int(rng.integers(1, N + 1))
    frozen = np.ones(N, np.uint8)
    frozen[rng.choice(N, K, replace=False)] = 0
    r = int(rng.integers(0, min(K - 1, 8) + 1))  # at least one payload bit
    poly = {0: 0, 1: 0x1, 2: 0x3, 3: 0x3, 4: 0x3, 5: 0x5, 6: 0x3, 7: 0x9, 8: 0x07}[r]
    return synth.PolarCode(N=N, K=K, r=r, poly=poly, design_ebn0_db=0.0, frozen=frozen)


@pytest.mark.parametrize("dtype", ["i8", "i16", "f32"])
@pytest.mark.parametrize("N", [2, 4, 8, 16, 32, 64])
def test_small_codes(dtype, N):
    rng = np.random.default_rng(1000 + N)
    for trial in range(6):
        code = _random_code(rng, N)
        for L in (1, 2, 4, 8, 16, 32):
            for mode, spc_max in ((0, 4), (0, N), (1, 4)):
                _say(f"N={N} K={code.K} r={code.r} L={L} mode={mode} spc={spc_max} {dtype}")
                b = synth.make_batch(code, 37, 1.0, (N, trial, L), dtype)
                g = gpu_decode(code, L, b.llr, dtype, spc_max, mode)
                o = oracle_decode(code, L, b.llr, dtype, spc_max, mode)
                compare(g, o, dtype, f"N={N} L={L} mode={mode}")


# ---------------------------------------------------------------------------
# The workloads: (1024,512) CRC-8 L=4; (2048,1723) CRC-32 L=32;
# (1024,860) CRC-32 L in {2..32}.
# ---------------------------------------------------------------------------

def _best_metric_fails_crc(code, L, llr, dtype):
    """Frames whose best-metric final path fails the CRC while another
    path passes (from the oracle's final list), so that the decoder has to
    fall back to a lower-metric path."""
    import oracle

    info = np.flatnonzero(code.frozen == 0)
    out = []
    for f in range(llr.shape[0]):
        cw, pm = oracle.decode_tree_list(code.N, code.K, code.frozen, L, llr[f], dtype)
        best = int(np.argsort(-pm, kind="stable")[0])
        ok = [oracle.crc(oracle.polar_transform(cw[j])[info], code.poly, code.r) == 0
              for j in range(cw.shape[0])]
        if not ok[best] and any(ok):
            out.append(f)
    return out


@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_crc_pick_below_the_best_metric(dtype):
    code, b = batch(256, 128, 8, synth.CRC8_POLY, 2.0, 300, 1.5, (7, 1), dtype)
    frames = _best_metric_fails_crc(code, 8, b.llr, dtype)
    _say(f"(256,128) L=8 {dtype}: {len(frames)} frames pick below the best metric")
    assert len(frames) >= 10
    g = gpu_decode(code, 8, b.llr, dtype)
    o = oracle_decode(code, 8, b.llr, dtype)
    compare(g, o, dtype, f"(256,128) L=8 {dtype} fallback pick")
    assert o[1][frames].all()  # each of those frames does find a passing path


def _wilson(k, n, z=1.959964):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * ((p * (1 - p) / n + z * z / (4 * n * n)) ** 0.5) / d
    return max(0.0, c - h), min(1.0, c + h)


@pytest.mark.parametrize("mode", [0, 1])
def test_1024_512_crc8_L4_f32(mode):
    """The (1024,512) CRC-8 L = 4 workload at 2.5 dB, its full 10,000
    frames: element by element against decoder A in both tree modes; the
    unrolled SC-list mode also element by element against the bit-by-bit
    SC-list decoder B, and the Dec-SPC-4 tree's frame error rate inside
    decoder B's 95 % interval widened by its own (overlapping intervals)."""
    import oracle

    code, b = batch(1024, 512, 8, synth.CRC8_POLY, 2.5, 10000, 2.5, (1, mode), "f32")
    _say(f"(1024,512) L=4 f32 mode={mode}, {b.F} frames")
    g = gpu_decode(code, 4, b.llr, "f32", mode=mode)
    o = oracle_decode(code, 4, b.llr, "f32", mode=mode)
    exact = compare(g, o, "f32", "(1024,512)", max_excused=b.F // 100)
    assert exact >= 0.99 * b.F
    s = oracle.decode_scl(1024, 512, code.frozen, code.poly, 8, 4, b.llr, "f32")
    if mode == 1:
        compare(g, s, "f32", "(1024,512) vs bit-by-bit SCL", max_excused=b.F // 100)
    else:
        k_g = int((g[0] != b.info).any(axis=1).sum())
        k_s = int((s[0] != b.info).any(axis=1).sum())
        lo_g, hi_g = _wilson(k_g, b.F)
        lo_s, hi_s = _wilson(k_s, b.F)
        _say(f"FER tree {k_g / b.F:.4f} [{lo_g:.4f}, {hi_g:.4f}], "
             f"SC-list {k_s / b.F:.4f} [{lo_s:.4f}, {hi_s:.4f}]")
        assert lo_g <= hi_s and lo_s <= hi_g


@pytest.mark.parametrize("dtype", ["f32", "i8"])
@pytest.mark.parametrize("ebn0", [3.5, 4.0, 4.5])
def test_2048_1723_crc32_L32(dtype, ebn0):
    code, b = batch(2048, 1723, 32, synth.CRC32_POLY, 4.0, 256, ebn0, (2, int(ebn0 * 4)), dtype)
    _say(f"(2048,1723) L=32 {dtype} {ebn0} dB")
    g = gpu_decode(code, 32, b.llr, dtype)
    o = oracle_decode(code, 32, b.llr, dtype)
    compare(g, o, dtype, f"(2048,1723) {dtype} {ebn0}")


@pytest.mark.parametrize("dtype", ["f32", "i16"])
@pytest.mark.parametrize("L", [2, 4, 8, 16, 32])
def test_1024_860_crc32_list_sizes(dtype, L):
    code, b = batch(1024, 860, 32, synth.CRC32_POLY, 4.0, 300, 4.0, (3, L), dtype)
    _say(f"(1024,860) L={L} {dtype}")
    g = gpu_decode(code, L, b.llr, dtype)
    o = oracle_decode(code, L, b.llr, dtype)
    compare(g, o, dtype, f"(1024,860) L={L}")


@pytest.mark.parametrize("N,K,r,L,dtype", [(4096, 3441, 32, 32, "i8"), (4096, 2048, 32, 8, "f32"),
                                           (256, 86, 8, 32, "i8"), (512, 430, 32, 2, "i16")])
def test_other_lengths(N, K, r, L, dtype):
    poly = synth.CRC8_POLY if r == 8 else synth.CRC32_POLY
    code, b = batch(N, K, r, poly, 2.5 if K <= N // 2 else 4.0, 64, 3.0, (4, N, L), dtype)
    _say(f"({N},{K}) L={L} {dtype}")
    g = gpu_decode(code, L, b.llr, dtype)
    o = oracle_decode(code, L, b.llr, dtype)
    compare(g, o, dtype, f"({N},{K}) L={L}")


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

def test_ragged_and_tiny_batches():
    import paper_1505_01466_amd as pk

    code, b = batch(1024, 512, 8, synth.CRC8_POLY, 2.5, 131, 2.0, 5, "i8")
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, 4, "i8")
    for F in (1, 2, 3, 7, 64, 131):
        _say(f"ragged F={F}")
        g = gpu_decode(code, 4, b.llr[:F], "i8", plan=plan)
        o = oracle_decode(code, 4, b.llr[:F], "i8")
        compare(g, o, "i8", f"F={F}")


def test_empty_batch_is_a_noop():
    import torch

    import paper_1505_01466_amd as pk

    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5)
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, 4, "f32")
    llr = torch.zeros((0, 256), dtype=torch.float32, device="cuda")
    u, ok, pm = plan.decode(llr)
    torch.cuda.synchronize()
    assert u.shape == (0, 128)


@pytest.mark.parametrize("dtype", ["f32", "i8"])
def test_degenerate_inputs(dtype):
    """All-zero LLRs (every decision a tie) and sign-flipped codewords (no
    path passes the CRC: the most reliable path is returned, crc_ok = 0)."""
    code, b = batch(1024, 512, 8, synth.CRC8_POLY, 2.5, 40, 3.0, 6, dtype)
    zeros = np.zeros_like(b.llr)
    flipped = (-b.llr.astype(np.int64)).astype(b.llr.dtype) if dtype != "f32" else -b.llr
    sat = np.where(b.llr >= 0, 127, -127).astype(b.llr.dtype) if dtype == "i8" else b.llr * 100
    for name, llr in (("zeros", zeros), ("flipped", flipped), ("saturated", sat)):
        for L in (1, 4, 32):
            _say(f"degenerate {name} L={L} {dtype}")
            g = gpu_decode(code, L, llr, dtype)
            o = oracle_decode(code, L, llr, dtype)
            compare(g, o, dtype, f"{name} L={L}")


@pytest.mark.parametrize("dtype", ["i8", "i16"])
def test_input_below_minus_q_reads_as_minus_q(dtype):
    """The integer domain is [-Q, Q]: an input of -Q - 1 (-128 / -32768) is
    saturated to -Q on load, by the kernel as by the oracle.  Frames with
    such values at every seventh position (channel F, G and leaves all read
    them), at the headline code and a code whose root is a Rate-1 leaf."""
    Q = 127 if dtype == "i8" else 32767
    for N, K, r, poly, d, L in ((2048, 1723, 32, synth.CRC32_POLY, 4.0, 32),
                                (256, 128, 8, synth.CRC8_POLY, 2.5, 8),
                                (64, 64, 8, synth.CRC8_POLY, 2.5, 4)):
        code, b = batch(N, K, r, poly, d, 24, 3.0, (11, N), dtype)
        llr = b.llr.copy()
        llr[:, ::7] = -Q - 1
        llr[::3, 1::5] = -Q - 1
        _say(f"({N},{K}) L={L} {dtype} with {-Q - 1} inputs")
        g = gpu_decode(code, L, llr, dtype)
        o = oracle_decode(code, L, llr, dtype)
        compare(g, o, dtype, f"({N},{K}) {dtype} -Q-1 inputs")
        o2 = oracle_decode(code, L, np.maximum(llr, -Q).astype(llr.dtype), dtype)
        compare(g, o2, dtype, f"({N},{K}) {dtype} as -Q")


def test_negative_zero_inputs():
    """float32 -0.0 decides 0 (eq. (sc:h) compares alpha < 0): all -0.0
    frames, and +/-2.0 frames with -0.0 sprinkled in, against the oracle,
    including codes whose root is one leaf."""
    rng = np.random.default_rng(12)
    cases = [(synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5), 4, 4)]
    for N, frozen in ((8, []), (4, [0]), (8, [0, 1, 2, 3, 4, 5, 6]), (32, list(range(16)))):
        fz = np.zeros(N, np.uint8)
        fz[frozen] = 1
        cases.append((synth.PolarCode(N=N, K=N - len(frozen), r=0, poly=0, design_ebn0_db=0.0,
                                      frozen=fz), 4, N))
    for code, L, spc_max in cases:
        llr = np.where(rng.random((40, code.N)) < 0.5, 2.0, -2.0).astype(np.float32)
        llr[rng.random((40, code.N)) < 0.3] = -0.0
        llr[:4] = -0.0
        for LL in (1, L):
            _say(f"-0.0 frames ({code.N},{code.K}) L={LL}")
            g = gpu_decode(code, LL, llr, "f32", spc_max=spc_max)
            o = oracle_decode(code, LL, llr, "f32", spc_max=spc_max)
            compare(g, o, "f32", f"-0.0 ({code.N},{code.K}) L={LL}", max_excused=0)


def test_deterministic():
    code, b = batch(2048, 1723, 32, synth.CRC32_POLY, 4.0, 128, 3.5, 7, "f32")
    g1 = gpu_decode(code, 32, b.llr, "f32")
    g2 = gpu_decode(code, 32, b.llr, "f32")
    for x, y in zip(g1, g2):
        assert x.tobytes() == y.tobytes()


def test_oneshot_entry_point():
    import torch

    import paper_1505_01466_amd as pk

    code, b = batch(1024, 512, 8, synth.CRC8_POLY, 2.5, 100, 2.5, 8, "i16")
    llr = torch.from_numpy(b.llr).cuda()
    u, ok = pk.decode(code.N, code.K, code.frozen, code.poly, code.r, 8, llr, "i16")
    torch.cuda.synchronize()
    o = oracle_decode(code, 8, b.llr, "i16")
    assert (u.cpu().numpy() == o[0]).all() and (ok.cpu().numpy() == o[1]).all()


def test_oneshot_calls_overlapping_on_streams():
    """The one-call entry point caches one group per code; calls for the same
    code issued on several streams without synchronising in between each get
    their own workspace and counter, so each equals its own solo decode."""
    import torch

    import paper_1505_01466_amd as pk

    code, _ = batch(1024, 512, 8, synth.CRC8_POLY, 2.5, 4, 2.5, 81, "i8")
    inputs = []
    for i in range(4):
        _, b = batch(1024, 512, 8, synth.CRC8_POLY, 2.5, 300 + 37 * i, 2.5, (82, i), "i8")
        inputs.append((b.llr, torch.from_numpy(b.llr).cuda()))
    solo = []
    for _, llr in inputs:
        solo.append(pk.decode(code.N, code.K, code.frozen, code.poly, code.r, 8, llr, "i8"))
        torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(4)]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    outs = []
    for st, (_, llr) in zip(streams, inputs):
        with torch.cuda.stream(st):
            outs.append(pk.decode(code.N, code.K, code.frozen, code.poly, code.r, 8, llr, "i8"))
    for st in streams:
        torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    for i, (out, ref) in enumerate(zip(outs, solo)):
        _say(f"overlapping one-call decode {i}: {inputs[i][0].shape[0]} frames")
        for x, y in zip(out, ref):
            assert x.cpu().numpy().tobytes() == y.cpu().numpy().tobytes(), i
    o = oracle_decode(code, 8, inputs[0][0], "i8")
    assert (outs[0][0].cpu().numpy() == o[0]).all() and (outs[0][1].cpu().numpy() == o[1]).all()


def test_autotuned_launch_shape():
    import paper_1505_01466_amd as pk
    import torch

    code, b = batch(512, 256, 8, synth.CRC8_POLY, 2.5, 512, 2.5, (9, 1), "i8")
    llr = torch.from_numpy(b.llr).cuda()
    cfg, ms = pk.autotune(code.N, code.K, code.frozen, code.poly, code.r, 8, llr, "i8")
    _say(f"(512,256) L=8 i8 autotuned {cfg} {ms:.3f} ms")
    assert cfg["threads"] in (64, 128, 256) and 8192 <= cfg["lds_budget"] <= 49152 and ms > 0
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, 8, "i8", **cfg)
    assert plan.info()["threads"] == cfg["threads"]
    g = gpu_decode(code, 8, b.llr, "i8", plan=plan)
    compare(g, oracle_decode(code, 8, b.llr, "i8"), "i8", "autotuned plan")


# ---------------------------------------------------------------------------
# Layout knobs: stages below the root stored or recomputed (none, one level,
# two levels) and the size of forking leaves run fused (float32), each
# against the oracle.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "i16", "i8"])
@pytest.mark.parametrize("recompute", [1, 2, 3])
@pytest.mark.parametrize("nk", [(2048, 1723, 32, 4.0, 3.75), (1024, 512, 8, 2.5, 2.0),
                                (256, 128, 8, 2.5, 2.0)])
def test_recomputed_stages(dtype, recompute, nk):
    import paper_1505_01466_amd as pk

    N, K, r, d, e = nk
    poly = synth.CRC32_POLY if r == 32 else synth.CRC8_POLY
    code, b = batch(N, K, r, poly, d, 96, e, (61, N, recompute), dtype)
    for budget in (0, 8192):  # default; small enough that the top levels spill
        plan = pk.Plan(N, K, code.frozen, code.poly, r, 32, dtype, recompute=recompute,
                       lds_budget=budget)
        _say(f"({N},{K}) L=32 {dtype} recompute={recompute} budget={budget}: {plan.info()}")
        g = gpu_decode(code, 32, b.llr, dtype, plan=plan)
        compare(g, oracle_decode(code, 32, b.llr, dtype), dtype,
                f"recompute={recompute} budget={budget}")
        plan.close()


# F / G passes of one or two tree levels (unroll 1, 2) in every dtype, at the
# default LDS budget (chained passes on chip and across the LDS / workspace
# boundary) and at one small enough that they read and write the workspace
@pytest.mark.parametrize("dtype", ["f32", "i16", "i8"])
@pytest.mark.parametrize("unroll", [1, 2])
@pytest.mark.parametrize("nk", [(1024, 860), (2048, 1723)])
def test_unrolled_passes(dtype, unroll, nk):
    import paper_1505_01466_amd as pk

    N, K = nk
    code, b = batch(N, K, 32, synth.CRC32_POLY, 4.0, 96, 3.5, (63, N, unroll), dtype)
    ref = oracle_decode(code, 32, b.llr, dtype)
    for budget in (0, 8192):
        plan = pk.Plan(N, K, code.frozen, code.poly, 32, 32, dtype, unroll=unroll,
                       lds_budget=budget)
        _say(f"({N},{K}) L=32 {dtype} unroll={unroll} budget={budget}: {plan.info()}")
        g = gpu_decode(code, 32, b.llr, dtype, plan=plan)
        compare(g, ref, dtype, f"unroll={unroll} budget={budget}")
        plan.close()


@pytest.mark.parametrize("fuse", [-1, 1, 3, 4, 5])
@pytest.mark.parametrize("L", [2, 8, 32])
def test_fused_fork_sizes(fuse, L):
    import paper_1505_01466_amd as pk

    code, b = batch(1024, 860, 32, synth.CRC32_POLY, 4.0, 128, 3.5, (62, L, fuse + 1), "f32")
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, L, "f32", fuse_log2=fuse)
    _say(f"(1024,860) L={L} f32 fuse_log2={fuse}")
    g = gpu_decode(code, L, b.llr, "f32", plan=plan)
    compare(g, oracle_decode(code, L, b.llr, "f32"), "f32", f"fuse={fuse} L={L}")
    plan.close()
