"""Mixed launches: frames of several codes of one dtype in one persistent
launch (pscl_group_decode / pscl_decode_mixed).  Every job must come out
identical to decoding it alone with its plan (same kernel code per frame),
and match the oracle to the parity bar."""

import sys

import pytest

import synth

from parity import compare, oracle_decode

pytestmark = pytest.mark.gpu

# (N, K, r, poly, design dB, L, Eb/N0 dB)
CODES = [
    (256, 128, 8, synth.CRC8_POLY, 2.5, 2, 2.5),
    (512, 256, 8, synth.CRC8_POLY, 2.5, 8, 2.5),
    (1024, 860, 32, synth.CRC32_POLY, 4.0, 32, 4.0),
    (2048, 1723, 32, synth.CRC32_POLY, 4.0, 8, 4.0),
    (4096, 2048, 32, synth.CRC32_POLY, 2.5, 2, 2.5),
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_01466_amd as pk

    return pk, torch


def _setup(pk, torch, dtype, frames, seed):
    codes, plans, work, host = [], [], [], []
    for i, (N, K, r, poly, d, L, e) in enumerate(CODES):
        code = synth.make_code(N, K, r, poly, d)
        codes.append((code, L))
        plans.append(pk.Plan(N, K, code.frozen, code.poly, r, L, dtype))
    for j, (pi, F) in enumerate(frames):
        code, L = codes[pi]
        b = synth.make_batch(code, F, CODES[pi][6], (seed, j), dtype)
        host.append(b.llr)
        work.append((pi, torch.from_numpy(b.llr).cuda()))
    return codes, plans, work, host


def _same(a, b):
    return all(bool((x == y).all()) for x, y in zip(a, b))


@pytest.mark.parametrize("dtype", ["i8", "i16", "f32"])
def test_group_equals_single_plan_decodes(env, dtype):
    pk, torch = env
    frames = [(0, 37), (3, 5), (1, 100), (2, 0), (4, 3), (2, 64), (0, 1), (3, 9)]
    codes, plans, work, host = _setup(pk, torch, dtype, frames, 31)
    g = pk.Group(plans, max_jobs=16)
    outs = g.decode(work)
    torch.cuda.synchronize()
    for j, ((pi, llr), out) in enumerate(zip(work, outs)):
        _say(f"job {j}: code {pi} F={llr.shape[0]} {dtype}")
        if llr.shape[0] == 0:
            continue
        alone = plans[pi].decode(llr)
        torch.cuda.synchronize()
        assert _same([o.cpu().numpy() for o in out], [a.cpu().numpy() for a in alone]), j
        code, L = codes[pi]
        ref = oracle_decode(code, L, host[j], dtype)
        compare(tuple(o.cpu().numpy() for o in out), ref, dtype, f"mixed job {j}")
    g.close()


def test_wide_group_with_short_lists(env):
    """A group holding a list above 32 paths runs the wide kernels, which
    have no fused forks: float32 plans of shorter lists (whose records let
    fused forks form their leaf values from the parent's stage) must give
    the same frames there as alone, and match the oracle."""
    pk, torch = env
    specs = [(1024, 860, 32, synth.CRC32_POLY, 4.0, 32, 3.5),
             (512, 256, 8, synth.CRC8_POLY, 2.5, 8, 2.0),
             (1024, 860, 32, synth.CRC32_POLY, 4.0, 64, 3.5)]
    plans, work, host, codes = [], [], [], []
    for i, (N, K, r, poly, d, L, e) in enumerate(specs):
        code = synth.make_code(N, K, r, poly, d)
        codes.append((code, L))
        plans.append(pk.Plan(N, K, code.frozen, code.poly, r, L, "f32"))
        b = synth.make_batch(code, 48, e, (71, i), "f32")
        host.append(b.llr)
        work.append((i, torch.from_numpy(b.llr).cuda()))
    g = pk.Group(plans, max_jobs=8)
    outs = g.decode(work)
    torch.cuda.synchronize()
    for j, ((pi, llr), out) in enumerate(zip(work, outs)):
        _say(f"wide group job {j}: L={codes[pi][1]}")
        alone = plans[pi].decode(llr)
        torch.cuda.synchronize()
        assert _same([o.cpu().numpy() for o in out], [a.cpu().numpy() for a in alone]), j
        code, L = codes[pi]
        compare(tuple(o.cpu().numpy() for o in out), oracle_decode(code, L, host[j], "f32"),
                "f32", f"wide group job {j}")
    g.close()


@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_autotuned_group_against_oracle(env, dtype):
    """pscl_autotune_group on a mixed batch, plans rebuilt with the tuned
    configuration, one launch: every job matches the oracle."""
    pk, torch = env
    frames = [(0, 40), (1, 33), (2, 20), (3, 12), (4, 6)]
    codes, plans, work, host = _setup(pk, torch, dtype, frames, 53)
    cfgs, threads, ms = pk.autotune_group(plans, work)
    _say(f"autotuned {dtype}: threads {threads}, cfg {cfgs[0]}, {ms:.3f} ms per call")
    assert threads in (64, 128, 256) and len(cfgs) == len(plans)
    tuned = [pk.Plan(c.N, c.K, c.frozen, c.poly, c.r, L, dtype, cfg=cfg)
             for (c, L), cfg in zip(codes, cfgs)]
    g = pk.Group(tuned, max_jobs=8, threads=threads)
    outs = g.decode(work)
    torch.cuda.synchronize()
    for j, ((pi, llr), out) in enumerate(zip(work, outs)):
        code, L = codes[pi]
        ref = oracle_decode(code, L, host[j], dtype)
        compare(tuple(o.cpu().numpy() for o in out), ref, dtype, f"autotuned job {j}")
    g.close()


def test_calls_in_flight_and_cached_entry_point(env):
    pk, torch = env
    frames = [(1, 20), (0, 50), (2, 8), (3, 4)]
    codes, plans, work, host = _setup(pk, torch, "i8", frames, 47)
    ref = [plans[pi].decode(llr) for pi, llr in work]
    torch.cuda.synchronize()
    g = pk.Group(plans, max_jobs=4)
    # more calls than job-table slots, without synchronising in between,
    # first on one stream, then spread over three
    results = [g.decode(work) for _ in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    for i in range(3):
        with torch.cuda.stream(streams[i]):
            results.append(g.decode(work))
    for st in streams:
        torch.cuda.current_stream().wait_stream(st)
    results.append(pk.decode_mixed(plans, work))
    results.append(pk.decode_mixed(plans, work[::-1]))
    torch.cuda.synchronize()
    for c, res in enumerate(results):
        order = work if c < 7 else work[::-1]
        expect = ref if c < 7 else ref[::-1]
        for (pi, llr), out, exp in zip(order, res, expect):
            assert _same([o.cpu().numpy() for o in out], [e.cpu().numpy() for e in exp]), (c, pi)
    g.close()
    # destroying a plan drops the cached group; a new list of plans still works
    plans[0].close()
    out = pk.decode_mixed(plans[1:], [(0, work[0][1])])
    torch.cuda.synchronize()
    assert _same([o.cpu().numpy() for o in out[0]], [e.cpu().numpy() for e in ref[0]])


def test_group_rejects_mixed_dtypes_and_too_many_jobs(env):
    pk, torch = env
    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5)
    a = pk.Plan(256, 128, code.frozen, code.poly, 8, 4, "i8")
    b = pk.Plan(256, 128, code.frozen, code.poly, 8, 4, "f32")
    with pytest.raises(pk.PsclError) as e:
        pk.Group([a, b])
    assert e.value.status == 2
    g = pk.Group([a], max_jobs=2)
    llr = torch.zeros((4, 256), dtype=torch.int8, device="cuda")
    with pytest.raises(pk.PsclError) as e:
        g.decode([(0, llr), (0, llr), (0, llr)])
    assert e.value.status == 1
    out = g.decode([(0, llr[:0]), (0, llr), (0, llr[:0])])  # empty jobs are skipped
    torch.cuda.synchronize()
    assert out[1][0].shape == (4, 128)
    g.close()
