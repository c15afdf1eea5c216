"""Serving: requests of mixed codes decoded as they arrive (pscl_server_*),
and the replay driver (pscl_replay) through a server and as plain
per-request launches.  Every request's result must equal decoding it alone
with its plan (int8: bit for bit)."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CODES = [
    (256, 128, 8, synth.CRC8_POLY, 2.5, 2),
    (512, 256, 8, synth.CRC8_POLY, 2.5, 8),
    (1024, 860, 32, synth.CRC32_POLY, 4.0, 32),
    (2048, 1723, 32, synth.CRC32_POLY, 4.0, 8),
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

    codes, plans = [], []
    for N, K, r, poly, d, L in CODES:
        code = synth.make_code(N, K, r, poly, d)
        codes.append(code)
        plans.append(pk.Plan(N, K, code.frozen, code.poly, r, L, "i8"))
    return pk, torch, codes, plans


def _requests(torch, codes, n, seed, fmax=64):
    rng = np.random.default_rng(seed)
    work = []
    for i in range(n):
        pi = int(rng.integers(len(codes)))
        F = int(rng.integers(1, fmax + 1))
        b = synth.make_batch(codes[pi], F, CODES[pi][4], (seed, i), "i8")
        work.append((pi, torch.from_numpy(b.llr).cuda()))
    return work


def _alone(torch, plans, work):
    out = [plans[pi].decode(llr) for pi, llr in work]
    torch.cuda.synchronize()
    return [[t.cpu().numpy() for t in o] for o in out]


def _check(got, ref):
    for i, (g, r) in enumerate(zip(got, ref)):
        for a, b in zip(g, r):
            assert (a.cpu().numpy() == b).all(), f"request {i}"


def test_server_results_equal_alone(env):
    pk, torch, codes, plans = env
    work = _requests(torch, codes, 60, 5)
    ref = _alone(torch, plans, work)
    sv = pk.Server(plans, streams=2)
    tickets = [sv.submit(pi, llr) for pi, llr in work]
    lats = [sv.wait(t) for t, _ in tickets]
    torch.cuda.synchronize()
    _check([o for _, o in tickets], ref)
    st = sv.stats()
    _say(f"server: {st}")
    assert st["requests"] == 60 and st["frames"] == sum(l.shape[0] for _, l in work)
    assert 1 <= st["launches"] <= 60 and min(lats) > 0 and st["p99_us"] >= st["p50_us"] > 0
    sv.close()


@pytest.mark.parametrize("through_server", [True, False])
def test_replay_poisson_arrivals(env, through_server):
    pk, torch, codes, plans = env
    n = 200
    work = _requests(torch, codes, n, 11)
    ref = _alone(torch, plans, work)
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(1e6 / 20000.0, n))  # 20k requests/s
    sv = pk.Server(plans, streams=3) if through_server else None
    if through_server:
        outs, lat, elapsed = pk.replay(plans, work, arrivals, server=sv)
    else:
        # per-request launches on 3 streams, a set of plans per stream
        sets = plans + [pk.Plan(c.N, c.K, c.frozen, c.poly, c.r, spec[5], "i8")
                        for _ in range(2) for c, spec in zip(codes, CODES)]
        outs, lat, elapsed = pk.replay(sets, work, arrivals, streams=3)
    torch.cuda.synchronize()
    _check(outs, ref)
    _say(f"replay server={through_server}: p50 {np.percentile(lat, 50):.0f} us, "
         f"p99 {np.percentile(lat, 99):.0f} us, elapsed {elapsed:.0f} us")
    assert (lat > 0).all() and elapsed >= arrivals[-1]
    if sv is not None:
        assert sv.stats()["requests"] == n
        sv.close()


def test_admission_control(env):
    pk, torch, codes, plans = env
    sv = pk.Server(plans, streams=1, max_requests=1, max_pending_frames=5000)
    big = synth.make_batch(codes[2], 4096, 4.0, (77, 1), "i8")
    big_llr = torch.from_numpy(big.llr).cuda()
    small = _requests(torch, codes, 1, 13)[0]
    t_big, out_big = sv.submit(2, big_llr)
    with pytest.raises(pk.PsclError) as e:
        sv.submit(*small)  # the server holds its one request
    assert e.value.status == 6
    sv.wait(t_big)
    t_small, out_small = sv.submit(*small)
    sv.wait(t_small)
    with pytest.raises(pk.PsclError) as e:  # larger than the queue admits, ever
        sv.submit(2, torch.zeros((5001, 1024), dtype=torch.int8, device="cuda"))
    assert e.value.status == 1
    torch.cuda.synchronize()
    _check([out_big, out_small], _alone(torch, plans, [(2, big_llr), small]))
    sv.close()


def test_server_with_large_lists(env):
    """A server over plans of L = 128, 64 and 8 (its launches run the
    wide-list kernel instance): every request equals decoding it alone."""
    pk, torch, _, _ = env
    specs = [(256, 128, 8, synth.CRC8_POLY, 2.5, 128, 1.5), (1024, 892, 32, synth.CRC32_POLY, 4.0, 64, 3.5),
             (512, 256, 8, synth.CRC8_POLY, 2.5, 8, 2.0)]
    codes, plans = [], []
    for N, K, r, poly, d, L, _ in specs:
        code = synth.make_code(N, K, r, poly, d)
        codes.append(code)
        plans.append(pk.Plan(N, K, code.frozen, poly, r, L, "i8"))
    rng = np.random.default_rng(77)
    work = []
    for i in range(24):
        pi = int(rng.integers(len(specs)))
        b = synth.make_batch(codes[pi], int(rng.integers(1, 33)), specs[pi][6], (77, i), "i8")
        work.append((pi, torch.from_numpy(b.llr).cuda()))
    ref = _alone(torch, plans, work)
    sv = pk.Server(plans, streams=2)
    tickets = [sv.submit(pi, llr) for pi, llr in work]
    for t, _ in tickets:
        sv.wait(t)
    torch.cuda.synchronize()
    _check([o for _, o in tickets], ref)
    _say(f"server with L up to 128: {sv.stats()}")
    sv.close()


@pytest.mark.parametrize("dtype", ["f32", "i16"])
def test_server_other_dtypes(env, dtype):
    """The server over float32 or int16 plans: every request equals decoding
    it alone (float32 bit for bit as well: the same kernel code per frame)."""
    pk, torch, _, _ = env
    specs = CODES[:3]
    codes, plans = [], []
    for N, K, r, poly, d, L in specs:
        code = synth.make_code(N, K, r, poly, d)
        codes.append(code)
        plans.append(pk.Plan(N, K, code.frozen, code.poly, r, L, dtype))
    rng = np.random.default_rng(91)
    work = []
    for i in range(20):
        pi = int(rng.integers(len(specs)))
        b = synth.make_batch(codes[pi], int(rng.integers(1, 40)), specs[pi][4], (91, i), dtype)
        work.append((pi, torch.from_numpy(b.llr).cuda()))
    ref = _alone(torch, plans, work)
    sv = pk.Server(plans, streams=2)
    tickets = [sv.submit(pi, llr) for pi, llr in work]
    for t, _ in tickets:
        sv.wait(t)
    torch.cuda.synchronize()
    _check([o for _, o in tickets], ref)
    _say(f"server {dtype}: {sv.stats()}")
    sv.close()


def test_submit_orders_after_the_producer(env):
    """Inputs still being written on the submitter's stream when submit() is
    called (a long chain of products first, then the device frame
    generator): the server decodes them only after that work."""
    pk, torch, codes, plans = env
    code = codes[3]
    gen = pk.Generator(code.N, code.K, code.frozen, code.poly, code.r, "i8")
    F = 512
    llr = torch.zeros((F, code.N), dtype=torch.int8, device="cuda")
    info = torch.zeros((F, code.K), dtype=torch.uint8, device="cuda")
    x = torch.randn(2048, 2048, device="cuda")
    sv = pk.Server(plans, streams=2)
    torch.cuda.synchronize()
    for _ in range(30):  # keeps the current stream busy for a while
        x = torch.tanh(x @ x) * 0.5
    gen.generate(F, 4.0, 99, llr=llr, info=info)
    t, out = sv.submit(3, llr)
    sv.wait(t)
    torch.cuda.synchronize()
    ref = _alone(torch, plans, [(3, llr)])
    _check([out], ref)
    assert int(llr.abs().sum().item()) > 0
    sv.close()
    gen.close()


def test_footprint_admission(env):
    """max_footprint_bytes: a request is charged F * pscl_plan_footprint
    bytes until it completes; a second request that would exceed the budget
    is refused (busy) until the first is done, and one that exceeds it alone
    is invalid."""
    pk, torch, codes, plans = env
    fp = plans[3].footprint()
    assert fp > code_bytes(codes[3])
    sv = pk.Server(plans, streams=1, max_footprint_bytes=int(1.5 * 64 * fp))
    a = synth.make_batch(codes[3], 64, 4.0, (55, 1), "i8")
    b = synth.make_batch(codes[3], 64, 4.0, (55, 2), "i8")
    la, lb = torch.from_numpy(a.llr).cuda(), torch.from_numpy(b.llr).cuda()
    torch.cuda.synchronize()
    ta, oa = sv.submit(3, la)
    with pytest.raises(pk.PsclError) as e:
        sv.submit(3, lb)
    assert e.value.status == 6
    sv.wait(ta)
    tb, ob = sv.submit(3, lb)
    sv.wait(tb)
    with pytest.raises(pk.PsclError) as e:  # 100 frames never fit
        sv.submit(3, torch.zeros((100, codes[3].N), dtype=torch.int8, device="cuda"))
    assert e.value.status == 1
    torch.cuda.synchronize()
    _check([oa, ob], _alone(torch, plans, [(3, la), (3, lb)]))
    sv.close()


def code_bytes(code):
    return code.N + code.K + 1 + 4


def test_wait_with_time_limit(env):
    """wait(timeout) returns 'timed out' while the request cannot have run
    (its inputs' stream is busy with a long chain of products), and the
    ticket stays valid for a later wait."""
    pk, torch, codes, plans = env
    b = synth.make_batch(codes[2], 256, 4.0, (56, 1), "i8")
    llr = torch.from_numpy(b.llr).cuda()
    x = torch.randn(4096, 4096, device="cuda")
    sv = pk.Server(plans, streams=1)
    torch.cuda.synchronize()
    for _ in range(40):
        x = torch.tanh(x @ x) * 0.5
    t, out = sv.submit(2, llr)
    with pytest.raises(pk.PsclError) as e:
        sv.wait(t, timeout_ms=1.0)
    assert e.value.status == 7
    lat = sv.wait(t, timeout_ms=60000.0)
    assert lat > 0
    torch.cuda.synchronize()
    _check([out], _alone(torch, plans, [(2, llr)]))
    sv.close()


@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_persistent_server_results_equal_alone(env, dtype):
    """Persistent mode: requests published into the ring and decoded by a
    persistent kernel, submitted in bursts with pauses longer than the
    kernel's idle time (so it ends and is relaunched): every request equals
    decoding it alone."""
    import time

    pk, torch, codes, plans = env
    if dtype != "i8":
        plans = [pk.Plan(c.N, c.K, c.frozen, c.poly, c.r, spec[5], dtype)
                 for c, spec in zip(codes, CODES)]
    rng = np.random.default_rng(101)
    work = []
    for i in range(90):
        pi = int(rng.integers(len(codes)))
        b = synth.make_batch(codes[pi], int(rng.integers(1, 65)), CODES[pi][4], (101, i), dtype)
        work.append((pi, torch.from_numpy(b.llr).cuda()))
    ref = _alone(torch, plans, work)
    sv = pk.Server(plans, persistent=True, idle_us=500)
    tickets = []
    for burst in range(3):
        for pi, llr in work[burst * 30:(burst + 1) * 30]:
            tickets.append(sv.submit(pi, llr))
        for t, _ in tickets[burst * 30:]:
            sv.wait(t, timeout_ms=60000.0)
        time.sleep(0.01)  # the kernel goes idle and ends
    torch.cuda.synchronize()
    _check([o for _, o in tickets], ref)
    st = sv.stats()
    _say(f"persistent server {dtype}: {st}")
    assert st["requests"] == 90 and st["launches"] >= 3
    sv.close()


def test_persistent_server_replay_and_producer_order(env):
    """Persistent mode through the replay driver (Poisson arrivals), and a
    request whose inputs are still being generated when it is submitted."""
    pk, torch, codes, plans = env
    n = 200
    work = _requests(torch, codes, n, 12)
    ref = _alone(torch, plans, work)
    rng = np.random.default_rng(4)
    arrivals = np.cumsum(rng.exponential(1e6 / 20000.0, n))
    sv = pk.Server(plans, persistent=True)
    outs, lat, elapsed = pk.replay(plans, work, arrivals, server=sv)
    torch.cuda.synchronize()
    _check(outs, ref)
    _say(f"persistent replay: p50 {np.percentile(lat, 50):.0f} us, "
         f"p99 {np.percentile(lat, 99):.0f} us, launches {sv.stats()['launches']}")
    code = codes[3]
    gen = pk.Generator(code.N, code.K, code.frozen, code.poly, code.r, "i8")
    llr = torch.zeros((256, code.N), dtype=torch.int8, device="cuda")
    x = torch.randn(2048, 2048, device="cuda")
    torch.cuda.synchronize()
    for _ in range(30):
        x = torch.tanh(x @ x) * 0.5
    gen.generate(256, 4.0, 98, llr=llr)
    t, out = sv.submit(3, llr)
    sv.wait(t, timeout_ms=60000.0)
    torch.cuda.synchronize()
    _check([out], _alone(torch, plans, [(3, llr)]))
    sv.close()
    gen.close()


@pytest.mark.parametrize("active", [1, 3])
def test_persistent_server_fixed_active_per_cu(env, active):
    """A fixed count of workgroups per CU taking frames (by default they are
    admitted by the frames outstanding on the device): every request equals
    decoding it alone."""
    pk, torch, codes, plans = env
    n = 120
    work = _requests(torch, codes, n, 13 + active)
    ref = _alone(torch, plans, work)
    rng = np.random.default_rng(5 + active)
    arrivals = np.cumsum(rng.exponential(1e6 / 50000.0, n))
    sv = pk.Server(plans, persistent=True, active_per_cu=active)
    outs, lat, elapsed = pk.replay(plans, work, arrivals, server=sv)
    torch.cuda.synchronize()
    _check(outs, ref)
    _say(f"persistent replay, {active} per CU: p50 {np.percentile(lat, 50):.0f} us, "
         f"p99 {np.percentile(lat, 99):.0f} us")
    sv.close()


def test_persistent_server_wraps_the_frame_records(env):
    """More frames through one persistent-mode server than its ring holds
    frame records (2^18), so every record position is reused, including
    the last: every request equals decoding it alone."""
    pk, torch, codes, plans = env
    code = codes[0]  # (256,128) L = 2: cheap frames
    b = synth.make_batch(code, 64, CODES[0][4], (202, 0), "i8")
    llr = torch.from_numpy(b.llr).cuda()
    ref = _alone(torch, plans, [(0, llr)])[0]
    sv = pk.Server(plans, persistent=True, max_requests=2048)
    n_req = (1 << 18) // 64 + 700  # 4,796 requests of 64 frames
    outs, live = [], []
    for i in range(n_req):
        while True:
            try:
                t, out = sv.submit(0, llr)
                break
            except pk.PsclError as e:
                assert e.status == 6
                sv.wait(live.pop(0)[0], timeout_ms=60000.0)
        live.append((t, out))
        outs.append(out)
    for t, _ in live:
        sv.wait(t, timeout_ms=60000.0)
    torch.cuda.synchronize()
    for i in range(0, n_req, 97):
        _check([outs[i]], [ref])
    _check([outs[-1]], [ref])
    st = sv.stats()
    _say(f"persistent server, {n_req * 64} frames: {st}")
    assert st["frames"] == n_req * 64
    sv.close()
