"""pscl_decode_noalloc (the entry point for callers that cannot allocate
device memory) against pscl_decode on the same plan and frames, both called
through the C ABI: two calls in a row, the second on fewer frames, every
output byte and metric identical.  Plans cover workspaces that spill to the
static scratch (the (2048,1723) L = 32 workload in float32 and int8, an
L = 128 int16 plan) and a code whose state stays in LDS."""

import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CASES = [
    # (N, K, r, design dB, Eb/N0, L, dtype, frames first call, second call)
    (2048, 1723, 32, 4.0, 4.0, 32, "f32", 3000, 700),
    (2048, 1723, 32, 4.0, 3.5, 32, "i8", 6000, 1111),
    (1024, 892, 32, 4.0, 3.0, 128, "i16", 1500, 333),
    (64, 40, 8, 2.0, 2.0, 8, "i8", 2000, 17),
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}_L{c[5]}_{c[6]}")
def test_noalloc_matches_decode(case):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_01466_amd as pk

    N, K, r, design, ebn0, L, dtype, F1, F2 = case
    poly = synth.CRC32_POLY if r == 32 else synth.CRC8_POLY
    code = synth.make_code(N, K, r, poly, design)
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, L, dtype)
    _say(f"noalloc N={N} K={K} L={L} {dtype} F={F1},{F2}: launch {plan.info()}")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pm_dt = torch.float32 if dtype == "f32" else torch.int32
    lib = pk.lib
    for call, F in enumerate((F1, F2)):
        b = synth.make_batch(code, F, ebn0, (777, N, L, call), dtype)
        llr = torch.from_numpy(b.llr).cuda()
        outs = []
        for fn in (lib.pscl_decode, lib.pscl_decode_noalloc):
            u = torch.full((F, K), 0xAB, dtype=torch.uint8, device="cuda")
            ok = torch.full((F,), 0xAB, dtype=torch.uint8, device="cuda")
            pm = torch.full((F,), -7, dtype=pm_dt, device="cuda")
            st = fn(plan._h, _ptr(llr), F, _ptr(u), _ptr(ok), _ptr(pm), stream)
            assert st == 0, f"{fn.__name__}: status {st}"
            torch.cuda.synchronize()
            outs.append((u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()))
        (u0, ok0, pm0), (u1, ok1, pm1) = outs
        assert np.array_equal(u0, u1), f"call {call}: u_hat differs"
        assert np.array_equal(ok0, ok1), f"call {call}: crc_ok differs"
        assert np.array_equal(pm0.view(np.uint32), pm1.view(np.uint32)), f"call {call}: pm differs"
        assert set(np.unique(u1)) <= {0, 1}
        fer = float((u1 != b.info).any(axis=1).mean())
        _say(f"  call {call}: {F} frames identical, FER {fer:.3g}")
    plan.close()


def test_noalloc_argument_errors():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_01466_amd as pk

    code = synth.make_code(64, 40, 8, synth.CRC8_POLY, 2.0)
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, 4, "i8")
    llr = torch.zeros((4, 64), dtype=torch.int8, device="cuda")
    u = torch.empty((4, code.K), dtype=torch.uint8, device="cuda")
    lib = pk.lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    none = ctypes.c_void_p(None)
    assert lib.pscl_decode_noalloc(none, _ptr(llr), 4, _ptr(u), none, none, stream) == 1
    assert lib.pscl_decode_noalloc(plan._h, _ptr(llr), -1, _ptr(u), none, none, stream) == 1
    assert lib.pscl_decode_noalloc(plan._h, none, 4, _ptr(u), none, none, stream) == 1
    assert lib.pscl_decode_noalloc(plan._h, ctypes.c_void_p(llr.data_ptr() + 1), 4, _ptr(u),
                                   none, none, stream) == 1
    assert lib.pscl_decode_noalloc(plan._h, _ptr(llr), 0, _ptr(u), none, none, stream) == 0
    # crc_ok / pm may be NULL
    assert lib.pscl_decode_noalloc(plan._h, _ptr(llr), 4, _ptr(u), none, none, stream) == 0
    torch.cuda.synchronize()
    assert set(np.unique(u.cpu().numpy())) <= {0, 1}
    plan.close()
