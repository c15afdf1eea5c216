"""Decoding captured in a HIP graph: every replay, with the program's own
eager work and synchronisations between replays, returns what an eager call
returns on the same input (and that matches the oracle).  The frame counter
is cleared by a one-thread kernel, not a memset, so the captured graph holds
kernels only."""

import sys

import numpy as np
import pytest

import synth

from parity import batch, compare, oracle_decode

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


@pytest.mark.parametrize("dtype,L", [("i8", 32), ("f32", 32), ("i16", 128)])
def test_captured_decode_replays_like_eager(pk, dtype, L):
    import torch

    F = 384
    code, b1 = batch(2048, 1723, 32, synth.CRC32_POLY, 4.0, F, 3.5, (31, L), dtype)
    b2 = synth.make_batch(code, F, 3.75, (32, L), dtype)
    plan = pk.Plan(2048, 1723, code.frozen, code.poly, 32, L, dtype)
    _say(f"graph capture (2048,1723) L={L} {dtype}")
    refs = []
    for bb in (b1, b2):
        u, ok, pm = plan.decode(torch.from_numpy(bb.llr).cuda())
        torch.cuda.synchronize()
        refs.append((u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()))
        compare(refs[-1], oracle_decode(code, L, bb.llr, dtype), dtype, f"eager L={L}")

    llr = torch.from_numpy(b1.llr).cuda()
    u = torch.empty((F, code.K), dtype=torch.uint8, device="cuda")
    ok = torch.empty(F, dtype=torch.uint8, device="cuda")
    pm = torch.empty(F, dtype=torch.float32 if dtype == "f32" else torch.int32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.decode(llr, u, ok, pm)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.decode(llr, u, ok, pm)
    torch.cuda.synchronize()
    for rep in range(6):
        which = rep % 2
        src = (b1, b2)[which]
        llr.copy_(torch.from_numpy(src.llr))  # eager work between replays
        u.zero_()
        ok.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy())
        for a, r in zip(got, refs[which]):
            assert np.array_equal(a, r), f"replay {rep} differs from the eager call"
    del g
    plan.close()
