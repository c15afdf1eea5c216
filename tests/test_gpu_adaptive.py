"""Adaptive decoding (Sec. VI): an L = 1 pass over every frame, then list
decoding of the frames whose CRC fails, all on the device.  The expected
result composes the oracle the same way: decoder A with L = 1, then decoder
A with L on exactly the frames whose CRC failed."""

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


def _oracle_adaptive(code, L, llr, dtype):
    u, ok, pm, nt = oracle_decode(code, 1, llr, dtype)
    fail = np.flatnonzero(ok == 0)
    u, ok, pm, nt = u.copy(), ok.copy(), pm.copy(), nt.copy()
    if fail.size:
        u2, ok2, pm2, nt2 = oracle_decode(code, L, np.ascontiguousarray(llr[fail]), dtype)
        u[fail], ok[fail], pm[fail], nt[fail] = u2, ok2, pm2, nt2
    return (u, ok, pm, nt), fail.size


@pytest.mark.parametrize("dtype", ["i8", "i16", "f32"])
@pytest.mark.parametrize("case", [(256, 128, 8, synth.CRC8_POLY, 2.0, 8, 400, 1.5),
                                  (2048, 1723, 32, synth.CRC32_POLY, 4.0, 32, 300, 3.5),
                                  (1024, 512, 8, synth.CRC8_POLY, 2.5, 4, 257, 2.0),
                                  (1024, 892, 32, synth.CRC32_POLY, 4.0, 128, 160, 3.5)])
def test_adaptive_matches_oracle_composition(pk, dtype, case):
    import torch

    N, K, r, poly, d, L, F, e = case
    code, b = batch(N, K, r, poly, d, F, e, (21, N), dtype)
    fast = pk.Plan(N, K, code.frozen, code.poly, r, 1, dtype)
    lst = pk.Plan(N, K, code.frozen, code.poly, r, L, dtype)
    ad = pk.Adaptive(fast, lst, max_frames=F)
    u, ok, pm, n_list = ad.decode(torch.from_numpy(b.llr).cuda())
    torch.cuda.synchronize()
    ref, n_fail = _oracle_adaptive(code, L, b.llr, dtype)
    _say(f"({N},{K}) L={L} {dtype}: {n_fail}/{F} frames list-decoded")
    assert 0 < n_fail < F
    assert int(n_list.item()) == n_fail
    compare((u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()), ref, dtype,
            f"adaptive ({N},{K}) L={L}")
    # a second call with fewer frames reuses the scratch
    u2, ok2, pm2, n2 = ad.decode(torch.from_numpy(np.ascontiguousarray(b.llr[:F // 3])).cuda())
    torch.cuda.synchronize()
    ref2, n_fail2 = _oracle_adaptive(code, L, np.ascontiguousarray(b.llr[:F // 3]), dtype)
    assert int(n2.item()) == n_fail2
    compare((u2.cpu().numpy(), ok2.cpu().numpy(), pm2.cpu().numpy()), ref2, dtype,
            f"adaptive ({N},{K}) second call")
    ad.close()


def test_adaptive_rejects_mismatched_plans(pk):
    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.0)
    other = synth.make_code(256, 128, 8, synth.CRC8_POLY, 3.0)
    fast = pk.Plan(256, 128, code.frozen, code.poly, 8, 1, "i8")
    with pytest.raises(pk.PsclError):  # other dtype
        pk.Adaptive(fast, pk.Plan(256, 128, code.frozen, code.poly, 8, 8, "f32"), 16)
    with pytest.raises(pk.PsclError):  # the first pass must be L = 1
        pk.Adaptive(pk.Plan(256, 128, code.frozen, code.poly, 8, 2, "i8"),
                    pk.Plan(256, 128, code.frozen, code.poly, 8, 8, "i8"), 16)
    if not np.array_equal(code.frozen, other.frozen):  # other frozen set
        with pytest.raises(pk.PsclError):
            pk.Adaptive(fast, pk.Plan(256, 128, other.frozen, other.poly, 8, 8, "i8"), 16)
