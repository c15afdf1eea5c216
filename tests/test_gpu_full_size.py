"""The benchmark's workload at full size: 65,536 frames of the (2048,1723)
CRC-32 code at L = 32 and 4.0 dB (the same seeded batch), decoded in one
launch with the default launch shape.  Sampled frames (the first, the last
and 510 drawn at random) are compared with the oracle element by element;
on every frame, the CRC flag must agree with the CRC recomputed from the
decoded bits."""

import sys

import numpy as np
import pytest

import synth

from parity import compare, oracle_decode

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def workload():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    code = synth.make_code(2048, 1723, 32, synth.CRC32_POLY, 4.0)
    b = synth.make_batch(code, 65536, 4.0, (20481723, 400), "f32")
    return code, b


@pytest.mark.parametrize("dtype", ["f32", "i8"])
def test_full_batch_sampled_against_oracle(workload, dtype):
    import torch

    import paper_1505_01466_amd as pk

    code, b = workload
    llr = synth.quantize(b.llr_f32, dtype)
    plan = pk.Plan(code.N, code.K, code.frozen, code.poly, code.r, 32, dtype)
    _say(f"(2048,1723) L=32 {dtype}: 65536 frames, launch {plan.info()}")
    u, ok, pm = plan.decode(torch.from_numpy(llr).cuda())
    torch.cuda.synchronize()
    u, ok, pm = u.cpu().numpy(), ok.cpu().numpy(), pm.cpu().numpy()
    rng = np.random.default_rng(65536)
    idx = np.unique(np.concatenate([[0, 65535], rng.choice(65536, 510, replace=False)]))
    ref = oracle_decode(code, 32, np.ascontiguousarray(llr[idx]), dtype)
    compare((u[idx], ok[idx], pm[idx]), ref, dtype, f"full batch {dtype}, sampled")
    # every frame: the flag says whether the decoded payload's CRC matches
    crc = synth.crc_remainder(u[:, :code.payload], code.poly, code.r)
    assert np.array_equal((crc == u[:, code.payload:]).all(axis=1), ok.astype(bool))
    fer = float((u != b.info).any(axis=1).mean())
    _say(f"{dtype}: FER {fer:.2e}, {int(ok.sum())} frames pass the CRC")
    assert fer < 1e-3
    plan.close()
