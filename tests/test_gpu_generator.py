"""The device frame generator: the same frames, value by value, as the host
definition in synth.philox (itself pinned to Philox's published vectors and
to the channel's statistics), and frames the decoder recovers."""

import sys

import numpy as np
import pytest

import synth
from synth.philox import channel_params, philox_batch

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


CODES = [(2048, 1723, 32, synth.CRC32_POLY, 4.0, 300, 4.0),
         (1024, 512, 8, synth.CRC8_POLY, 2.5, 257, 2.0),
         (256, 128, 0, 0, 2.0, 129, 1.0),
         (64, 40, 8, synth.CRC8_POLY, 3.0, 65, 6.0),
         (4096, 3441, 32, synth.CRC32_POLY, 4.0, 33, 3.0),
         (16, 8, 4, 0x3, 2.0, 50, 4.0),
         (2, 1, 0, 0, 2.0, 20, 3.0)]


def _check_llr(dev, host, dtype, scale):
    if dtype == "f32":
        d = np.abs(dev.astype(np.float64) - host.astype(np.float64))
        tol = 2e-6 * (float(scale) + np.abs(host.astype(np.float64)))
        assert (d <= tol).all(), float((d / tol).max())
    else:
        d = np.abs(dev.astype(np.int64) - host.astype(np.int64))
        assert d.max() <= 1
        assert int((d != 0).sum()) <= max(2, dev.size // 10000)


@pytest.mark.parametrize("dtype", ["f32", "i16", "i8"])
@pytest.mark.parametrize("case", CODES)
def test_device_frames_match_host_definition(pk, dtype, case):
    import torch

    N, K, r, poly, d, F, e = case
    seed = 0x5EED_0000_0000 + N
    first = 7 if N != 64 else (1 << 32) - 20  # crosses the 32-bit frame-index boundary
    _say(f"generator ({N},{K}) r={r} {dtype} F={F} first={first}")
    code = synth.make_code(N, K, r, poly, d)
    g = pk.Generator(N, K, code.frozen, poly, r, dtype)
    llr, info = g.generate(F, e, seed, first_frame=first)
    torch.cuda.synchronize()
    host = philox_batch(code, F, e, seed, first=first, dtype=dtype)
    assert (info.cpu().numpy() == host.info).all()
    _check_llr(llr.cpu().numpy(), host.llr, dtype, channel_params(code, e)[1])
    g.close()


def test_chunked_calls_give_the_same_frames(pk):
    import torch

    code = synth.make_code(1024, 512, 8, synth.CRC8_POLY, 2.5)
    g = pk.Generator(1024, 512, code.frozen, code.poly, 8, "f32")
    whole, wi = g.generate(5000, 2.0, 11)
    a, ai = g.generate(1234, 2.0, 11)
    b, bi = g.generate(5000 - 1234, 2.0, 11, first_frame=1234)
    none, _ = g.generate(0, 2.0, 11)
    noinfo, ni = g.generate(100, 2.0, 11, first_frame=4900, want_info=False)
    torch.cuda.synchronize()
    assert ni is None and none.shape == (0, 1024)
    assert torch.equal(whole, torch.cat([a, b])) and torch.equal(wi, torch.cat([ai, bi]))
    assert torch.equal(noinfo, whole[4900:])
    g.close()


@pytest.mark.parametrize("dtype", ["f32", "i8"])
def test_decoder_recovers_generated_frames(pk, dtype):
    """Headline code at a high Eb/N0: every generated frame decodes to the
    generated information bits and passes its CRC."""
    import torch

    code = synth.make_code(2048, 1723, 32, synth.CRC32_POLY, 4.0)
    g = pk.Generator(2048, 1723, code.frozen, code.poly, 32, dtype)
    plan = pk.Plan(2048, 1723, code.frozen, code.poly, 32, 32, dtype)
    llr, info = g.generate(4096, 5.5, 2024)
    u, ok, pm = plan.decode(llr)
    torch.cuda.synchronize()
    assert bool(ok.all())
    assert torch.equal(u, info)
    g.close()


def test_resumable_fer_sweep(tmp_path):
    """bench's FER sweep with a JSONL log: an interrupted sweep (the log
    truncated to its first chunks) resumes, decodes only the missing chunks
    and reaches the same frame-error counts as an uninterrupted one."""
    import json
    import os
    import sys

    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    import paper_1505_01466_amd as pk

    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5)
    path = str(tmp_path / "sweep.jsonl")
    kw = dict(points=(1.5, 2.0), dtypes=("i8",), chunk=4096)
    full = bench.fer_sweep_leg(pk, torch, code, 20000, jsonl=path, **kw)
    lines = open(path).read().splitlines()
    assert len(lines) == 2 * 5  # 5 chunks per point
    with open(path, "w") as fh:
        fh.write("\n".join(lines[:3]) + "\n")
    again = bench.fer_sweep_leg(pk, torch, code, 20000, jsonl=path, **kw)
    assert len(open(path).read().splitlines()) == 10
    for e in ("1.5", "2.0"):
        assert again["i8"]["points"][e]["errors"] == full["i8"]["points"][e]["errors"]
        assert again["i8"]["points"][e]["frames"] == 20000
    assert full["i8"]["points"]["1.5"]["errors"] > 0
    # every recorded chunk once
    keys = [(r["ebn0_db"], r["first_frame"]) for r in map(json.loads, open(path))]
    assert len(set(keys)) == 10
