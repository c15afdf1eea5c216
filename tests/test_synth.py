"""The seeded workload generator (transmitter + channel)."""

import numpy as np

import synth


def test_encoder_closed_form():
    N = 32
    u = np.eye(N, dtype=np.uint8)
    x = synth.encode(u)
    for i in range(N):
        assert list(x[i]) == [int((j & i) == j) for j in range(N)]


def test_encoder_involution():
    rng = np.random.default_rng(0)
    u = rng.integers(0, 2, (7, 1024), dtype=np.uint8)
    assert (synth.encode(synth.encode(u)) == u).all()


def test_bhattacharyya_sizes_and_nesting():
    for N, K in ((1024, 512), (2048, 1723), (4096, 3441)):
        f = synth.bhattacharyya_frozen(N, K, 4.0)
        assert int((f == 0).sum()) == K
    # the last position (all upgrading steps) is the most reliable
    f = synth.bhattacharyya_frozen(1024, 1, 2.0)
    assert f[-1] == 0 and f[:-1].all()
    # each upgrading step only improves: sets are nested as K grows
    prev = None
    for K in (128, 256, 512, 768):
        info = set(np.flatnonzero(synth.bhattacharyya_frozen(1024, K, 2.0, rate=0.5) == 0))
        if prev is not None:
            assert prev <= info
        prev = info


def test_batch_is_deterministic_and_valid():
    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5)
    a = synth.make_batch(code, 50, 2.0, (1, 2, 3), "i8")
    b = synth.make_batch(code, 50, 2.0, (1, 2, 3), "i8")
    assert (a.llr == b.llr).all() and (a.info == b.info).all()
    c = synth.make_batch(code, 50, 2.0, (1, 2, 4), "i8")
    assert not (a.llr == c.llr).all()
    # CRC inside K: remainder over payload matches the CRC field
    crc = synth.crc_remainder(a.info[:, : code.payload], code.poly, code.r)
    assert (crc == a.info[:, code.payload:]).all()
    # transmitted words are codewords of the polar code
    u = synth.encode(a.x)
    assert not u[:, code.frozen == 1].any()


def test_quantisation():
    llr = np.array([0.125, 0.375, -0.125, 40.0, -40.0, 0.0, 1.0 / 128], np.float32)
    assert list(synth.quantize(llr, "i8")) == [0, 2, 0, 127, -127, 0, 0]
    assert list(synth.quantize(llr, "i16")) == [8, 24, -8, 2560, -2560, 0, 0]
    big = np.array([1e6, -1e6], np.float32)
    assert list(synth.quantize(big, "i16")) == [32767, -32767]


def test_awgn_statistics():
    code = synth.make_code(1024, 512, 8, synth.CRC8_POLY, 2.5)
    b = synth.make_batch(code, 200, 2.5, 5, "f32")
    sigma2 = 1.0 / (2 * code.rate * 10 ** 0.25)
    y = b.llr_f32.astype(np.float64) * sigma2 / 2
    s = 1 - 2 * b.x.astype(np.float64)
    noise = y - s
    assert abs(noise.mean()) < 0.01
    assert abs(noise.var() / sigma2 - 1) < 0.02
