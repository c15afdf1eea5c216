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


# Known-answer vectors published with Philox4x32-10 (Salmon et al., SC 2011,
# distributed with their Random123 library): (counter, key) -> output.
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    from synth.philox import philox4x32_10

    for ctr, key, want in PHILOX_KAT:
        got = philox4x32_10(np.array([ctr], dtype=np.uint32), key)[0]
        assert tuple(int(v) for v in got) == want


def test_philox_frames_are_valid_codewords_and_independent_of_chunking():
    from synth.philox import philox_batch

    code = synth.make_code(1024, 512, 8, synth.CRC8_POLY, 2.5)
    b = philox_batch(code, 40, 2.0, seed=0x1234_5678_9ABC, first=3)
    assert (synth.crc_remainder(b.info[:, :code.payload], code.poly, code.r) == b.info[:, code.payload:]).all()
    u = np.zeros((b.F, code.N), np.uint8)
    u[:, code.info_pos] = b.info
    assert (synth.encode(u) == b.x).all()
    # frame f depends only on (seed, f)
    c = philox_batch(code, 10, 2.0, seed=0x1234_5678_9ABC, first=13)
    assert (c.info == b.info[10:20]).all() and (c.llr_f32 == b.llr_f32[10:20]).all()
    # frame index beyond 32 bits, other seed: different bits
    d = philox_batch(code, 10, 2.0, seed=0x1234_5678_9ABC, first=13 + (1 << 32))
    e = philox_batch(code, 10, 2.0, seed=0x1234_5678_9ABD, first=13)
    assert (d.info != c.info).any() and (e.info != c.info).any()
    # integer dtypes quantise the same float32 LLRs
    q = philox_batch(code, 40, 2.0, seed=0x1234_5678_9ABC, first=3, dtype="i8")
    assert (q.llr == synth.quantize(b.llr_f32, "i8")).all()


def test_philox_channel_statistics():
    """Payload bits fair and uncorrelated; the noise recovered from the LLRs
    is standard normal (mean, variance, tail mass, kurtosis)."""
    from synth.philox import channel_params, philox_batch

    code = synth.make_code(2048, 1723, 32, synth.CRC32_POLY, 4.0)
    b = philox_batch(code, 200, 3.0, seed=99)
    p = b.info[:, :code.payload].astype(np.float64)
    assert abs(p.mean() - 0.5) < 0.005
    assert abs(np.corrcoef(p[:, :-1].ravel(), p[:, 1:].ravel())[0, 1]) < 0.01
    sigma, scale = channel_params(code, 3.0)
    s = 1.0 - 2.0 * b.x.astype(np.float64)
    n = (b.llr_f32.astype(np.float64) / float(scale) - s) / float(sigma)
    assert abs(n.mean()) < 0.01 and abs(n.var() - 1.0) < 0.01
    assert abs(np.mean(np.abs(n) > 2.0) - 0.0455) < 0.002
    assert abs(np.mean(n ** 4) - 3.0) < 0.05
    # the four Box-Muller outputs of one block are uncorrelated
    blk = n.reshape(-1, 4)
    cc = np.corrcoef(blk.T)
    assert np.abs(cc - np.eye(4)).max() < 0.01
