"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: each test checks a closed form,
a worked example from the paper, a brute-force enumeration, an exact identity
or a textbook special case.
"""

import itertools
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = v
    return out


def _dist(x, llr):
    """Codeword distance sum_i |llr_i| [x_i != h(llr_i)] in exact double."""
    a = np.asarray(llr, dtype=np.float64)
    return float(np.sum(np.abs(a) * (x != (a < 0))))


def _tree_classes(frozen, spc_max=4):
    """Leaf node classes of the decoding tree (Sec. II-C/II-D), for choosing
    test codes.  Returns a list of (class, size)."""
    out = []

    def rec(f):
        nv = len(f)
        nf = int(np.sum(f))
        if nv == 1:
            out.append(("R0" if nf else "R1", 1))
        elif nf == nv:
            out.append(("R0", nv))
        elif nf == 0:
            out.append(("R1", nv))
        elif nf == nv - 1 and not f[-1]:
            out.append(("REP", nv))
        elif nf == 1 and f[0] and 4 <= nv <= spc_max:
            out.append(("SPC", nv))
        else:
            rec(f[: nv // 2])
            rec(f[nv // 2:])

    rec(np.asarray(frozen))
    return out


# --------------------------------------------------------------------------
# CRC
# --------------------------------------------------------------------------

def test_crc_catalogue_check_values(orc):
    g = _golden("crc_check_values.txt")
    msg = np.unpackbits(np.frombuffer(b"123456789", dtype=np.uint8))
    for key in ("crc8", "crc32"):
        poly, r, check = int(g[key][0], 16), int(g[key][1]), int(g[key][2], 16)
        assert orc.crc(msg, poly, r) == check


def test_crc_codeword_has_zero_remainder(orc):
    rng = np.random.default_rng(5)
    for poly, r in ((0x07, 8), (0x04C11DB7, 32), (0x3, 2)):
        for n in (1, 7, 100, 1691):
            m = rng.integers(0, 2, n, dtype=np.uint8)
            rem = orc.crc(m, poly, r)
            tail = np.array([(rem >> (r - 1 - t)) & 1 for t in range(r)], np.uint8)
            assert orc.crc(np.concatenate([m, tail]), poly, r) == 0


def test_crc_matches_independent_linear_map(orc):
    """The generator's CRC (a GF(2) matrix) and the oracle's bit-serial
    register are written independently and must agree."""
    rng = np.random.default_rng(6)
    for poly, r in ((0x07, 8), (0x04C11DB7, 32)):
        bits = rng.integers(0, 2, (20, 333), dtype=np.uint8)
        lin = synth.crc_remainder(bits, poly, r)
        for row, ref in zip(bits, lin):
            v = orc.crc(row, poly, r)
            assert [(v >> (r - 1 - t)) & 1 for t in range(r)] == list(ref)


# --------------------------------------------------------------------------
# Polar transform and code construction
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2, 8, 64])
def test_transform_closed_form(orc, N):
    """Row i of F^{(x)n} (F = [[1,0],[1,1]]) has a 1 in column j exactly when
    j is a sub-mask of i."""
    for i in range(N):
        e = np.zeros(N, np.uint8)
        e[i] = 1
        x = orc.polar_transform(e)
        ref = np.array([(j & i) == j for j in range(N)], np.uint8)
        assert (x == ref).all()


def test_transform_is_involution_and_matches_encoder(orc):
    rng = np.random.default_rng(1)
    u = rng.integers(0, 2, (5, 256), dtype=np.uint8)
    x = synth.encode(u)
    for row_u, row_x in zip(u, x):
        assert (orc.polar_transform(row_u) == row_x).all()
        assert (orc.polar_transform(row_x) == row_u).all()


def test_fig1_frozen_set():
    g = _golden("fig1_code_8_4.txt")
    want = [int(v) for v in g["frozen"]]
    for design in (0.0, 1.0, 2.0, 3.0, 4.0):
        f = synth.bhattacharyya_frozen(8, 4, design, rate=0.5)
        assert list(np.flatnonzero(f)) == want


def test_fig2_tree_classes():
    g = _golden("fig1_code_8_4.txt")
    frozen = np.zeros(8, np.uint8)
    frozen[[int(v) for v in g["frozen"]]] = 1
    assert _tree_classes(frozen) == [("REP", 4), ("SPC", 4)]


# --------------------------------------------------------------------------
# Selection rule (Alg. 1)
# --------------------------------------------------------------------------

def test_select_matches_sort(orc):
    rng = np.random.default_rng(2)
    for _ in range(300):
        n = int(rng.integers(1, 80))
        L = int(rng.integers(1, 40))
        pm = rng.integers(-6, 1, n).astype(np.float64)  # many exact ties
        keep = orc.select(pm, L)
        if n <= L:
            assert list(keep) == list(range(n))
        else:
            assert list(keep) == sorted(range(n), key=lambda e: (-pm[e], e))[:L]


# --------------------------------------------------------------------------
# Round trip on noiseless input
# --------------------------------------------------------------------------

CODES = [
    (1024, 512, 8, synth.CRC8_POLY, 2.5),
    (2048, 1723, 32, synth.CRC32_POLY, 4.0),
    (1024, 860, 32, synth.CRC32_POLY, 4.0),
    (256, 128, 8, synth.CRC8_POLY, 2.5),
]


@pytest.mark.parametrize("dtype", ["f32", "i16", "i8"])
@pytest.mark.parametrize("ci", range(len(CODES)))
def test_noiseless_round_trip(orc, ci, dtype):
    N, K, r, poly, d = CODES[ci]
    code = synth.make_code(N, K, r, poly, d)
    b = synth.make_batch(code, 6, None, (7, ci), dtype)
    for L, mode in ((1, 0), (4, 0), (32, 0), (4, 1)):
        u, ok, pm, _ = orc.decode_tree(N, K, code.frozen, poly, r, L, b.llr, dtype, mode=mode)
        assert (u == b.info).all() and ok.all() and (pm == 0).all()
    u, ok, pm, _ = orc.decode_scl(N, K, code.frozen, poly, r, 4, b.llr, dtype)
    assert (u == b.info).all() and ok.all() and (pm == 0).all()


# --------------------------------------------------------------------------
# Maximum likelihood: exhaustive lists reproduce brute force
# --------------------------------------------------------------------------

def _small_codes(spc_max=4):
    """Small codes whose tree nodes all enumerate every codeword of their
    constituent code (Rate-0, repetition, SPC-4, Rate-1 of size <= 2)."""
    rng = np.random.default_rng(11)
    found = []
    for N in (8, 16):
        tries = 0
        while len([c for c in found if c[0] == N]) < 4 and tries < 5000:
            tries += 1
            K = int(rng.integers(2, 6))
            frozen = np.ones(N, np.uint8)
            frozen[rng.choice(N, K, replace=False)] = 0
            cls = _tree_classes(frozen, spc_max)
            if all(c in ("R0", "REP", "SPC") or (c == "R1" and s <= 2) for c, s in cls):
                found.append((N, K, frozen))
    g = _golden("fig1_code_8_4.txt")
    f84 = np.zeros(8, np.uint8)
    f84[[int(v) for v in g["frozen"]]] = 1
    found.append((8, 4, f84))
    return found


@pytest.mark.parametrize("dtype", ["i16", "f32"])
def test_exhaustive_list_equals_ml(orc, dtype):
    """With L >= 2^K nothing is pruned, so the CRC-aided pick is the ML
    codeword among CRC-valid words, and its metric is minus its distance
    (the min-sum path-metric identity)."""
    rng = np.random.default_rng(3)
    for N, K, frozen in _small_codes():
        for r, poly in ((0, 0), (1, 0x1), (2, 0x3)):
            if K - r < 1:
                continue
            L = 1 << K
            if dtype == "i16":
                llr = rng.integers(-9, 10, (40, N)).astype(np.int16)
            else:
                llr = rng.normal(1.0, 2.0, (40, N)).astype(np.float32)
            u_ml, d_ml = orc.decode_ml(N, K, frozen, poly, r, llr, dtype)
            for dec in ("tree", "scl"):
                if dec == "tree":
                    u, ok, pm, _ = orc.decode_tree(N, K, frozen, poly, r, L, llr, dtype)
                else:
                    u, ok, pm, _ = orc.decode_scl(N, K, frozen, poly, r, L, llr, dtype)
                assert ok.all()
                if dtype == "i16":
                    assert (-pm == d_ml).all()
                else:
                    assert np.allclose(-pm, d_ml, rtol=1e-5, atol=1e-5)
                # the decoded word is a minimiser
                pos = np.flatnonzero(frozen == 0)
                for f in range(llr.shape[0]):
                    uu = np.zeros(N, np.uint8)
                    uu[pos] = u[f]
                    x = orc.polar_transform(uu)
                    assert _dist(x, llr[f]) == pytest.approx(d_ml[f], rel=1e-6, abs=1e-6)


def test_min_sum_identity_every_path(orc):
    """Every complete path of an unpruned SC list carries PM = -D(x)."""
    rng = np.random.default_rng(4)
    for N, K, frozen in _small_codes():
        L = 1 << K
        for _ in range(10):
            llr = rng.integers(-7, 8, N).astype(np.int8)
            for mode in (1, 0):
                cw, pm = orc.decode_tree_list(N, K, frozen, L, llr, "i8", mode=mode)
                assert len(cw) == L
                assert len({bytes(c) for c in cw}) == L
                for c, p in zip(cw, pm):
                    assert -p == _dist(c, llr)


# --------------------------------------------------------------------------
# Node decoders: candidate sets by brute force
# --------------------------------------------------------------------------

def _lrb(a, m):
    return list(np.argsort(np.abs(a), kind="stable")[:m])


def _words(nv):
    return [np.array(w, np.uint8) for w in itertools.product((0, 1), repeat=nv)]


@pytest.mark.parametrize("nv", [2, 4, 8])
def test_rate1_candidates(orc, nv):
    """Rate-1 (Sec. III-C): the candidates are exactly the words that differ
    from the hard decision only within the two least reliable positions, each
    with metric -D; the first is the ML word."""
    rng = np.random.default_rng(nv)
    frozen = np.zeros(nv, np.uint8)
    for _ in range(50):
        a = rng.normal(0, 2, nv).astype(np.float32)
        cw, pm = orc.decode_tree_list(nv, nv, frozen, 4, a, "f32")
        hd = (a < 0).astype(np.uint8)
        m = _lrb(a, 2)
        want = {bytes(w) for w in _words(nv)
                if all(w[i] == hd[i] for i in range(nv) if i not in m)}
        assert {bytes(c) for c in cw} == want
        for c, p in zip(cw, pm):
            assert -p == pytest.approx(_dist(c, a), rel=1e-6)
        assert (cw[0] == hd).all()


@pytest.mark.parametrize("nv", [4, 8])
def test_spc_candidates(orc, nv):
    """SPC (Sec. III-D): with L >= 8 the candidates are exactly the
    even-parity words that differ from the hard decision only within the four
    least reliable positions; with L = 2 they are the two best even-parity
    words overall."""
    rng = np.random.default_rng(10 + nv)
    frozen = np.zeros(nv, np.uint8)
    frozen[0] = 1
    even = [w for w in _words(nv) if w.sum() % 2 == 0]
    for _ in range(50):
        a = rng.normal(0.5, 2, nv).astype(np.float32)
        hd = (a < 0).astype(np.uint8)
        m = _lrb(a, 4)
        cw, pm = orc.decode_tree_list(nv, nv - 1, frozen, 8, a, "f32", spc_max=nv)
        want = {bytes(w) for w in even if all(w[i] == hd[i] for i in range(nv) if i not in m)}
        assert {bytes(c) for c in cw} == want
        for c, p in zip(cw, pm):
            assert -p == pytest.approx(_dist(c, a), rel=1e-6)
        best2 = sorted(even, key=lambda w: _dist(w, a))[:2]
        cw2, _ = orc.decode_tree_list(nv, nv - 1, frozen, 2, a, "f32", spc_max=nv)
        assert [bytes(c) for c in cw2] == [bytes(w) for w in best2]


@pytest.mark.parametrize("nv", [2, 4, 16])
def test_repetition_candidates(orc, nv):
    """Repetition (Sec. III-E): all-zero and all-one words, ML first; the ML
    word is all-zero exactly when sum(alpha) >= 0 (eq. (rep))."""
    rng = np.random.default_rng(20 + nv)
    frozen = np.ones(nv, np.uint8)
    frozen[-1] = 0
    for _ in range(50):
        a = rng.integers(-20, 21, nv).astype(np.int16)
        cw, pm = orc.decode_tree_list(nv, 1, frozen, 4, a, "i16")
        assert len(cw) == 2
        first = 0 if a.astype(np.int64).sum() >= 0 else 1
        assert (cw[0] == first).all() and (cw[1] == 1 - first).all()
        for c, p in zip(cw, pm):
            assert -p == _dist(c, a)


def test_rate0_metric_is_distance_to_zero_word(orc):
    """Rate-0 (Sec. III-B, eq. (rel:frozen-h)): no fork, metric minus the
    distance of the all-zero word.  A code made of a Rate-0 left half and a
    Rate-1 right half exposes it: every final path has metric -D(x)."""
    rng = np.random.default_rng(30)
    for nv in (2, 8, 32):
        N = 2 * nv
        frozen = np.zeros(N, np.uint8)
        frozen[:nv] = 1
        assert _tree_classes(frozen) == [("R0", nv), ("R1", nv)]
        for _ in range(20):
            a = rng.integers(-9, 10, N).astype(np.int16)
            cw, pm = orc.decode_tree_list(N, nv, frozen, 4, a, "i16", mode=0)
            assert len(cw) == 4
            for c, p in zip(cw, pm):
                assert -p == _dist(c, a)


# --------------------------------------------------------------------------
# Special cases and equivalences
# --------------------------------------------------------------------------

def _fast_ssc(a, frozen, Q=32767, stats=None):
    """Textbook single-path Fast-SSC (Sec. II-C) on integer LLRs saturated to
    [-Q, Q]: Rate-0 -> zeros, Rate-1 -> hard decision (eq. (info)),
    repetition -> sign of the sum (eq. (rep)), SPC -> hard decision with the
    least reliable bit fixing the parity (eq. (spc)).  Returns (x, pm): the
    codeword and its path metric, minus the summed leaf penalties
    |alpha_i| [x_i != h(alpha_i)] of eq. (pm).  Q=None: no saturation.
    stats["sat"] counts G results that had to be saturated."""
    a = np.asarray(a, dtype=np.int64)
    nv = len(a)
    nf = int(frozen.sum())

    def pen(x):
        return -int(np.sum(np.abs(a) * (x != (a < 0))))

    if nv == 1:
        x = np.array([0 if nf else int(a[0] < 0)], np.uint8)
        return x, pen(x)
    if nf == nv:
        x = np.zeros(nv, np.uint8)
        return x, pen(x)
    if nf == 0:
        return (a < 0).astype(np.uint8), 0
    if nf == nv - 1 and not frozen[-1]:
        x = np.full(nv, 0 if a.sum() >= 0 else 1, np.uint8)
        return x, pen(x)
    if nf == 1 and frozen[0] and nv == 4:
        x = (a < 0).astype(np.uint8)
        if x.sum() % 2:
            x[int(np.argmin(np.abs(a)))] ^= 1
        return x, pen(x)
    h = nv // 2
    x, y = a[:h], a[h:]
    al = np.sign(x) * np.sign(y) * np.minimum(np.abs(x), np.abs(y))
    bl, pl = _fast_ssc(al, frozen[:h], Q, stats)
    ar = y + np.where(bl == 1, -x, x)
    if Q is not None:
        if stats is not None:
            stats["sat"] = stats.get("sat", 0) + int(np.sum(np.abs(ar) > Q))
        ar = np.clip(ar, -Q, Q)
    br, pr = _fast_ssc(ar, frozen[h:], Q, stats)
    return np.concatenate([bl ^ br, br]), pl + pr


def test_list_of_one_is_fast_ssc(orc):
    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5)
    b = synth.make_batch(code, 60, 1.5, 9, "i16")
    u, ok, pm, _ = orc.decode_tree(256, 128, code.frozen, code.poly, 8, 1, b.llr, "i16")
    for f in range(b.F):
        x, p = _fast_ssc(b.llr[f], code.frozen)
        uu = orc.polar_transform(x)
        assert (uu[code.info_pos] == u[f]).all()
        assert pm[f] == p


def _saturating_frames(dtype, N, F, seed):
    """Integer frames whose G results leave [-Q, Q] all the time: int8 at the
    headline quantisation (scale 4) of a high-SNR channel plus uniform
    full-range frames; int16 full-range frames (|G| up to 65534).  Some
    frames carry the one value below -Q (-128 / -32768)."""
    rng = np.random.default_rng(seed)
    Q = 127 if dtype == "i8" else 32767
    nt = np.int8 if dtype == "i8" else np.int16
    out = rng.integers(-Q, Q + 1, (F, N))
    if dtype == "i8":
        y = 1.0 - 2.0 * rng.integers(0, 2, (F // 2, N)) + 0.45 * rng.normal(size=(F // 2, N))
        out[: F // 2] = np.clip(np.rint(4 * 2 * y / 0.45 ** 2), -Q, Q)
    out[F - 4:, ::7] = -Q - 1
    return out.astype(nt)


@pytest.mark.parametrize("dtype", ["i8", "i16"])
def test_integer_saturation_pinned_by_fast_ssc(orc, dtype):
    """G saturates every integer result to [-Q, Q] (Q = 127 / 32767), and a
    channel value of -Q - 1 is read as -Q.  At L = 1 the list decoder is
    Fast-SSC, whose decisions and metric (eq. (pm)) depend on the saturated
    magnitudes: the oracle must equal the reference with bound Q on every
    frame, while a bound of Q + 1 or no bound gives other results on some of
    these frames, so a wrong bound in the oracle cannot pass."""
    Q = 127 if dtype == "i8" else 32767
    wrong_bound = {Q + 1: 0, None: 0}
    for N, K in ((256, 128), (128, 64), (64, 32), (64, 40), (1024, 860)):
        code = synth.make_code(N, K, 0, 0, 2.0 if K <= N // 2 else 4.0)
        llr = _saturating_frames(dtype, N, 24, (N, K, Q))
        u, ok, pm, _ = orc.decode_tree(N, K, code.frozen, 0, 0, 1, llr, dtype)
        stats = {}
        for f in range(llr.shape[0]):
            a = np.maximum(llr[f].astype(np.int64), -Q)  # -Q - 1 read as -Q
            x, p = _fast_ssc(a, code.frozen, Q, stats)
            assert (orc.polar_transform(x)[code.info_pos] == u[f]).all(), (N, f)
            assert pm[f] == p, (N, f, pm[f], p)
            for alt in wrong_bound:
                xa, pa = _fast_ssc(a, code.frozen, alt)
                wrong_bound[alt] += int(pa != p or (xa != x).any())
        assert stats["sat"] > 100, stats  # the inputs really saturate
        # the -Q - 1 inputs are read as -Q
        u2, _, pm2, _ = orc.decode_tree(N, K, code.frozen, 0, 0, 1,
                                        np.maximum(llr, -Q).astype(llr.dtype), dtype)
        assert (u2 == u).all() and (pm2 == pm).all()
    assert min(wrong_bound.values()) >= 5, wrong_bound


def test_final_pick_hand_frames(orc):
    """Sec. II-B: the output is the best-metric path that passes the CRC, and
    when none passes the best-metric path with crc_ok = 0.  Frames worked out
    by hand in tests/golden/crc_pick_hand_frames.txt (a (4,4) code whose root
    is one Rate-1 node, CRC-2)."""
    rows = []
    with open(os.path.join(GOLDEN, "crc_pick_hand_frames.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    assert len(rows) >= 3
    frozen = np.zeros(4, np.uint8)
    for row in rows:
        L = int(row[0])
        llr = [int(v) for v in row[1:5]]
        u_want = [int(v) for v in row[5]]
        ok_want, pm_want = int(row[6]), int(row[7])
        for dtype in ("i8", "i16", "f32"):
            a = np.array(llr, dtype={"i8": np.int8, "i16": np.int16, "f32": np.float32}[dtype])
            u, ok, pm, _ = orc.decode_tree(4, 4, frozen, 0x3, 2, L, a, dtype)
            assert list(u[0]) == u_want and ok[0] == ok_want and pm[0] == pm_want, (row, dtype)


def test_negative_zero_decides_zero(orc):
    """eq. (sc:h): the hard decision is 1 exactly when alpha < 0, so an LLR
    of -0.0 decides 0 (a sign-bit decision would decide 1).  The all-zero
    codeword received as exact -0.0 values (G of two -0.0 stays -0.0, so the
    zeros reach the leaves along right branches), or as +2.0 with some
    values -0.0 at the input of a code whose root is one leaf (Rate-1,
    SPC, repetition), decodes to u = 0 with metric 0."""
    code = synth.make_code(256, 128, 8, synth.CRC8_POLY, 2.5)
    llr = np.full((1, 256), -0.0, np.float32)
    for L in (1, 4):
        for mode in (0, 1):
            u, ok, pm, _ = orc.decode_tree(256, 128, code.frozen, code.poly, 8, L, llr, "f32",
                                           mode=mode)
            assert (u == 0).all() and ok.all() and (pm == 0).all(), (L, mode)
    u, ok, pm, _ = orc.decode_scl(256, 128, code.frozen, code.poly, 8, 4, llr, "f32")
    assert (u == 0).all() and ok.all() and (pm == 0).all()
    rng = np.random.default_rng(0)
    for N, frozen in ((8, []), (4, [0]), (8, [0, 1, 2, 3, 4, 5, 6])):
        fz = np.zeros(N, np.uint8)
        fz[frozen] = 1
        K = N - len(frozen)
        x = np.full((6, N), 2.0, np.float32)
        for f in range(6):
            x[f, rng.choice(N, f % N + 1, replace=False)] = -0.0
        for L in (1, 2, 4):
            u, ok, pm, _ = orc.decode_tree(N, K, fz, 0, 0, L, x, "f32", spc_max=N)
            assert (u == 0).all() and (pm == 0).all(), (N, L)


@pytest.mark.parametrize("dtype", ["f32", "i16", "i8"])
def test_leaves_mode_equals_bit_by_bit_scl(orc, dtype):
    """Decoder A with size-1 leaves and decoder B are written independently
    and compute the same list decoder, so they agree exactly."""
    code = synth.make_code(256, 136, 8, synth.CRC8_POLY, 2.0)
    b = synth.make_batch(code, 100, 1.5, 12, dtype)
    for L in (1, 2, 8):
        a = orc.decode_tree(256, 136, code.frozen, code.poly, 8, L, b.llr, dtype, mode=1)
        s = orc.decode_scl(256, 136, code.frozen, code.poly, 8, L, b.llr, dtype)
        for x, y in zip(a, s):
            assert (x == y).all()


def test_rate0_rep_nodes_equal_scl_on_exact_integers(orc):
    """Rate-0 and repetition nodes enumerate their whole constituent code and,
    with unsaturated integer LLRs, reproduce SC-list exactly (the min-sum
    metric identity applied per node)."""
    rng = np.random.default_rng(13)
    for N in (32, 64, 128):
        code = synth.make_code(N, N // 2, 4, 0x3, 2.0)
        for L in (2, 4, 8):
            llr = rng.integers(-60, 61, (60, N)).astype(np.int16)
            a = orc.decode_tree(N, N // 2, code.frozen, code.poly, 4, L, llr, "i16", mode=2)
            s = orc.decode_scl(N, N // 2, code.frozen, code.poly, 4, L, llr, "i16")
            for x, y in zip(a, s):
                assert (x == y).all()


def _wilson(k, n, z=1.96):
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return c - h, c + h


def test_dec_spc4_fer_matches_sc_list():
    """Sec. VII-C: without SPC nodes longer than four, the proposed decoder's
    FER matches SC-list.  Checked as overlapping 95% intervals."""
    import oracle as orc

    code = synth.make_code(512, 256, 8, synth.CRC8_POLY, 2.0)
    b = synth.make_batch(code, 3000, 1.75, 99, "f32")
    a = orc.decode_tree(512, 256, code.frozen, code.poly, 8, 4, b.llr, "f32")[0]
    s = orc.decode_scl(512, 256, code.frozen, code.poly, 8, 4, b.llr, "f32")[0]
    ea = int((a != b.info).any(1).sum())
    es = int((s != b.info).any(1).sum())
    la, ha = _wilson(ea, b.F)
    ls, hs = _wilson(es, b.F)
    assert ea > 0 and es > 0
    assert la <= hs and ls <= ha


def test_near_tie_flag(orc):
    """An exact metric tie at the pruning boundary is reported for float32
    and never for integers (where ties are resolved exactly)."""
    frozen = np.zeros(2, np.uint8)
    a = np.array([1.5, -1.5], np.float32)
    _, _, _, nt = orc.decode_tree(2, 2, frozen, 0, 0, 2, a, "f32")
    assert nt[0] == 1
    a = np.array([3, -3], np.int8)
    _, _, _, nt = orc.decode_tree(2, 2, frozen, 0, 0, 2, a, "i8")
    assert nt[0] == 0


def test_int8_metrics_stay_within_127_N():
    """Every int8 path metric lies in [-127 N, 0]: a position's |LLR| is at
    most 127 after saturation and each position is charged by one leaf only.
    (The int8 kernels pack metric and candidate index into 32-bit ranking
    keys on this bound.)  Checked on the whole final list, with saturated and
    adversarial inputs, including every-value-negative frames."""
    import oracle

    rng = np.random.default_rng(127)
    for N, K, L in ((4096, 3441, 32), (1024, 512, 128), (256, 128, 32)):
        code = synth.make_code(N, K, 0, 0, 2.0)
        for trial in range(3):
            if trial == 0:
                llr = np.where(rng.random(N) < 0.5, -127, 127).astype(np.int8)
            elif trial == 1:
                llr = np.full(N, -127, np.int8)
            else:
                llr = rng.integers(-128, 128, N).astype(np.int8)
            _, pm = oracle.decode_tree_list(N, K, code.frozen, L, llr[None, :], "i8")
            assert pm.max() <= 0 and pm.min() >= -127 * N, (N, trial, pm.min())
