"""The C-ABI library: it loads, exports every declared entry point, and its
host-only schedule compiler builds the decoding tree of Sec. II-D.  No GPU
needed (no decode calls)."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def pk():
    import paper_1505_01466_amd as pk

    return pk


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "pscl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pscl_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(pk):
    names = _declared_functions()
    assert "pscl_decode" in names and "pscl_plan_create" in names
    for name in names:
        assert hasattr(pk.lib, name), name


def test_status_strings_and_version(pk):
    for s in range(8):
        assert pk.lib.pscl_status_str(s)
    assert pk.lib.pscl_status_str(7) == b"timed out"
    assert pk.lib.pscl_version() >= 100


def _golden_ops():
    for line in open(os.path.join(GOLDEN, "fig1_code_8_4.txt")):
        if line.startswith("fast_ssc_ops"):
            return line.split()[1:]
        if line.startswith("frozen"):
            frozen_pos = [int(v) for v in line.split()[1:]]
    raise AssertionError


def test_schedule_of_fig2_code(pk):
    frozen = np.zeros(8, np.uint8)
    frozen[[0, 1, 2, 4]] = 1
    ops = pk.schedule(8, frozen, L=4)
    got = [f"{pk.OP_NAMES[t]}{1 << k}" for t, k, _, _ in ops]
    assert got == _golden_ops()
    # Rep<4> forks into 2 paths, SPC<4> into 2 x 8 -> capped at L = 4
    assert [p for *_, p in ops] == [1, 2, 2, 4, 4]


def _leaves(frozen, spc_max, mode):
    out = []

    def rec(f):
        nv = len(f)
        nf = int(f.sum())
        if nv == 1:
            out.append(("R0" if nf else "R1", 0))
            return
        if mode == 0:
            if nf == nv:
                return out.append(("R0", nv.bit_length() - 1))
            if nf == 0:
                return out.append(("R1", nv.bit_length() - 1))
            if nf == nv - 1 and not f[-1]:
                return out.append(("REP", nv.bit_length() - 1))
            if nf == 1 and f[0] and 4 <= nv <= spc_max:
                return out.append(("SPC", nv.bit_length() - 1))
        rec(f[: nv // 2])
        rec(f[nv // 2:])

    rec(frozen)
    return out


@pytest.mark.parametrize("N,K,r,d", [(1024, 512, 8, 2.5), (2048, 1723, 32, 4.0),
                                     (1024, 860, 32, 4.0), (4096, 3441, 32, 4.0)])
@pytest.mark.parametrize("mode,spc_max", [(0, 4), (0, 4096), (1, 4)])
def test_schedule_leaves_and_paths(pk, N, K, r, d, mode, spc_max):
    code = synth.make_code(N, K, r, synth.CRC32_POLY, d)
    L = 32
    ops = pk.schedule(N, code.frozen, L, spc_max, mode)
    leaves = [(pk.OP_NAMES[t], k) for t, k, _, _ in ops if t >= 3]
    assert leaves == _leaves(code.frozen, spc_max, mode)
    # every internal node appears as F, G, Combine in that order
    n_int = sum(1 for t, *_ in ops if t == 0)
    assert n_int == sum(1 for t, *_ in ops if t == 1) == sum(1 for t, *_ in ops if t == 2)
    # list size grows by the candidate count, capped at L
    P = 1
    cands = {"R0": 1, "REP": 2, "SPC": 8}
    for t, k, side, paths in ops:
        name = pk.OP_NAMES[t]
        if name in cands or name == "R1":
            c = cands.get(name, 2 if k == 0 else 4)
            P = min(L, P * c)
        assert paths == P
    # the covered leaf sizes add up to N
    assert sum(1 << k for _, k in leaves) == N


def test_schedule_rejects_bad_arguments(pk):
    frozen = np.zeros(8, np.uint8)
    n = ctypes.c_int()
    buf = np.zeros(64, np.int32)
    p = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    u8 = frozen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert pk.lib.pscl_schedule(12, u8, 4, 4, 0, p, 16, ctypes.byref(n)) == 1  # N not 2^n
    assert pk.lib.pscl_schedule(8, u8, 3, 4, 0, p, 16, ctypes.byref(n)) == 1  # L not 2^k
    assert pk.lib.pscl_schedule(8, u8, 4, 4, 7, p, 16, ctypes.byref(n)) == 1  # bad mode
    assert pk.lib.pscl_schedule(8, u8, 4, 4, 0, p, 0, ctypes.byref(n)) == 1  # no room
    assert n.value == 1  # count still reported (root is one Rate-1 node)


def test_plan_create_validates_before_touching_the_device(pk):
    frozen = np.zeros(8, np.uint8)
    frozen[:4] = 1
    h = ctypes.c_void_p()
    u8 = frozen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    # K does not match the mask
    assert pk.lib.pscl_plan_create(8, 5, u8, 0, 0, 4, 0, 4, 0, ctypes.byref(h)) == 1
    # crc longer than K
    assert pk.lib.pscl_plan_create(8, 4, u8, 0x7, 8, 4, 0, 4, 0, ctypes.byref(h)) == 1
    # bad dtype, bad L
    assert pk.lib.pscl_plan_create(8, 4, u8, 0, 0, 4, 9, 4, 0, ctypes.byref(h)) == 1
    assert pk.lib.pscl_plan_create(8, 4, u8, 0, 0, 256, 0, 4, 0, ctypes.byref(h)) == 1
    assert pk.lib.pscl_plan_create(8, 4, u8, 0, 0, 48, 0, 4, 0, ctypes.byref(h)) == 1
    # L = 128 needs two wavefronts (at most 64 paths per wavefront)
    cfg = pk.LaunchCfg(64, 0, 0)
    assert pk.lib.pscl_plan_create_cfg(8, 4, u8, 0, 0, 128, 0, 4, 0, ctypes.byref(cfg),
                                       ctypes.byref(h)) == 2
    assert not h.value


def test_decode_rejects_null_plan(pk):
    assert pk.lib.pscl_decode(None, None, 0, None, None, None, None) == 1


def test_launch_cfg_and_autotune_validate_arguments(pk):
    frozen = np.zeros(8, np.uint8)
    frozen[:4] = 1
    h = ctypes.c_void_p()
    u8 = frozen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    for threads in (32, 96, 2048, -64):
        cfg = pk.LaunchCfg(threads, 0, 0)
        assert pk.lib.pscl_plan_create_cfg(8, 4, u8, 0, 0, 4, 0, 4, 0, ctypes.byref(cfg),
                                           ctypes.byref(h)) == 1
    # negative budget; recompute outside 1..3; fused-leaf size outside -1..5;
    # levels per F / G pass outside 1..2
    for bad in (pk.LaunchCfg(64, -1, 0), pk.LaunchCfg(64, 0, 0, 4), pk.LaunchCfg(64, 0, 0, -1),
                pk.LaunchCfg(64, 0, 0, 0, 6), pk.LaunchCfg(64, 0, 0, 0, -2),
                pk.LaunchCfg(64, 0, 0, 0, 0, 3), pk.LaunchCfg(64, 0, 0, 0, 0, -1)):
        assert pk.lib.pscl_plan_create_cfg(8, 4, u8, 0, 0, 4, 0, 4, 0, ctypes.byref(bad),
                                           ctypes.byref(h)) == 1
    assert not h.value
    best = pk.LaunchCfg(0, 0, 0)
    # no output, no frames, no input
    assert pk.lib.pscl_autotune(8, 4, u8, 0, 0, 4, 0, 4, 0, None, 1, None, None, None) == 1
    assert pk.lib.pscl_autotune(8, 4, u8, 0, 0, 4, 0, 4, 0, None, 1, None, ctypes.byref(best),
                                None) == 1


def test_mixed_launch_validates_arguments(pk):
    h = ctypes.c_void_p()
    vp = ctypes.c_void_p
    # no plans, bad job bound
    assert pk.lib.pscl_group_create(None, 1, 8, 4, None, ctypes.byref(h)) == 1
    plans = (vp * 1)(None)
    assert pk.lib.pscl_group_create(plans, 1, 8, 4, None, ctypes.byref(h)) == 1
    assert pk.lib.pscl_group_create(plans, 0, 8, 4, None, ctypes.byref(h)) == 1
    assert not h.value
    assert pk.lib.pscl_group_decode(None, None, 0, None) == 1
    assert pk.lib.pscl_decode_mixed(None, 1, None, 0, None) == 1
    assert pk.lib.pscl_decode_mixed(plans, 1, None, 0, None) == 1
    assert pk.lib.pscl_decode_mixed(plans, 1, None, -1, None) == 1
    pk.lib.pscl_group_destroy(None)


def test_server_and_replay_validate_arguments(pk):
    h = ctypes.c_void_p()
    vp = ctypes.c_void_p
    assert pk.lib.pscl_server_create(None, ctypes.byref(h)) == 1
    plans = (vp * 1)(None)
    for bad in (dict(n_plans=0), dict(n_plans=1), dict(n_plans=1, streams=9),
                dict(n_plans=1, max_requests=-1), dict(n_plans=1, footprint=-1)):
        cfg = pk.ServerCfg(plans, bad.get("n_plans", 1), bad.get("streams", 0),
                           bad.get("max_requests", 0), 0, 0, 0, bad.get("footprint", 0))
        assert pk.lib.pscl_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert not h.value
    t = ctypes.c_uint64()
    d = ctypes.c_int()
    assert pk.lib.pscl_server_submit(None, None, None, ctypes.byref(t)) == 1
    assert pk.lib.pscl_server_poll(None, 1, ctypes.byref(d), None) == 1
    assert pk.lib.pscl_server_wait(None, 1, -1.0, None) == 1
    assert pk.lib.pscl_server_wait(None, 1, 5.0, None) == 1
    assert pk.lib.pscl_plan_footprint(None, None) == 1
    assert pk.lib.pscl_server_stats(None, None, None, None, None, None, 0) == 1
    pk.lib.pscl_server_destroy(None)
    # replay: no plans for the baseline, stream count outside 1..8, negative
    # count, missing arrays
    assert pk.lib.pscl_replay(None, None, 0, 1, None, None, 0, None, None) == 1
    assert pk.lib.pscl_replay(None, plans, 1, 0, None, None, 0, None, None) == 1
    assert pk.lib.pscl_replay(None, plans, 1, 9, None, None, 0, None, None) == 1
    assert pk.lib.pscl_replay(None, plans, 1, 1, None, None, -1, None, None) == 1
    assert pk.lib.pscl_replay(None, plans, 1, 1, None, None, 2, None, None) == 1


def test_adaptive_validates_arguments(pk):
    h = ctypes.c_void_p()
    assert pk.lib.pscl_adaptive_create(None, None, 8, ctypes.byref(h)) == 1
    assert pk.lib.pscl_adaptive_create(None, None, 0, ctypes.byref(h)) == 1
    assert not h.value
    assert pk.lib.pscl_adaptive_decode(None, None, 1, None, None, None, None, None) == 1
    pk.lib.pscl_adaptive_destroy(None)


def test_generator_validates_arguments(pk):
    h = ctypes.c_void_p()
    fz = np.ones(8, np.uint8)
    fz[[3, 5, 6, 7]] = 0
    p = fz.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert pk.lib.pscl_generator_create(8, 4, None, 0x7, 3, 0, ctypes.byref(h)) == 1
    assert pk.lib.pscl_generator_create(12, 4, p, 0x7, 3, 0, ctypes.byref(h)) == 1  # N not 2^n
    assert pk.lib.pscl_generator_create(8, 5, p, 0x7, 3, 0, ctypes.byref(h)) == 1  # K != unfrozen
    assert pk.lib.pscl_generator_create(8, 4, p, 0x7, 4, 0, ctypes.byref(h)) == 1  # r >= K
    assert pk.lib.pscl_generator_create(8, 4, p, 0x7, 3, 9, ctypes.byref(h)) == 1  # dtype
    assert not h.value
    assert pk.lib.pscl_generate(None, 1, 0, 1, 4.0, None, None, None) == 1
    pk.lib.pscl_generator_destroy(None)


def test_import_fails_loudly_without_the_library(tmp_path):
    """The package has no CPU fallback: a copy of it without libpscl.so
    refuses to import."""
    import shutil
    import subprocess
    import sys

    src = os.path.join(ROOT, "paper_1505_01466_amd")
    dst = tmp_path / "paper_1505_01466_amd"
    dst.mkdir()
    for name in os.listdir(src):
        if name.endswith(".py"):
            shutil.copy(os.path.join(src, name), dst / name)
    r = subprocess.run([sys.executable, "-c", "import paper_1505_01466_amd"], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=120,
                       env={**os.environ, "PYTHONPATH": str(tmp_path)})
    assert r.returncode != 0
    assert "libpscl.so not found" in r.stderr
