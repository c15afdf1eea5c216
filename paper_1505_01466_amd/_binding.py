"""ctypes binding of libpscl.so.  Argument marshalling only: every step of
decoding runs in the library's HIP kernels.  torch provides device memory
and the current stream.

The library must have been built (``python -m paper_1505_01466_amd.build`` or
``__graft_entry__.build()``); importing this module fails loudly otherwise.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpscl.so")

PSCL_F32, PSCL_I16, PSCL_I8 = 0, 1, 2
DTYPES = {"f32": PSCL_F32, "i16": PSCL_I16, "i8": PSCL_I8}
MODE_TREE, MODE_SCL_LEAVES = 0, 1
OP_NAMES = ("F", "G", "COMB", "R0", "REP", "R1", "SPC")

_STATUS = {
    0: "ok",
    1: "invalid argument",
    2: "unsupported configuration",
    3: "device out of memory",
    4: "HIP runtime error",
    5: "no gfx950 device",
    6: "busy",
    7: "timed out",
}


class PsclError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_STATUS.get(status, 'unknown')} (status {status})")
        self.status = status


class LaunchCfg(ctypes.Structure):
    """pscl_launch_cfg: threads per workgroup and LDS budget (0 = default)."""

    _fields_ = [("threads", ctypes.c_int), ("lds_budget", ctypes.c_int),
                ("max_wg_per_cu", ctypes.c_int), ("recompute", ctypes.c_int),
                ("fuse_log2", ctypes.c_int), ("unroll", ctypes.c_int)]


class Job(ctypes.Structure):
    """pscl_job: F frames of plans[plan] with their own device buffers."""

    _fields_ = [("plan", ctypes.c_int), ("llr", ctypes.c_void_p), ("F", ctypes.c_int64),
                ("u_hat", ctypes.c_void_p), ("crc_ok", ctypes.c_void_p), ("pm", ctypes.c_void_p)]


class ServerCfg(ctypes.Structure):
    """pscl_server_cfg (zero fields take the defaults)."""

    _fields_ = [("plans", ctypes.POINTER(ctypes.c_void_p)), ("n_plans", ctypes.c_int),
                ("streams", ctypes.c_int), ("max_requests", ctypes.c_int),
                ("max_pending_frames", ctypes.c_int64), ("max_batch_frames", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int), ("max_footprint_bytes", ctypes.c_int64),
                ("persistent", ctypes.c_int), ("idle_us", ctypes.c_int),
                ("wg_per_cu", ctypes.c_int), ("active_per_cu", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libpscl.so not found at {LIB_PATH}; build it with "
            "`python -m paper_1505_01466_amd.build` (hipcc, gfx950)"
        )
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_i64, c_u64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    ip = ctypes.POINTER(c_int)
    lib.pscl_status_str.argtypes = [c_int]
    lib.pscl_status_str.restype = ctypes.c_char_p
    lib.pscl_version.argtypes = []
    lib.pscl_version.restype = c_int
    lib.pscl_schedule.argtypes = [c_int, u8p, c_int, c_int, c_int, i32p, c_int, ip]
    lib.pscl_schedule.restype = c_int
    lib.pscl_plan_create.argtypes = [c_int, c_int, u8p, c_u64, c_int, c_int, c_int, c_int, c_int,
                                     ctypes.POINTER(vp)]
    lib.pscl_plan_create.restype = c_int
    lib.pscl_plan_destroy.argtypes = [vp]
    lib.pscl_plan_destroy.restype = None
    lib.pscl_plan_footprint.argtypes = [vp, ctypes.POINTER(c_i64)]
    lib.pscl_plan_footprint.restype = c_int
    lib.pscl_plan_reserve.argtypes = [vp]
    lib.pscl_plan_reserve.restype = c_int
    lib.pscl_decode.argtypes = [vp, vp, c_i64, vp, vp, vp, vp]
    lib.pscl_decode.restype = c_int
    lib.pscl_decode_noalloc.argtypes = [vp, vp, c_i64, vp, vp, vp, vp]
    lib.pscl_decode_noalloc.restype = c_int
    lib.pscl_decode_oneshot.argtypes = [c_int, c_int, u8p, c_u64, c_int, c_int, c_int, vp, c_i64,
                                        vp, vp, vp]
    lib.pscl_decode_oneshot.restype = c_int
    lib.pscl_plan_info.argtypes = [vp, ip, ip, ip, ip, ctypes.POINTER(c_i64), ip]
    lib.pscl_plan_info.restype = c_int
    lib.pscl_plan_create_cfg.argtypes = [c_int, c_int, u8p, c_u64, c_int, c_int, c_int, c_int,
                                         c_int, ctypes.POINTER(LaunchCfg), ctypes.POINTER(vp)]
    lib.pscl_plan_create_cfg.restype = c_int
    lib.pscl_autotune.argtypes = [c_int, c_int, u8p, c_u64, c_int, c_int, c_int, c_int, c_int,
                                  vp, c_i64, vp, ctypes.POINTER(LaunchCfg),
                                  ctypes.POINTER(ctypes.c_float)]
    lib.pscl_autotune.restype = c_int
    lib.pscl_group_create.argtypes = [ctypes.POINTER(vp), c_int, c_int, c_int,
                                      ctypes.POINTER(LaunchCfg), ctypes.POINTER(vp)]
    lib.pscl_group_create.restype = c_int
    lib.pscl_autotune_group.argtypes = [ctypes.POINTER(vp), c_int, ctypes.POINTER(Job), c_int, vp,
                                        ctypes.POINTER(LaunchCfg), ip,
                                        ctypes.POINTER(ctypes.c_float)]
    lib.pscl_autotune_group.restype = c_int
    lib.pscl_group_destroy.argtypes = [vp]
    lib.pscl_group_destroy.restype = None
    lib.pscl_group_decode.argtypes = [vp, ctypes.POINTER(Job), c_int, vp]
    lib.pscl_group_decode.restype = c_int
    lib.pscl_decode_mixed.argtypes = [ctypes.POINTER(vp), c_int, ctypes.POINTER(Job), c_int, vp]
    lib.pscl_decode_mixed.restype = c_int
    lib.pscl_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]
    lib.pscl_server_create.restype = c_int
    lib.pscl_server_destroy.argtypes = [vp]
    lib.pscl_server_destroy.restype = None
    lib.pscl_server_submit.argtypes = [vp, ctypes.POINTER(Job), vp, ctypes.POINTER(c_u64)]
    lib.pscl_server_submit.restype = c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pscl_server_poll.argtypes = [vp, c_u64, ip, dp]
    lib.pscl_server_poll.restype = c_int
    lib.pscl_server_wait.argtypes = [vp, c_u64, ctypes.c_double, dp]
    lib.pscl_server_wait.restype = c_int
    i64p = ctypes.POINTER(c_i64)
    lib.pscl_server_stats.argtypes = [vp, i64p, i64p, i64p, dp, dp, c_int]
    lib.pscl_server_stats.restype = c_int
    lib.pscl_replay.argtypes = [vp, ctypes.POINTER(vp), c_int, c_int, ctypes.POINTER(Job), dp,
                                c_int, dp, dp]
    lib.pscl_replay.restype = c_int
    lib.pscl_adaptive_create.argtypes = [vp, vp, c_i64, ctypes.POINTER(vp)]
    lib.pscl_adaptive_create.restype = c_int
    lib.pscl_adaptive_destroy.argtypes = [vp]
    lib.pscl_adaptive_destroy.restype = None
    lib.pscl_adaptive_decode.argtypes = [vp, vp, c_i64, vp, vp, vp, vp, vp]
    lib.pscl_adaptive_decode.restype = c_int
    lib.pscl_generator_create.argtypes = [c_int, c_int, u8p, c_u64, c_int, c_int,
                                          ctypes.POINTER(vp)]
    lib.pscl_generator_create.restype = c_int
    lib.pscl_generator_destroy.argtypes = [vp]
    lib.pscl_generator_destroy.restype = None
    lib.pscl_generate.argtypes = [vp, c_u64, c_i64, c_i64, ctypes.c_double, vp, vp, vp]
    lib.pscl_generate.restype = c_int
    return lib


lib = _load()


def _check(status: int, what: str):
    if status != 0:
        raise PsclError(status, what)


def _mask(frozen) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8))


def _u8p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def schedule(N: int, frozen, L: int, spc_max: int = 4, mode: int = MODE_TREE) -> np.ndarray:
    """Operation schedule of the decoding tree (host only, no GPU needed):
    rows of (op type, log2 node size, side, active paths after)."""
    fz = _mask(frozen)
    n = ctypes.c_int(0)
    cap = 4 * N + 8
    ops = np.zeros((cap, 4), dtype=np.int32)
    _check(lib.pscl_schedule(N, _u8p(fz), L, spc_max, mode,
                             ops.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap,
                             ctypes.byref(n)), "pscl_schedule")
    return ops[: n.value].copy()


def _stream_handle(device):
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A decoding plan on the current device (see pscl_plan_create)."""

    def __init__(self, N: int, K: int, frozen, crc_poly: int, crc_len: int, L: int,
                 dtype: str = "f32", spc_max: int = 4, mode: int = MODE_TREE,
                 threads: int = 0, lds_budget: int = 0, max_wg_per_cu: int = 0,
                 recompute: int = 0, fuse_log2: int = 0, unroll: int = 0,
                 cfg: dict | None = None):
        import torch

        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        self.N, self.K, self.L, self.dtype = N, K, L, dtype
        self.crc_poly, self.crc_len, self.spc_max, self.mode = crc_poly, crc_len, spc_max, mode
        self.device = torch.device("cuda", torch.cuda.current_device())
        fz = _mask(frozen)
        h = ctypes.c_void_p(None)
        if cfg is not None:  # a configuration as autotune() returns it
            threads, lds_budget = cfg.get("threads", 0), cfg.get("lds_budget", 0)
            max_wg_per_cu = cfg.get("max_wg_per_cu", 0)
            recompute, fuse_log2 = cfg.get("recompute", 0), cfg.get("fuse_log2", 0)
            unroll = cfg.get("unroll", 0)
        self.cfg = {"threads": threads, "lds_budget": lds_budget, "max_wg_per_cu": max_wg_per_cu,
                    "recompute": recompute, "fuse_log2": fuse_log2, "unroll": unroll}
        cfg = LaunchCfg(threads, lds_budget, max_wg_per_cu, recompute, fuse_log2, unroll)
        _check(lib.pscl_plan_create_cfg(N, K, _u8p(fz), crc_poly, crc_len, L, DTYPES[dtype],
                                        spc_max, mode, ctypes.byref(cfg), ctypes.byref(h)),
               "pscl_plan_create_cfg")
        self._h = h

    def info(self) -> dict:
        fw, nt, wg, lds, glob = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(),
                                 ctypes.c_int())
        ws = ctypes.c_int64()
        _check(lib.pscl_plan_info(self._h, ctypes.byref(fw), ctypes.byref(nt), ctypes.byref(wg),
                                  ctypes.byref(lds), ctypes.byref(ws), ctypes.byref(glob)),
               "pscl_plan_info")
        return {"frames_per_wg": fw.value, "threads": nt.value, "workgroups": wg.value,
                "lds_bytes": lds.value, "workspace_bytes": ws.value,
                "first_global_stage": glob.value}

    def footprint(self) -> int:
        """Device bytes per frame in flight (pscl_plan_footprint)."""
        b = ctypes.c_int64(0)
        _check(lib.pscl_plan_footprint(self._h, ctypes.byref(b)), "pscl_plan_footprint")
        return b.value

    def reserve(self):
        """Allocate the plan's workspace now (pscl_plan_reserve)."""
        _check(lib.pscl_plan_reserve(self._h), "pscl_plan_reserve")

    def decode(self, llr, u_hat=None, crc_ok=None, pm=None):
        """Decode llr (F x N device tensor in the plan's dtype) into
        (u_hat F x K uint8, crc_ok F uint8, pm F float32/int32)."""
        import torch

        want = {"f32": torch.float32, "i16": torch.int16, "i8": torch.int8}[self.dtype]
        if llr.dtype != want or llr.dim() != 2 or llr.shape[1] != self.N:
            raise ValueError(f"llr must be an F x {self.N} {want} tensor")
        if llr.device != self.device or not llr.is_contiguous():
            raise ValueError("llr must be a contiguous tensor on the plan's device")
        F = llr.shape[0]
        if u_hat is None:
            u_hat = torch.empty((F, self.K), dtype=torch.uint8, device=self.device)
        if crc_ok is None:
            crc_ok = torch.empty(F, dtype=torch.uint8, device=self.device)
        if pm is None:
            pm = torch.empty(F, dtype=torch.float32 if self.dtype == "f32" else torch.int32,
                             device=self.device)
        _check(lib.pscl_decode(self._h, llr.data_ptr(), F, u_hat.data_ptr(), crc_ok.data_ptr(),
                               pm.data_ptr(), _stream_handle(self.device)), "pscl_decode")
        return u_hat, crc_ok, pm

    def decode_noalloc(self, llr, u_hat, crc_ok, pm):
        """pscl_decode_noalloc into caller-provided outputs: the library's
        static device scratch instead of the plan's workspace (no device
        allocation; overlapping calls on one device race)."""
        if llr.device != self.device or not llr.is_contiguous() or llr.shape[1] != self.N:
            raise ValueError(f"llr must be a contiguous F x {self.N} tensor on the plan's device")
        F = llr.shape[0]
        _check(lib.pscl_decode_noalloc(self._h, llr.data_ptr(), F, u_hat.data_ptr(),
                                       crc_ok.data_ptr(), pm.data_ptr(),
                                       _stream_handle(self.device)), "pscl_decode_noalloc")
        return u_hat, crc_ok, pm

    def close(self):
        if getattr(self, "_h", None):
            lib.pscl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode(N: int, K: int, frozen, crc_poly: int, crc_len: int, L: int, llr, dtype: str = "f32"):
    """decode(N, K, frozen_mask, crc_poly, L, llr[F x N]) -> (u_hat[F x K], crc_ok[F]) with the
    plan cached inside the library (Dec-SPC-4 tree)."""
    import torch

    F = llr.shape[0]
    u_hat = torch.empty((F, K), dtype=torch.uint8, device=llr.device)
    crc_ok = torch.empty(F, dtype=torch.uint8, device=llr.device)
    fz = _mask(frozen)
    _check(lib.pscl_decode_oneshot(N, K, _u8p(fz), crc_poly, crc_len, L, DTYPES[dtype],
                                   llr.data_ptr(), F, u_hat.data_ptr(), crc_ok.data_ptr(),
                                   _stream_handle(llr.device)), "pscl_decode_oneshot")
    return u_hat, crc_ok


def autotune(N: int, K: int, frozen, crc_poly: int, crc_len: int, L: int, llr,
             dtype: str = "f32", spc_max: int = 4, mode: int = MODE_TREE):
    """pscl_autotune on the frames llr (F x N device tensor in dtype): returns
    ({"threads": t, "lds_budget": b}, milliseconds per decode call)."""
    if llr.dim() != 2 or llr.shape[1] != N or not llr.is_contiguous():
        raise ValueError(f"llr must be a contiguous F x {N} tensor")
    fz = _mask(frozen)
    best = LaunchCfg(0, 0, 0)
    ms = ctypes.c_float(0.0)
    _check(lib.pscl_autotune(N, K, _u8p(fz), crc_poly, crc_len, L, DTYPES[dtype], spc_max, mode,
                             llr.data_ptr(), llr.shape[0], _stream_handle(llr.device),
                             ctypes.byref(best), ctypes.byref(ms)), "pscl_autotune")
    return ({"threads": best.threads, "lds_budget": best.lds_budget,
             "max_wg_per_cu": best.max_wg_per_cu, "recompute": best.recompute,
             "fuse_log2": best.fuse_log2, "unroll": best.unroll}, ms.value)


def _jobs(plans, work):
    """Marshals [(plan index, llr tensor), ...] into pscl_job entries with
    freshly allocated outputs; returns (ctypes array, outputs)."""
    import torch

    arr = (Job * max(1, len(work)))()
    outs = []
    for i, (pi, llr) in enumerate(work):
        pl = plans[pi]
        want = {"f32": torch.float32, "i16": torch.int16, "i8": torch.int8}[pl.dtype]
        if llr.dtype != want or llr.dim() != 2 or llr.shape[1] != pl.N or not llr.is_contiguous():
            raise ValueError(f"job {i}: llr must be a contiguous F x {pl.N} {want} tensor")
        F = llr.shape[0]
        u = torch.empty((F, pl.K), dtype=torch.uint8, device=llr.device)
        ok = torch.empty(F, dtype=torch.uint8, device=llr.device)
        pm = torch.empty(F, dtype=torch.float32 if pl.dtype == "f32" else torch.int32,
                         device=llr.device)
        arr[i] = Job(pi, llr.data_ptr(), F, u.data_ptr(), ok.data_ptr(), pm.data_ptr())
        outs.append((u, ok, pm))
    return arr, outs


def autotune_group(plans, work):
    """pscl_autotune_group on work = [(plan index, llr tensor), ...]: returns
    (one configuration dict per plan, group threads, milliseconds per
    call).  Rebuild the plans with Plan(..., cfg=c) and the group with
    Group(plans, threads=t)."""
    plans = list(plans)
    hs = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    arr, _ = _jobs(plans, work)
    cfgs = (LaunchCfg * len(plans))()
    t = ctypes.c_int(0)
    ms = ctypes.c_float(0.0)
    _check(lib.pscl_autotune_group(hs, len(plans), arr, len(work), _stream_handle(plans[0].device),
                                   cfgs, ctypes.byref(t), ctypes.byref(ms)), "pscl_autotune_group")
    out = [{"threads": c.threads, "lds_budget": c.lds_budget, "max_wg_per_cu": c.max_wg_per_cu,
            "recompute": c.recompute, "fuse_log2": c.fuse_log2, "unroll": c.unroll} for c in cfgs]
    return out, t.value, ms.value


class Group:
    """A group of plans of one dtype decoded together in one persistent
    launch (see pscl_group_create); the plans must outlive it."""

    def __init__(self, plans, max_jobs: int = 64, max_inflight: int = 4, threads: int = 0):
        self.plans = list(plans)
        hs = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        cfg = LaunchCfg(threads, 0, 0)
        h = ctypes.c_void_p(None)
        _check(lib.pscl_group_create(hs, len(self.plans), max_jobs, max_inflight,
                                     ctypes.byref(cfg), ctypes.byref(h)), "pscl_group_create")
        self._h = h

    def decode(self, work):
        """work: [(plan index, llr F x N device tensor), ...] -> [(u_hat, crc_ok, pm), ...]."""
        arr, outs = _jobs(self.plans, work)
        dev = self.plans[0].device
        _check(lib.pscl_group_decode(self._h, arr, len(work), _stream_handle(dev)),
               "pscl_group_decode")
        return outs

    def close(self):
        if getattr(self, "_h", None):
            lib.pscl_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_mixed(plans, work):
    """pscl_decode_mixed: the group for this list of plans is cached by the
    library.  work: [(plan index, llr tensor), ...] -> [(u_hat, crc_ok, pm), ...]."""
    plans = list(plans)
    hs = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    arr, outs = _jobs(plans, work)
    _check(lib.pscl_decode_mixed(hs, len(plans), arr, len(work), _stream_handle(plans[0].device)),
           "pscl_decode_mixed")
    return outs


class Server:
    """A serving loop over a list of plans of one dtype (see
    pscl_server_create).  submit() keeps each request's buffers alive until
    it has been reported done."""

    def __init__(self, plans, streams: int = 2, max_requests: int = 0,
                 max_pending_frames: int = 0, max_batch_frames: int = 0,
                 max_batch_requests: int = 0, max_footprint_bytes: int = 0,
                 persistent: bool = False, idle_us: int = 0, wg_per_cu: int = 0,
                 active_per_cu: int = 0):
        self.plans = list(plans)
        self._hs = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        cfg = ServerCfg(self._hs, len(self.plans), streams, max_requests, max_pending_frames,
                        max_batch_frames, max_batch_requests, max_footprint_bytes,
                        1 if persistent else 0, idle_us, wg_per_cu, active_per_cu)
        h = ctypes.c_void_p(None)
        _check(lib.pscl_server_create(ctypes.byref(cfg), ctypes.byref(h)), "pscl_server_create")
        self._h = h
        self._live = {}

    def submit(self, plan_index: int, llr):
        """Queue F frames (llr F x N device tensor) of plans[plan_index];
        returns (ticket, (u_hat, crc_ok, pm)).  The request is decoded after
        the work already issued on the current stream (which may still be
        producing llr).  Raises PsclError (status 6) when the server is full."""
        arr, outs = _jobs(self.plans, [(plan_index, llr)])
        t = ctypes.c_uint64(0)
        _check(lib.pscl_server_submit(self._h, arr, _stream_handle(llr.device), ctypes.byref(t)),
               "pscl_server_submit")
        self._live[t.value] = (llr, outs[0])
        return t.value, outs[0]

    def poll(self, ticket: int):
        """(done, latency in microseconds or None)."""
        d = ctypes.c_int(0)
        lat = ctypes.c_double(0.0)
        _check(lib.pscl_server_poll(self._h, ticket, ctypes.byref(d), ctypes.byref(lat)),
               "pscl_server_poll")
        if d.value:
            self._live.pop(ticket, None)
            return True, lat.value
        return False, None

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> float:
        """Latency in microseconds; raises PsclError (status 7) when the
        request is not done within timeout_ms (negative: no limit)."""
        lat = ctypes.c_double(0.0)
        _check(lib.pscl_server_wait(self._h, ticket, float(timeout_ms), ctypes.byref(lat)),
               "pscl_server_wait")
        self._live.pop(ticket, None)
        return lat.value

    def stats(self, reset: bool = False) -> dict:
        r, f, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        p50, p99 = ctypes.c_double(), ctypes.c_double()
        _check(lib.pscl_server_stats(self._h, ctypes.byref(r), ctypes.byref(f), ctypes.byref(n),
                                     ctypes.byref(p50), ctypes.byref(p99), int(reset)),
               "pscl_server_stats")
        return {"requests": r.value, "frames": f.value, "launches": n.value,
                "p50_us": p50.value, "p99_us": p99.value}

    def close(self):
        if getattr(self, "_h", None):
            lib.pscl_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(plans, work, arrival_us, server=None, streams: int = 1):
    """pscl_replay: request i = work[i] = (plan index, llr tensor) arrives
    arrival_us[i] microseconds after the start; through `server`, or, when
    server is None, as one pscl_decode per request round-robin on `streams`
    streams, plans then holding `streams` sets of the codes' plans
    (len(plans) = streams * codes; a plan index in work names a code).
    Returns (outputs, latencies in microseconds as a numpy array, elapsed
    microseconds)."""
    plans = list(plans)
    if server is None and len(plans) % streams:
        raise ValueError("plans must hold one set of plans per stream")
    n_codes = len(plans) if server is not None else len(plans) // streams
    hs = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    arr, outs = _jobs(plans[:n_codes], work)
    arrivals = np.ascontiguousarray(np.asarray(arrival_us, dtype=np.float64))
    if arrivals.shape != (len(work),):
        raise ValueError("one arrival time per request")
    lat = np.zeros(len(work), dtype=np.float64)
    el = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.pscl_replay(server._h if server is not None else None, hs, n_codes, streams, arr,
                           arrivals.ctypes.data_as(dp), len(work), lat.ctypes.data_as(dp),
                           ctypes.byref(el)), "pscl_replay")
    return outs, lat, el.value


class Adaptive:
    """Adaptive decoding (see pscl_adaptive_create): `fast` (an L = 1 plan)
    first, `list` for the frames whose CRC fails.  The plans must outlive it."""

    def __init__(self, fast: Plan, list_plan: Plan, max_frames: int):
        self.fast, self.list = fast, list_plan
        h = ctypes.c_void_p(None)
        _check(lib.pscl_adaptive_create(fast._h, list_plan._h, max_frames, ctypes.byref(h)),
               "pscl_adaptive_create")
        self._h = h

    def decode(self, llr, u_hat=None, crc_ok=None, pm=None, n_list=None):
        """-> (u_hat, crc_ok, pm, n_list) with n_list a one-element int64 device
        tensor: the frames that were list-decoded."""
        import torch

        p = self.list
        want = {"f32": torch.float32, "i16": torch.int16, "i8": torch.int8}[p.dtype]
        if llr.dtype != want or llr.dim() != 2 or llr.shape[1] != p.N or not llr.is_contiguous():
            raise ValueError(f"llr must be a contiguous F x {p.N} {want} tensor")
        F = llr.shape[0]
        dev = llr.device
        if u_hat is None:
            u_hat = torch.empty((F, p.K), dtype=torch.uint8, device=dev)
        if crc_ok is None:
            crc_ok = torch.empty(F, dtype=torch.uint8, device=dev)
        if pm is None:
            pm = torch.empty(F, dtype=torch.float32 if p.dtype == "f32" else torch.int32,
                             device=dev)
        if n_list is None:
            n_list = torch.zeros(1, dtype=torch.int64, device=dev)
        _check(lib.pscl_adaptive_decode(self._h, llr.data_ptr(), F, u_hat.data_ptr(),
                                        crc_ok.data_ptr(), pm.data_ptr(), n_list.data_ptr(),
                                        _stream_handle(dev)), "pscl_adaptive_decode")
        return u_hat, crc_ok, pm, n_list

    def close(self):
        if getattr(self, "_h", None):
            lib.pscl_adaptive_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Generator:
    """Synthetic frames on the device (see pscl_generator_create)."""

    def __init__(self, N: int, K: int, frozen, crc_poly: int, crc_len: int, dtype: str = "f32"):
        import torch

        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        self.N, self.K, self.dtype = N, K, dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        fz = _mask(frozen)
        h = ctypes.c_void_p(None)
        _check(lib.pscl_generator_create(N, K, _u8p(fz), crc_poly, crc_len, DTYPES[dtype],
                                         ctypes.byref(h)), "pscl_generator_create")
        self._h = h

    def generate(self, F: int, ebn0_db: float, seed: int, first_frame: int = 0, llr=None,
                 info=None, want_info: bool = True):
        """-> (llr F x N in the dtype, info F x K uint8 or None)."""
        import torch

        want = {"f32": torch.float32, "i16": torch.int16, "i8": torch.int8}[self.dtype]
        if llr is None:
            llr = torch.empty((F, self.N), dtype=want, device=self.device)
        if info is None and want_info:
            info = torch.empty((F, self.K), dtype=torch.uint8, device=self.device)
        _check(lib.pscl_generate(self._h, seed, first_frame, F, ebn0_db, llr.data_ptr(),
                                 info.data_ptr() if info is not None else None,
                                 _stream_handle(self.device)), "pscl_generate")
        return llr, info

    def close(self):
        if getattr(self, "_h", None):
            lib.pscl_generator_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
