"""Frames and digests for the full-scale parity check of the (2048,1723)
CRC-32 L=32 workload at Eb/N0 3.5-4.5 dB (2^20 frames per point, float32
and int8 LLRs from the same channel output).

Shared by the oracle-side writer (tests/golden/make_c2_digests.py) and the
GPU test (tests/test_gpu_scale_parity.py).  It holds the seeded input recipe
and an output digest (a hash of the decoded bits, CRC flags and metric bits);
none of the decoder's arithmetic.
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np

import synth

N, K, R_CRC, DESIGN_DB, L = 2048, 1723, 32, 4.0, 32
POINTS = (3.5, 3.75, 4.0, 4.25, 4.5)
SUB = 16384  # frames per sub-chunk
SUBS = 64  # sub-chunks per point: 2^20 frames
DTYPES = ("f32", "i8")
DIGESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "c2_oracle_digests.jsonl")


def code():
    return synth.make_code(N, K, R_CRC, synth.CRC32_POLY, DESIGN_DB)


def frames(point_idx: int, sub: int):
    """Sub-chunk `sub` of point POINTS[point_idx]: (info bits, {dtype: llr})."""
    c = code()
    b = synth.make_batch(c, SUB, POINTS[point_idx], (21, point_idx, sub), "f32")
    return b.info, {"f32": b.llr, "i8": synth.quantize(b.llr_f32, "i8")}


def write_frames(args) -> dict:
    """Process-pool worker: writes sub-chunk `sub` of point POINTS[pi] as .npy
    files (information bits, float32 and int8 LLRs) into directory d and
    returns their paths."""
    pi, sub, d = args
    info, llr = frames(pi, sub)
    out = {}
    for name, arr in (("info", info), ("f32", llr["f32"]), ("i8", llr["i8"])):
        path = os.path.join(d, f"p{pi}_s{sub}_{name}.npy")
        np.save(path, arr)
        out[name] = path
    return out


def records(u: np.ndarray, ok: np.ndarray, pm: np.ndarray, dtype: str) -> np.ndarray:
    """One row of bytes per frame: packed u_hat bits, the CRC flag and the
    metric's 32 bits (float32 or int32)."""
    F = u.shape[0]
    if dtype == "f32":
        pmb = np.asarray(pm, dtype=np.float64).astype(np.float32).view(np.uint8).reshape(F, 4)
    else:
        pmb = np.asarray(pm).astype(np.int64).astype(np.int32).view(np.uint8).reshape(F, 4)
    return np.concatenate([np.packbits(np.asarray(u, np.uint8), axis=1),
                           np.asarray(ok, np.uint8).reshape(F, 1), pmb], axis=1)


def digest(u, ok, pm, dtype) -> str:
    return hashlib.blake2b(np.ascontiguousarray(records(u, ok, pm, dtype)).tobytes(),
                           digest_size=16).hexdigest()


def key(dtype: str, point_idx: int, sub: int) -> str:
    return f"{dtype}/{POINTS[point_idx]}/{sub}"


def load_digests(path: str = DIGESTS) -> dict:
    out = {}
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                line = line.strip()
                if line:
                    rec = json.loads(line)
                    out[rec["key"]] = rec
    return out
