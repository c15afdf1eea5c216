"""Polar encoding, BPSK over AWGN and LLR quantisation (Sec. VII-A: BPSK over
an AWGN channel with random codewords).

    s = 1 - 2x,   y = s + sigma * n,   n ~ N(0, 1),
    sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)),   LLR = 2 y / sigma^2  (float32).

Integer LLRs are formed from the float32 LLRs:
    int8  = clip(round_half_even(4 * LLR), -127, 127)
    int16 = clip(round_half_even(64 * LLR), -32767, 32767)
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .codes import PolarCode, crc_remainder

DTYPES = ("f32", "i16", "i8")
_NP = {"f32": np.float32, "i16": np.int16, "i8": np.int8}


def encode(u: np.ndarray) -> np.ndarray:
    """x = u F^{(x)n} over GF(2), natural order, for each row of u (F x N).

    Butterfly form: at span s = 1, 2, 4, ..., within every block of 2s the
    first half is XORed with the second half.
    """
    x = np.array(u, dtype=np.uint8, copy=True)
    F, N = x.shape
    s = 1
    while s < N:
        v = x.reshape(F, N // (2 * s), 2, s)
        v[:, :, 0, :] ^= v[:, :, 1, :]
        s *= 2
    return x


def quantize(llr: np.ndarray, dtype: str) -> np.ndarray:
    """Quantise float32 LLRs for the integer decoders (see module doc)."""
    if dtype == "f32":
        return np.ascontiguousarray(llr, dtype=np.float32)
    if dtype == "i8":
        q = np.clip(np.rint(4.0 * llr.astype(np.float64)), -127, 127)
        return q.astype(np.int8)
    if dtype == "i16":
        q = np.clip(np.rint(64.0 * llr.astype(np.float64)), -32767, 32767)
        return q.astype(np.int16)
    raise ValueError(f"unknown dtype {dtype!r}")


@dataclass
class Batch:
    """One seeded batch of frames."""

    code: PolarCode
    info: np.ndarray  # F x K uint8: payload then CRC, the expected decoder output
    x: np.ndarray  # F x N uint8 transmitted codewords
    llr_f32: np.ndarray  # F x N float32
    llr: np.ndarray  # F x N in the requested dtype
    dtype: str
    ebn0_db: float | None

    @property
    def F(self) -> int:
        return self.info.shape[0]


def make_batch(code: PolarCode, F: int, ebn0_db: float | None, seed, dtype: str = "f32") -> Batch:
    """F frames of uniform random payload, CRC appended, encoded, sent over
    BPSK-AWGN at ebn0_db (None = noiseless, LLR = 2 s / sigma^2 at a nominal
    4 dB scale so magnitudes are realistic), then quantised to dtype.

    seed: anything numpy.random.SeedSequence accepts (int or tuple of ints).
    """
    if dtype not in DTYPES:
        raise ValueError(f"unknown dtype {dtype!r}")
    ss = np.random.SeedSequence(seed if not isinstance(seed, tuple) else list(seed))
    rng = np.random.Generator(np.random.PCG64(ss))
    N, K, r = code.N, code.K, code.r
    payload = rng.integers(0, 2, size=(F, K - r), dtype=np.uint8)
    crc = crc_remainder(payload, code.poly, r) if r else np.zeros((F, 0), np.uint8)
    info = np.concatenate([payload, crc], axis=1)
    u = np.zeros((F, N), dtype=np.uint8)
    u[:, code.info_pos] = info
    x = encode(u)
    s = 1.0 - 2.0 * x.astype(np.float64)
    R = code.rate
    snr = 4.0 if ebn0_db is None else ebn0_db
    sigma2 = 1.0 / (2.0 * R * 10.0 ** (snr / 10.0))
    if ebn0_db is None:
        y = s
    else:
        y = s + np.sqrt(sigma2) * rng.standard_normal(size=(F, N))
    llr_f32 = (2.0 * y / sigma2).astype(np.float32)
    return Batch(code=code, info=info, x=x, llr_f32=llr_f32, llr=quantize(llr_f32, dtype),
                 dtype=dtype, ebn0_db=ebn0_db)
