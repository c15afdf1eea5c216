"""Counter-based frames: the same transmitter and channel as ``make_batch``,
but with every random number drawn from Philox4x32-10 (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) keyed by the
seed and counted by frame index, so that any frame can be produced on its
own, on the host or on the device.  The device generator follows the same
definition; this module is its host counterpart.

Frame f under seed S (key k0 = S mod 2^32, k1 = S div 2^32):

* payload bit j (0 <= j < K - r) is bit j mod 32 of word (j div 32) mod 4 of
  Philox((j div 128, f mod 2^32, f div 2^32, 1));
* block i of Philox((i, f mod 2^32, f div 2^32, 2)), words (w0, w1, w2, w3),
  gives the noise of channel uses 4i .. 4i+3 by Box-Muller:
  u_k = (floor(w_k / 2^9) + 1/2) / 2^23,  rad_a = sqrt(-2 ln u_0),
  rad_b = sqrt(-2 ln u_2),  phi_a = 2 pi u_1,  phi_b = 2 pi u_3,
  n = (rad_a cos phi_a, rad_a sin phi_a, rad_b cos phi_b, rad_b sin phi_b);
* LLR = scale * (s + sigma * n) in float32 steps (sigma and scale = 2 /
  sigma^2 rounded to float32 once), then quantised as in ``quantize``.

The float32 steps mirror the device's, so LLRs agree with the device's to a
few units in the last place (its log, sin and cos round differently).
"""

from __future__ import annotations

import numpy as np

from .channel import Batch, encode, quantize
from .codes import PolarCode, crc_remainder

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_LO = np.uint64(0xFFFFFFFF)

DOM_PAYLOAD, DOM_NOISE = 1, 2


def philox4x32_10(ctr: np.ndarray, key: tuple[int, int]) -> np.ndarray:
    """Philox4x32 with 10 rounds on each row of ctr (... x 4, uint32) under
    key (k0, k1).  Each round multiplies words 0 and 2 by the two round
    constants, then mixes the halves of the products with words 1 and 3 and
    the round key; the key grows by the two Weyl constants between rounds."""
    c = [np.asarray(ctr, dtype=np.uint32)[..., i].astype(np.uint64) for i in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & _LO,
             (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & _LO]
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([v.astype(np.uint32) for v in c], axis=-1)


def _counters(frames: np.ndarray, n_blocks: int, domain: int) -> np.ndarray:
    F = frames.shape[0]
    ctr = np.empty((F, n_blocks, 4), dtype=np.uint32)
    ctr[:, :, 0] = np.arange(n_blocks, dtype=np.uint32)[None, :]
    ctr[:, :, 1] = (frames & 0xFFFFFFFF).astype(np.uint32)[:, None]
    ctr[:, :, 2] = (frames >> 32).astype(np.uint32)[:, None]
    ctr[:, :, 3] = domain
    return ctr


def payload_bits(frames: np.ndarray, P: int, seed: int) -> np.ndarray:
    """F x P payload bits of the given frame indices."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    words = philox4x32_10(_counters(frames, (P + 127) // 128, DOM_PAYLOAD), key)
    words = words.reshape(frames.shape[0], -1)  # word w = block w // 4, lane w % 4
    bits = (words[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1
    return bits.reshape(frames.shape[0], -1)[:, :P].astype(np.uint8)


def normals(frames: np.ndarray, N: int, seed: int) -> np.ndarray:
    """F x N standard normals (float32) of the given frame indices."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    w = philox4x32_10(_counters(frames, (N + 3) // 4, DOM_NOISE), key)
    u = ((w >> 9).astype(np.float32) + np.float32(0.5)) * np.float32(2.0 ** -23)
    rad = np.sqrt(-2.0 * np.log(u[..., [0, 2]].astype(np.float64))).astype(np.float32)
    phi = (np.float32(2.0 * np.pi) * u[..., [1, 3]]).astype(np.float64)
    c, s = np.cos(phi).astype(np.float32), np.sin(phi).astype(np.float32)
    n = np.stack([rad[..., 0] * c[..., 0], rad[..., 0] * s[..., 0],
                  rad[..., 1] * c[..., 1], rad[..., 1] * s[..., 1]], axis=-1)
    return n.reshape(frames.shape[0], -1)[:, :N]


def channel_params(code: PolarCode, ebn0_db: float) -> tuple[np.float32, np.float32]:
    """(sigma, scale = 2 / sigma^2) as float32, from sigma^2 = 1 / (2 R 10^(EbN0/10))."""
    sigma2 = 1.0 / (2.0 * code.rate * 10.0 ** (ebn0_db / 10.0))
    return np.float32(np.sqrt(sigma2)), np.float32(2.0 / sigma2)


def philox_batch(code: PolarCode, F: int, ebn0_db: float, seed: int, first: int = 0,
                 dtype: str = "f32") -> Batch:
    """Frames first .. first + F - 1 under seed (a 64-bit integer)."""
    frames = np.arange(first, first + F, dtype=np.uint64)
    P = code.payload
    payload = payload_bits(frames, P, seed)
    crc = crc_remainder(payload, code.poly, code.r) if code.r else np.zeros((F, 0), np.uint8)
    info = np.concatenate([payload, crc], axis=1)
    u = np.zeros((F, code.N), dtype=np.uint8)
    u[:, code.info_pos] = info
    x = encode(u)
    sigma, scale = channel_params(code, ebn0_db)
    s = np.float32(1.0) - np.float32(2.0) * x.astype(np.float32)
    llr_f32 = scale * (s + sigma * normals(frames, code.N, seed))
    return Batch(code=code, info=info, x=x, llr_f32=llr_f32, llr=quantize(llr_f32, dtype),
                 dtype=dtype, ebn0_db=ebn0_db)
