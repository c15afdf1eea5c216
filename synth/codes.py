"""Polar code construction and CRC attachment (transmitter side).

The paper does not say how its frozen sets were built; the workloads use the
Bhattacharyya-parameter construction at a design Eb/N0, with natural (not
bit-reversed) index order, matching the (8, 4) example of Fig. 1 (frozen
positions {0, 1, 2, 4}).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CRC8_POLY = 0x07
CRC32_POLY = 0x04C11DB7


def bhattacharyya_frozen(N: int, K: int, design_ebn0_db: float, rate: float | None = None) -> np.ndarray:
    """Frozen mask (1 = frozen) keeping the K positions of smallest
    Bhattacharyya parameter.

    The channel parameter is z0 = exp(-R * Eb/N0) for BPSK-AWGN with rate R
    (the payload rate (K - r) / N by default of the callers).  Position i is
    reached from the channel by one polarising step per bit of i, most
    significant bit first: a 0 bit takes the degraded channel, z -> 2z - z^2,
    a 1 bit the upgraded one, z -> z^2.  Computed in the log domain.  Equal
    parameters are broken by freezing the lower index first; a tie across the
    frozen/unfrozen boundary raises.
    """
    if N < 2 or N & (N - 1):
        raise ValueError("N must be a power of two >= 2")
    if not 0 < K <= N:
        raise ValueError("need 0 < K <= N")
    n = N.bit_length() - 1
    R = (K / N) if rate is None else rate
    lz0 = -R * 10.0 ** (design_ebn0_db / 10.0)
    lz = np.full(N, lz0, dtype=np.float64)
    idx = np.arange(N)
    for b in range(n - 1, -1, -1):
        bit = (idx >> b) & 1
        up = 2.0 * lz
        # ln(2z - z^2) = ln z + ln(2 - z)
        down = lz + np.log(2.0 - np.exp(lz))
        lz = np.where(bit == 1, up, down)
    # Largest parameter first; equal values: lower index first.
    order = sorted(range(N), key=lambda i: (-lz[i], i))
    nf = N - K
    if 0 < nf < N and lz[order[nf - 1]] == lz[order[nf]]:
        raise ValueError("Bhattacharyya tie across the frozen/unfrozen boundary")
    frozen = np.zeros(N, dtype=np.uint8)
    frozen[order[:nf]] = 1
    return frozen


def _crc_matrix(nbits: int, poly: int, r: int) -> np.ndarray:
    """GF(2) matrix M (nbits x r) with remainder(bits) = bits @ M mod 2.

    Row i is x^(nbits - 1 - i + r) mod g(x), g(x) = x^r + poly, written
    MSB-first: the last payload bit contributes x^r mod g = poly, and each
    earlier bit is one more multiplication by x.
    """
    mask = (1 << r) - 1
    top = 1 << (r - 1)
    rows = np.zeros((nbits, r), dtype=np.uint8)
    v = poly & mask  # x^r mod g
    for i in range(nbits - 1, -1, -1):
        for t in range(r):
            rows[i, t] = (v >> (r - 1 - t)) & 1
        # multiply by x modulo g
        carry = v & top
        v = (v << 1) & mask
        if carry:
            v ^= poly & mask
    return rows


def crc_remainder(bits: np.ndarray, poly: int, r: int) -> np.ndarray:
    """CRC of each row of bits (F x nbits, values 0/1): generator x^r + poly,
    register initialised to zero, bits fed MSB-first, no reflection, no final
    XOR.  Returns F x r bits, most significant first."""
    bits = np.asarray(bits, dtype=np.uint8)
    if bits.ndim == 1:
        return crc_remainder(bits[None, :], poly, r)[0]
    if r == 0:
        return np.zeros((bits.shape[0], 0), dtype=np.uint8)
    M = _crc_matrix(bits.shape[1], poly, r).astype(np.float32)
    # exact: counts stay far below 2^24
    acc = bits.astype(np.float32) @ M
    return (acc.astype(np.int64) & 1).astype(np.uint8)


@dataclass
class PolarCode:
    """A polar-CRC code: K unfrozen positions carry K - r payload bits followed
    by r CRC bits (the CRC is counted inside K)."""

    N: int
    K: int
    r: int
    poly: int
    design_ebn0_db: float
    frozen: np.ndarray = field(repr=False)

    @property
    def info_pos(self) -> np.ndarray:
        return np.flatnonzero(self.frozen == 0)

    @property
    def payload(self) -> int:
        return self.K - self.r

    @property
    def rate(self) -> float:
        """Payload rate used for the construction and the channel."""
        return self.payload / self.N


def make_code(N: int, K: int, r: int, poly: int, design_ebn0_db: float) -> PolarCode:
    """Bhattacharyya construction at the design point, payload rate (K - r)/N."""
    frozen = bhattacharyya_frozen(N, K, design_ebn0_db, rate=(K - r) / N)
    return PolarCode(N=N, K=K, r=r, poly=poly, design_ebn0_db=design_ebn0_db, frozen=frozen)
