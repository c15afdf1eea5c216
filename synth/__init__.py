"""Seeded synthetic workloads for polar list decoding.

This package is the transmitter and channel side of the link used to feed
decoders: code construction (frozen set), CRC attachment, polar encoding,
BPSK over AWGN and LLR quantisation.  It holds no decoder arithmetic, and it
is shared by the tests, the benchmark and the oracle-driven checks alike: the
decoder under test and the oracle receive exactly the same bytes.
"""

from .codes import (  # noqa: F401
    CRC8_POLY,
    CRC32_POLY,
    PolarCode,
    bhattacharyya_frozen,
    crc_remainder,
    make_code,
)
from .channel import (  # noqa: F401
    Batch,
    encode,
    make_batch,
    quantize,
)
