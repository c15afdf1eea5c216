"""pscl: CRC-aided list decoding of polar codes with hand-written HIP kernels
for MI355X (gfx950), after "Fast List Decoders for Polar Codes".

The decoder is the C-ABI library ``_lib/libpscl.so`` (declared in
``include/pscl.h``); this package only marshals arguments to it.
"""

from ._binding import (  # noqa: F401
    DTYPES,
    Adaptive,
    Generator,
    LIB_PATH,
    Group,
    Job,
    LaunchCfg,
    MODE_SCL_LEAVES,
    MODE_TREE,
    OP_NAMES,
    Plan,
    PsclError,
    Server,
    ServerCfg,
    autotune,
    autotune_group,
    decode,
    decode_mixed,
    lib,
    replay,
    schedule,
)
