"""MI355X (gfx950) CT-AUX submatrix-update library: Python binding.

The compute path is the HIP library `lib/libctaux_hip.so` (C ABI in
include/ctaux.h); this package only marshals arguments to it.
"""

from .ctaux import (CTAUX_BF16X3, CTAUX_FP32, CTAUX_FP64, CtauxBatch, CtauxError, Options,  # noqa: F401
                    load_library)
