"""CT-AUX oracle package (TEST INFRASTRUCTURE ONLY).

A plain FP64 CPU CT-AUX walk with rank-1 updates (C library
`libctaux_oracle.so`) and a ctypes wrapper.  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import this package; the GPU
library never links or calls it.
"""

from .oracle import OracleChain, build_oracle, philox4x32_10, draws, gamma_of  # noqa: F401
