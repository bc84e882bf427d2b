"""MI355X-native closed-shell EOM-CCSD sigma / SA-PNO Davidson (arXiv:1802.06738).

The compute path is the HIP library libpnoeom.so (C ABI in include/pnoeom.h);
this package holds its ctypes binding.  PyTorch provides device memory and
streams only.
"""
from .pnoeom import (PnoEom, PnoEomError, load_library, library_path, host_eig, host_syev, gemm_bf16, gemm_bf16_time, FP64, FP32, BF16,
                     CANONICAL, PNO, LADDER_AUTO, LADDER_CACHED, LADDER_STREAMED, EXPORTED_SYMBOLS)

__all__ = ["PnoEom", "PnoEomError", "load_library", "library_path", "host_eig", "host_syev", "gemm_bf16", "gemm_bf16_time", "FP64", "FP32", "BF16",
           "CANONICAL", "PNO", "LADDER_AUTO", "LADDER_CACHED", "LADDER_STREAMED", "EXPORTED_SYMBOLS"]
