"""MI355X-native Tensorized Pauli Decomposition (arXiv:2310.13421).

The compute path is libtpd.so (HIP kernels for gfx950 behind the C ABI in
include/tpd.h); ``paper_2310_13421_amd.tpd`` is its ctypes binding.
"""
