"""MI355X-native MCQSG hot path: Metropolis + parallel tempering over the
Trotter-Suzuki (2+1)-D lattice of the 2D +-J quantum Ising spin glass.

The compute lives in libqsg.so (HIP kernels for gfx950 behind the C ABI of
include/qsg.h); `paper_2402_03920_amd.qsg` is its ctypes binding.
"""
__all__ = ["qsg"]
