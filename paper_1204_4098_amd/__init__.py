"""MI355X-native pseudopotential lattice Boltzmann hot path (Li, Luo & Li, arXiv:1204.4098).

The compute lives in liblbm_hip.so (hand-written HIP for gfx950, C ABI in
include/lbm.h); `paper_1204_4098_amd.lbm` is its ctypes binding.  Import the
submodules explicitly: `from paper_1204_4098_amd import lbm`.
"""
