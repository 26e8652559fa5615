"""MI355X-native Monte-Carlo shot pipeline for distributed transversal QEC operations.

The compute path is libtmcs.so (hand-written HIP kernels for gfx950 behind the
C ABI in include/tmcs.h); ``paper_2504_05611_amd.tmcs`` is its ctypes binding.
"""
