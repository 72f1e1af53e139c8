"""MI355X (gfx950) implementation of the quasi-regression Monte-Carlo backward
step (Gobet, Lopez-Salas, Vazquez, arXiv 2407.21084).

The method runs in libqrmc.so (HIP kernels behind the C ABI of
include/qrmc.h); ``paper_2407_21084_amd.qrmc`` is its ctypes binding.
"""
__all__ = ["qrmc"]
