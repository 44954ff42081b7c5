"""HIF-preconditioned Crank-Nicolson solves on AMD MI355X (gfx950).

The compute path is the HIP library libhifcn.so (C ABI in include/hifcn.h); ``hifcn`` is its
ctypes binding.  Build with ``python -m paper_2004_05566_amd.build``.
"""
