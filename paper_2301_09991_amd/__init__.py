"""MI355X (gfx950) ConvFEM space-angle multigrid solver for fixed-source Boltzmann transport.

The solver is the HIP library ``libctf.so`` (C-ABI in ``include/ctf.h``); ``ctf`` is its ctypes
binding, with PyTorch supplying device memory and streams.
"""
from . import ctf  # noqa: F401
