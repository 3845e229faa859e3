"""MI355X-native time-domain preconditioner for the Helmholtz equation.

The compute path is the HIP library ``libtdp.so`` behind the C ABI declared in
``include/tdp.h``; ``paper_2006_16861_amd.tdp`` is its thin ctypes binding and
raises if the library is missing (there is no CPU fallback).
"""
__all__ = ["inputs", "tdp"]
