"""tsk: time-stepper Arnoldi for linear stability analysis on AMD MI355X (gfx950).

Method: Loiseau, Bucci, Cherubini & Robinet, arXiv:1804.03859 -- eigenvalues of
the exponential propagator exp(A T) by Arnoldi, each matvec a time integration.
The computation lives in the HIP library libtsk.so (csrc/, C ABI in
include/tsk.h); ``tsk`` is its ctypes binding.
"""
from . import tsk  # noqa: F401
from .tsk import load  # noqa: F401
