"""MI355X (gfx950) implementation of the compact FAM scheme with single-step OE.

The compute path is the HIP library libfam.so (C ABI in include/fam.h); the
Python module ``fam`` is a thin ctypes binding and ``autograd`` wraps the
hand-written adjoint as a torch.autograd.Function.
"""
from .fam import Fam, FamConfig, FamError, NonPhysicalError, load_library  # noqa: F401
