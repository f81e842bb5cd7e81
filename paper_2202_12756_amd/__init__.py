"""MI355X-native slab-decomposed 3D real FFT (one GPU's share).

The transform of Verma et al., "Scalable Multi-node Fast Fourier Transform on
GPUs": section 2 defines the unnormalized forward/inverse 3D DFT of a real
field with the half spectrum stored along z; section 3 gives the slab
algorithm (2D R2C over yz on each local plane, transpose into all-to-all
chunks, strided 1D C2C along x; reversed for the inverse).  Everything runs
in hand-written HIP kernels for gfx950 behind the C ABI of include/gfft.h
(``libgfft.so``); this package is its Python binding.
"""
from ._lib import GfftError, load  # noqa: F401
from .fft import Plan, PencilPlan, device_copy  # noqa: F401
from .autograd import RFFT3, IRFFT3, rfft3, irfft3  # noqa: F401

__all__ = ["Plan", "PencilPlan", "device_copy", "GfftError", "load", "RFFT3", "IRFFT3", "rfft3", "irfft3"]
