"""obfft: the Ozaki-Bailey full-FP64 complex 3-D FFT on AMD MI355X (gfx950).

The transform, its adjoint/inverse, an FP32-target variant and a native FP64
comparator all run in the HIP kernels of libobfft.so (built in-tree by
``paper_2606_23698_amd.build.build()``); the Python layer only marshals
arguments.  Importing the package does not load the library; the first call
does, and fails loudly if it was not built.
"""
from ._lib import ObfftError  # noqa: F401

__all__ = ["api", "autograd", "inputs", "ObfftError"]
