"""MI355X (gfx950) FFT -> filter -> IFFT: the radix-2 Cooley-Tukey transform of
"Construction of an algorithm in parallel for the Fast Fourier Transform"
(1/N-normalised DFT, eq. E2; 2D form eq. 5), its inverse, and the frequency
filter of the paper's Section 6, as hand-written HIP kernels behind a C-ABI
(include/fftmi.h).

The tensor-level functions import torch lazily; the ctypes binding itself
(``_binding``) needs only the built library.
"""
__all__ = ["fft", "ifft", "fft2", "ifft2", "transform", "fft2d_filter", "mask_grad", "filter_ragged",
           "fft_filter", "FFTFilterFn", "Plan", "FFTError"]

from ._binding import FFTError  # noqa: E402


def __getattr__(name):
    if name in ("fft", "ifft", "fft2", "ifft2", "transform", "fft2d_filter", "mask_grad", "filter_ragged",
                "Plan", "get_plan"):
        from . import api
        return getattr(api, name)
    if name in ("fft_filter", "FFTFilterFn"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
