"""FP64 CPU oracle for the FFT -> filter -> IFFT path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library: the arithmetic lives in
``oracle_fft.c`` (plain C, double precision), loaded here through ctypes, and
the complexity model of the paper's Section 4 lives in ``complexity.py``.

Conventions (paper, Sections 2, 3 and 5):
  * 1D forward, eq. (E2):   H[k] = (1/N) sum_j f[j] e^{-2 pi i kj/N}
  * 1D inverse, eq. (E3):   f[j] = sum_k c_k e^{+2 pi i jk/N}          (unscaled)
  * 2D forward, eq. (5):    F[u,v] = (1/N) sum_x sum_y f[x,y] e^{-2 pi i (ux/N+vy/M)}
  * 2D inverse (2D-IDFT):   f[x,y] = (1/M) sum_u sum_v F[u,v] e^{+2 pi i (ux/N+vy/M)}
Arrays are row-major: x (length N) is the row index, y (length M) runs along
a row.  Inputs are promoted to complex128 / float64 before the call.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    sig = {
        "orc_dft_direct": [_i64, _dp, _dp, ctypes.c_int, ctypes.c_double],
        "orc_tree_partial": [_i64, _dp, _dp, ctypes.c_int],
        "orc_fft_fwd": [_i64, _i64, _dp, _dp],
        "orc_fft_inv": [_i64, _i64, _dp, _dp],
        "orc_fft_batch": [_i64, _i64, _dp, _dp, ctypes.c_int, ctypes.c_int],
        "orc_fft2_fwd": [_i64, _i64, _i64, _dp, _dp, ctypes.c_int],
        "orc_fft2_inv": [_i64, _i64, _i64, _dp, _dp, ctypes.c_int],
        "orc_filter2": [_i64, _i64, _i64, _dp, _dp, _dp, ctypes.c_int],
        "orc_mask_gaussian": [_i64, _i64, ctypes.c_double, _dp],
        "orc_mask_butterworth": [_i64, _i64, ctypes.c_double, ctypes.c_int, _dp],
        "orc_mask_disc": [_i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp],
        "orc_loss_grad": [_i64, _i64, _i64, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def default_threads() -> int:
    """Host threads the oracle uses unless told otherwise."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


class OracleError(RuntimeError):
    pass


def _chk(code: int, what: str):
    if code != 0:
        raise OracleError("%s failed with status %d" % (what, code))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


# --------------------------------------------------------------------------- 1D
def dft_direct(f, sign: int = -1, scale: float = None) -> np.ndarray:
    """Definition (eq. E2 with sign -1 and scale 1/N by default): O(N^2) sum."""
    f = _c128(f).reshape(-1)
    n = f.shape[0]
    if scale is None:
        scale = 1.0 / n if sign < 0 else 1.0
    out = np.empty_like(f)
    _chk(_load().orc_dft_direct(n, _ptr(f.view(np.float64)), _ptr(out.view(np.float64)), int(sign), float(scale)),
         "orc_dft_direct")
    return out


def tree_partial(f, levels: int) -> np.ndarray:
    """Array contents after `levels` levels of the Section-2 tree (unscaled)."""
    f = _c128(f).reshape(-1)
    out = np.empty_like(f)
    _chk(_load().orc_tree_partial(f.shape[0], _ptr(f.view(np.float64)), _ptr(out.view(np.float64)), int(levels)),
         "orc_tree_partial")
    return out


def fft(f, threads: int = 1) -> np.ndarray:
    """Forward 1D transform with 1/N (eq. E2) along the last axis."""
    f = _c128(f)
    n = f.shape[-1]
    out = np.empty_like(f)
    batch = f.size // n if n else 0
    _chk(_load().orc_fft_batch(n, batch, _ptr(f.view(np.float64)), _ptr(out.view(np.float64)), 0, int(threads)),
         "orc_fft_batch")
    return out


def ifft(c, threads: int = 1) -> np.ndarray:
    """Unscaled inverse (eq. E3) along the last axis, by the Section-3 route."""
    c = _c128(c)
    n = c.shape[-1]
    out = np.empty_like(c)
    batch = c.size // n if n else 0
    _chk(_load().orc_fft_batch(n, batch, _ptr(c.view(np.float64)), _ptr(out.view(np.float64)), 1, int(threads)),
         "orc_fft_batch")
    return out


# --------------------------------------------------------------------------- 2D
def _batch2(a):
    N, M = a.shape[-2], a.shape[-1]
    return N, M, (a.size // (N * M)) if N * M else 0


def fft2(f, threads: int = None) -> np.ndarray:
    """eq. (5) over the last two axes: rows -> x M -> columns, factor 1/N."""
    f = _c128(f)
    N, M, B = _batch2(f)
    out = np.empty_like(f)
    _chk(_load().orc_fft2_fwd(N, M, B, _ptr(f.view(np.float64)), _ptr(out.view(np.float64)),
                              threads or default_threads()), "orc_fft2_fwd")
    return out


def ifft2(F, threads: int = None) -> np.ndarray:
    """2D-IDFT over the last two axes: unscaled inverse on columns and rows, then 1/M."""
    F = _c128(F)
    N, M, B = _batch2(F)
    out = np.empty_like(F)
    _chk(_load().orc_fft2_inv(N, M, B, _ptr(F.view(np.float64)), _ptr(out.view(np.float64)),
                              threads or default_threads()), "orc_fft2_inv")
    return out


def filter2(f, mask, threads: int = None) -> np.ndarray:
    """2D-IDFT(mask * 2D-DFT(f)) over the last two axes; mask is real [N][M]."""
    f = _c128(f)
    N, M, B = _batch2(f)
    mask = _f64(mask)
    if mask.shape != (N, M):
        raise ValueError("mask shape %s != (%d, %d)" % (mask.shape, N, M))
    out = np.empty_like(f)
    _chk(_load().orc_filter2(N, M, B, _ptr(f.view(np.float64)), _ptr(mask), _ptr(out.view(np.float64)),
                             threads or default_threads()), "orc_filter2")
    return out


# ------------------------------------------------- Section 6 padding/cropping
def next_pow2(n: int) -> int:
    """Smallest power of two >= n (Section 6 pads each axis to such a length)."""
    p = 1
    while p < n:
        p <<= 1
    return p


def pad2(f) -> np.ndarray:
    """Zero padding of the last two axes (n0 x m0) to the next powers of two,
    the added rows at the bottom and columns at the right (Section 6)."""
    f = np.asarray(f)
    n0, m0 = f.shape[-2], f.shape[-1]
    widths = [(0, 0)] * (f.ndim - 2) + [(0, next_pow2(n0) - n0), (0, next_pow2(m0) - m0)]
    return np.pad(f, widths)


def filter2_padded(f, mask, threads: int = None) -> np.ndarray:
    """Section 6 on an image of any size: pad to powers of two, filter with the
    real mask given for the padded N x M grid, crop back to n0 x m0."""
    f = np.asarray(f)
    n0, m0 = f.shape[-2], f.shape[-1]
    return filter2(pad2(f), mask, threads)[..., :n0, :m0]


def spectrum_padded(f, threads: int = None) -> np.ndarray:
    """|2D-DFT| (eq. 5) of the zero-padded image, unshifted (Section 6's spectrum)."""
    return np.abs(fft2(pad2(f), threads))


# ------------------------------------------------------------------------ masks
def mask_gaussian(N: int, M: int, sigma_f: float) -> np.ndarray:
    """exp(-r^2 / (2 sigma_f^2)), r in cycles/pixel on the fftfreq grid."""
    out = np.empty((N, M), np.float64)
    _chk(_load().orc_mask_gaussian(N, M, float(sigma_f), _ptr(out)), "orc_mask_gaussian")
    return out


def mask_butterworth(N: int, M: int, cutoff: float, order: int) -> np.ndarray:
    """1 / (1 + (r / cutoff)^(2 order)), r in cycles/pixel on the fftfreq grid."""
    out = np.empty((N, M), np.float64)
    _chk(_load().orc_mask_butterworth(N, M, float(cutoff), int(order), _ptr(out)), "orc_mask_butterworth")
    return out


def mask_disc(N: int, M: int, b: float, c1: float = None, c2: float = None) -> np.ndarray:
    """eq. (filtro): 0 inside the disc of radius b about (c1, c2), 1 outside."""
    c1 = N / 2.0 if c1 is None else c1
    c2 = M / 2.0 if c2 is None else c2
    out = np.empty((N, M), np.float64)
    _chk(_load().orc_mask_disc(N, M, float(b), float(c1), float(c2), _ptr(out)), "orc_mask_disc")
    return out


# ------------------------------------------------------------- learnable mask
def loss_grad(noisy, clean, mask, threads: int = None):
    """(y, L, dL/dmask) for y = 2D-IDFT(mask * 2D-DFT(noisy)), L = mean |y - clean|^2.

    noisy: [B][N][M] (real or complex), clean: [B][N][M] real, mask: [N][M] real.
    """
    x = _c128(noisy)
    N, M, B = _batch2(x)
    c = _f64(clean).reshape(B, N, M)
    m = _f64(mask)
    if m.shape != (N, M):
        raise ValueError("mask shape %s != (%d, %d)" % (m.shape, N, M))
    y = np.empty_like(x)
    g = np.empty((N, M), np.float64)
    loss = ctypes.c_double(0.0)
    _chk(_load().orc_loss_grad(N, M, B, _ptr(x.view(np.float64)), _ptr(c), _ptr(m), _ptr(y.view(np.float64)),
                               ctypes.pointer(loss), _ptr(g), threads or default_threads()), "orc_loss_grad")
    return y, loss.value, g
