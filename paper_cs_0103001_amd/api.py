"""Tensor-level wrappers over the C-ABI.  PyTorch supplies device memory and the
current HIP stream; every step of every transform runs in libfftmi's kernels.

Conventions (the paper's, selected by norm="paper"): 1D forward carries 1/N
(eq. E2), 1D inverse is unscaled (eq. E3); 2D forward carries 1/N with N the
row count (eq. 5) and the 2D inverse 1/M (2D-IDFT).  norm="numpy" gives an
unscaled forward and a 1/(number of points) inverse.
"""
import ctypes
import threading

import torch

from . import _binding as B

_NORM = {"paper": B.FFT_NORM_PAPER, "numpy": B.FFT_NORM_NUMPY}


class Plan:
    """Owns one fft_plan_t (created on the tensor's device)."""

    def __init__(self, rank, dims, batch, flags=0, device=None, ragged_sizes=None, padded=False):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device.index)
        with torch.cuda.device(self.device):
            if ragged_sizes is not None:
                self.h = B.fft_plan_ragged(ragged_sizes, flags)
            elif padded:
                self.h = B.fft_plan_padded(dims, batch, flags)
            else:
                self.h = B.fft_plan(rank, dims, batch, flags)
        self.rank, self.dims, self.batch, self.flags = rank, tuple(dims), batch, flags
        self.workspace_bytes = B.fft_workspace_size(self.h)
        self.spectrum_bytes = B.fft_spectrum_size(self.h) if rank == 2 and ragged_sizes is None else 0
        self.padded = padded

    def workspace(self):
        n = max(self.workspace_bytes, 1)
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B is not None and getattr(B, "_lib", None) is not None:
            try:
                B.fft_plan_destroy(h)
            except Exception:
                pass
            self.h = None


_cache = {}
_cache_lock = threading.Lock()


def get_plan(rank, dims, batch, flags, device, ragged_sizes=None, padded=False):
    key = (rank, tuple(dims), int(batch), int(flags), device.index,
           tuple(ragged_sizes) if ragged_sizes is not None else None, bool(padded))
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = Plan(rank, dims, batch, flags, device, ragged_sizes, padded)
            _cache[key] = p
    return p


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _prep(x, allow_real=True):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if x.dtype == torch.complex64:
        return x.contiguous(), B.FFT_IN_C64
    if x.dtype == torch.float32 and allow_real:
        return x.contiguous(), B.FFT_IN_REAL_F32
    raise TypeError("expected complex64%s, got %s" % (" or float32" if allow_real else "", x.dtype))


def transform(x, rank, direction, norm="paper", real_output=False):
    """One batched transform over the last `rank` axes (fft_exec)."""
    x, fin = _prep(x)
    if x.dim() < rank:
        raise ValueError("tensor has fewer than %d dims" % rank)
    dims = tuple(x.shape[-rank:])
    n = 1
    for d in dims:
        n *= d
    batch = x.numel() // n if n else 0
    flags = fin | _NORM[norm] | (B.FFT_OUT_REAL_F32 if real_output else 0)
    plan = get_plan(rank, dims, batch, flags, x.device)
    out = torch.empty(x.shape, dtype=torch.float32 if real_output else torch.complex64, device=x.device)
    if batch == 0:
        return out
    ws = plan.workspace()
    B.fft_exec(plan.h, _ptr(x), _ptr(out), _ptr(ws), direction, _stream(x.device))
    return out


def fft(x, norm="paper"):
    """eq. E2 along the last axis: H[k] = (1/N) sum_j f[j] e^{-2 pi i kj/N}."""
    return transform(x, 1, B.FFT_FORWARD, norm)


def ifft(c, norm="paper", real_output=False):
    """eq. E3 along the last axis: f[j] = sum_k c[k] e^{+2 pi i jk/N}."""
    return transform(c, 1, B.FFT_INVERSE, norm, real_output)


def fft2(x, norm="paper"):
    """eq. 5 over the last two axes (factor 1/N, N rows)."""
    return transform(x, 2, B.FFT_FORWARD, norm)


def ifft2(F, norm="paper", real_output=False):
    """2D-IDFT over the last two axes (factor 1/M, M columns)."""
    return transform(F, 2, B.FFT_INVERSE, norm, real_output)


def _mask_struct(mask, N, M, device):
    """(fft_mask, keepalive) from a dict spec, a float32 [N][M] tensor or None."""
    if mask is None:
        return B.make_mask("none"), None
    if isinstance(mask, torch.Tensor):
        if mask.dtype != torch.float32 or tuple(mask.shape) != (N, M) or mask.device != device:
            raise ValueError("tensor mask must be float32 [%d, %d] on %s" % (N, M, device))
        m = mask.contiguous()
        return B.make_mask("tensor", data_ptr=m.data_ptr()), m
    spec = dict(mask)
    kind = spec.pop("kind")
    if kind == "disc":
        spec.setdefault("c1", N / 2.0)
        spec.setdefault("c2", M / 2.0)
    return B.make_mask(kind, **spec), None


def fft2d_filter(x, mask, norm="paper", real_output=False, spectrum=False, real_even=False):
    """Section 6: 2D-IDFT(H . 2D-DFT(x)) over the last two axes of x.

    mask: dict(kind="gaussian", sigma_f=...), dict(kind="butterworth",
    cutoff=..., order=...), dict(kind="disc", b=..., c1=..., c2=...), a float32
    [N][M] tensor, or None.  With spectrum=True also returns the saved forward
    spectrum (internal layout) used by mask_grad.  real_even=True takes the
    half-spectrum path (FFT_REAL_EVEN): float32 input and a mask even in
    frequency; the output is then real (its imaginary parts are zero).
    """
    x, fin = _prep(x)
    N, M = x.shape[-2], x.shape[-1]
    batch = x.numel() // (N * M) if N * M else 0
    flags = fin | _NORM[norm] | (B.FFT_OUT_REAL_F32 if real_output else 0)
    if real_even:
        if fin != B.FFT_IN_REAL_F32:
            raise TypeError("real_even needs float32 input")
        flags |= B.FFT_REAL_EVEN
    padded = not (_pow2(N) and _pow2(M))
    if padded and spectrum:
        raise ValueError("the saved spectrum needs power-of-two sides")
    plan = get_plan(2, (N, M), batch, flags, x.device, padded=padded)
    out = torch.empty(x.shape, dtype=torch.float32 if real_output else torch.complex64, device=x.device)
    mk, keep = _mask_struct(mask, _next_pow2(N), _next_pow2(M), x.device)
    ws = plan.workspace()
    st = _stream(x.device)
    if spectrum:
        spec = torch.empty(max(plan.spectrum_bytes, 1), dtype=torch.uint8, device=x.device)
        if batch:
            B.fft2d_filter_save(plan.h, _ptr(x), _ptr(out), mk, _ptr(spec), _ptr(ws), st)
        return out, spec
    if batch:
        B.fft2d_filter(plan.h, _ptr(x), _ptr(out), mk, _ptr(ws), st)
    del keep
    return out


def _pow2(n):
    return n > 0 and (n & (n - 1)) == 0


def _next_pow2(n):
    p = 1
    while p < n:
        p <<= 1
    return p


def spectrum(x, norm="paper"):
    """|2D-DFT| (eq. 5) over the last two axes, zero-padded to powers of two
    as in Section 6: float32 [..., N, M] with N, M the padded sides, unshifted."""
    x, fin = _prep(x)
    n0, m0 = x.shape[-2], x.shape[-1]
    batch = x.numel() // (n0 * m0) if n0 * m0 else 0
    N, M = _next_pow2(n0), _next_pow2(m0)
    plan = get_plan(2, (n0, m0), batch, fin | _NORM[norm], x.device, padded=not (N == n0 and M == m0))
    out = torch.empty(tuple(x.shape[:-2]) + (N, M), dtype=torch.float32, device=x.device)
    if batch:
        ws = plan.workspace()
        B.fft2d_spectrum(plan.h, _ptr(x), _ptr(out), _ptr(ws), _stream(x.device))
    return out


def _check_images(x, what="x"):
    if not isinstance(x, torch.Tensor):
        raise TypeError("%s must be a tensor" % what)
    if x.dim() < 2 or x.shape[-2] < 1 or x.shape[-1] < 1:
        raise ValueError("%s must have at least two non-empty axes, got %s" % (what, tuple(x.shape)))


def _check_mask_tensor(mask, N, M, device):
    """A learnable mask: float32 [N][M] on the images' device."""
    if not isinstance(mask, torch.Tensor):
        raise TypeError("mask must be a tensor")
    if mask.dtype != torch.float32 or tuple(mask.shape) != (N, M):
        raise ValueError("mask must be float32 [%d, %d], got %s %s" % (N, M, mask.dtype, tuple(mask.shape)))
    if mask.device != device:
        raise ValueError("mask is on %s, the images on %s" % (mask.device, device))


def _check_spectrum(spectrum, plan, device):
    """A saved spectrum from fft2d_filter(spectrum=True) or filter_mse for this plan's shape."""
    if not isinstance(spectrum, torch.Tensor):
        raise TypeError("spectrum must be a tensor")
    if spectrum.device != device or not spectrum.is_contiguous():
        raise ValueError("spectrum must be a contiguous tensor on %s" % device)
    have = spectrum.numel() * spectrum.element_size()
    if have < plan.spectrum_bytes:
        raise ValueError("spectrum holds %d bytes, this batch's plan needs %d" % (have, plan.spectrum_bytes))


def mask_grad(grad_y, spectrum, norm="paper"):
    """sum_b Re(conj(X_b) . (2D-IDFT^H grad_y_b)) for a saved spectrum X."""
    _check_images(grad_y, "grad_y")
    g, _ = _prep(grad_y, allow_real=False)
    N, M = g.shape[-2], g.shape[-1]
    batch = g.numel() // (N * M)
    plan = get_plan(2, (N, M), batch, B.FFT_IN_C64 | _NORM[norm], g.device)
    _check_spectrum(spectrum, plan, g.device)
    out = torch.empty((N, M), dtype=torch.float32, device=g.device)
    ws = plan.workspace()
    B.fft2d_filter_mask_grad(plan.h, _ptr(g), _ptr(spectrum), _ptr(out), _ptr(ws), _stream(g.device))
    return out


def mse_grad(x, c, spectrum, mask, weight, norm="paper"):
    """weight * sum_b [Re(conj X_b . 2D-IDFT^H (x_b - c_b)) + (a_inv/a_fwd)(m - 1)|X_b|^2]:
    the mask gradient of (weight/2) sum |2D-IDFT(m . X) - c|^2; c=None means x is
    already the residual x - c."""
    _check_images(x)
    if c is not None and (not isinstance(c, torch.Tensor) or tuple(c.shape) != tuple(x.shape)):
        raise ValueError("c must have the shape of x %s" % (tuple(x.shape),))
    if c is not None and c.dtype != x.dtype:
        raise TypeError("c must have the dtype of x (%s)" % x.dtype)
    _check_mask_tensor(mask, x.shape[-2], x.shape[-1], x.device)
    r, fin = _prep(x)
    N, M = r.shape[-2], r.shape[-1]
    batch = r.numel() // (N * M)
    m = mask.contiguous()
    cc = None
    if c is not None:
        cc, _ = _prep(c)
    plan = get_plan(2, (N, M), batch, fin | _NORM[norm], r.device)
    _check_spectrum(spectrum, plan, r.device)
    out = torch.empty((N, M), dtype=torch.float32, device=r.device)
    ws = plan.workspace()
    B.fft2d_filter_mse_grad(plan.h, _ptr(r), _ptr(cc), _ptr(spectrum), _ptr(m), weight, _ptr(out), _ptr(ws),
                            _stream(r.device))
    return out


def filter_mse(x, c, mask, weight, norm="paper"):
    """(loss, spectrum): loss = weight * sum |2D-IDFT(m . 2D-DFT(x)) - c|^2 (a
    0-dim float32 tensor) for float32 x, c [..., N, M], and the saved spectrum."""
    _check_images(x)
    if not isinstance(c, torch.Tensor) or tuple(c.shape) != tuple(x.shape):
        raise ValueError("c must have the shape of x %s" % (tuple(x.shape),))
    if x.dtype != torch.float32 or c.dtype != torch.float32:
        raise TypeError("filter_mse takes float32 images")
    _check_mask_tensor(mask, x.shape[-2], x.shape[-1], x.device)
    if c.device != x.device:
        raise ValueError("c is on %s, x on %s" % (c.device, x.device))
    x, fin = _prep(x)
    c, _ = _prep(c)
    N, M = x.shape[-2], x.shape[-1]
    batch = x.numel() // (N * M)
    m = mask.contiguous()
    plan = get_plan(2, (N, M), batch, fin | _NORM[norm], x.device)
    spec = torch.empty(max(plan.spectrum_bytes, 1), dtype=torch.uint8, device=x.device)
    loss = torch.empty((), dtype=torch.float32, device=x.device)
    ws = plan.workspace()
    B.fft2d_filter_mse(plan.h, _ptr(x), _ptr(c), _ptr(m), weight, _ptr(spec), _ptr(loss), _ptr(ws),
                       _stream(x.device))
    return loss, spec


def filter_mse_spectral(x, c, mask, weight, norm="paper"):
    """(loss, state): loss = weight * sum |2D-IDFT(m . 2D-DFT(x)) - c|^2 evaluated
    in the frequency domain (no inverse transform), and the state that
    mse_spectral_grad reads.  Raises FFTError(FFT_ERR_UNSUPPORTED) for shapes
    the frequency-domain pass does not take (rows of more than 4096 points)."""
    _check_images(x)
    if not isinstance(c, torch.Tensor) or tuple(c.shape) != tuple(x.shape):
        raise ValueError("c must have the shape of x %s" % (tuple(x.shape),))
    if x.dtype != torch.float32 or c.dtype != torch.float32:
        raise TypeError("filter_mse_spectral takes float32 images")
    _check_mask_tensor(mask, x.shape[-2], x.shape[-1], x.device)
    if c.device != x.device:
        raise ValueError("c is on %s, x on %s" % (c.device, x.device))
    x, fin = _prep(x)
    c, _ = _prep(c)
    N, M = x.shape[-2], x.shape[-1]
    batch = x.numel() // (N * M)
    m = mask.contiguous()
    plan = get_plan(2, (N, M), batch, fin | _NORM[norm], x.device)
    state = torch.empty(max(plan.spectrum_bytes, 1), dtype=torch.uint8, device=x.device)
    loss = torch.empty((), dtype=torch.float32, device=x.device)
    ws = plan.workspace()
    B.fft2d_filter_mse_spectral(plan.h, _ptr(x), _ptr(c), _ptr(m), weight, _ptr(state), _ptr(loss), _ptr(ws),
                                _stream(x.device))
    return loss, state


def mse_spectral_grad(x, state, mask, weight, norm="paper"):
    """weight * ((m - 1) sum_b |X_b|^2 + sum_b Re(conj X_b . R_b)) / (N M): the mask
    gradient of (weight/2) sum |y - c|^2 from filter_mse_spectral's state for
    the batch x (used for its shape and device only)."""
    _check_images(x)
    _check_mask_tensor(mask, x.shape[-2], x.shape[-1], x.device)
    N, M = x.shape[-2], x.shape[-1]
    batch = x.numel() // (N * M)
    plan = get_plan(2, (N, M), batch, B.FFT_IN_REAL_F32 | _NORM[norm], x.device)
    _check_spectrum(state, plan, x.device)
    out = torch.empty((N, M), dtype=torch.float32, device=x.device)
    B.fft2d_filter_mse_spectral_grad(plan.h, _ptr(state), _ptr(mask.contiguous()), weight, _ptr(out),
                                     _stream(x.device))
    return out


def filter_ragged(packed, sizes, mask, real_output=False):
    """Ragged batch: square images of sizes[i]^2 packed back to back in one
    1D tensor (float32 or complex64); returns the filtered images, packed."""
    x, fin = _prep(packed)
    sizes = [int(s) for s in sizes]
    total = sum(s * s for s in sizes)
    if x.numel() != total:
        raise ValueError("packed tensor has %d elements, sizes need %d" % (x.numel(), total))
    flags = fin | (B.FFT_OUT_REAL_F32 if real_output else 0)
    plan = get_plan(0, (), len(sizes), flags, x.device, ragged_sizes=sizes)
    out = torch.empty(total, dtype=torch.float32 if real_output else torch.complex64, device=x.device)
    mk, keep = _mask_struct(mask, 1, 1, x.device) if not isinstance(mask, torch.Tensor) else (None, None)
    if mk is None:
        raise ValueError("ragged batches take an analytic mask")
    ws = plan.workspace()
    B.fft2d_filter_ragged(plan.h, _ptr(x), _ptr(out), mk, _ptr(ws), _stream(x.device))
    return out


def tune_ragged(packed, sizes, mask, real_output=False):
    """Autotune the cached ragged plan for these sides on this batch (blocking);
    returns the chosen schedule."""
    x, fin = _prep(packed)
    sizes = [int(s) for s in sizes]
    flags = fin | (B.FFT_OUT_REAL_F32 if real_output else 0)
    plan = get_plan(0, (), len(sizes), flags, x.device, ragged_sizes=sizes)
    out = torch.empty(x.numel(), dtype=torch.float32 if real_output else torch.complex64, device=x.device)
    mk, keep = _mask_struct(mask, 1, 1, x.device)
    ws = plan.workspace()
    B.fft_plan_tune(plan.h, _ptr(x), _ptr(out), mk, _ptr(ws), _stream(x.device))
    return B.fft_plan_schedule(plan.h)


class TreePlan:
    """Owns one tree plan (fft_plan_tree) on a device."""

    def __init__(self, n, log2_procs, flags, device):
        self.device = device
        with torch.cuda.device(device):
            self.h = B.fft_plan_tree(n, log2_procs, flags)
        self.n, self.log2_procs = n, log2_procs
        self.workspace_bytes = B.fft_workspace_size(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and B is not None and getattr(B, "_lib", None) is not None:
            try:
                B.fft_plan_destroy(h)
            except Exception:
                pass
            self.h = None


_tree_cache = {}


def tree_fft(x, log2_procs, norm="paper", spin_limit=1 << 24):
    """Section 2's parallel tree on 2^log2_procs processes, emulated with one
    workgroup per process, on one complex64 signal x [n].  Returns
    (out, stats, mailbox): the transform (eq. E2's 1/N under norm="paper"),
    the per-process statistics (products generated, busy and waiting device
    ticks, receiver and level of each send, status), and the mailboxes
    [log2_procs][n], row i - 1 holding the vectors sent at merge level m1 + i,
    each at its place in the bit-reversed tree array."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.complex64 or x.dim() != 1:
        raise TypeError("expected a 1-D complex64 CUDA (HIP) tensor")
    x = x.contiguous()
    n = x.numel()
    key = (n, int(log2_procs), _NORM[norm], x.device.index)
    with _cache_lock:
        p = _tree_cache.get(key)
        if p is None:
            p = TreePlan(n, int(log2_procs), _NORM[norm], x.device)
            _tree_cache[key] = p
    out = torch.empty_like(x)
    ws = torch.empty(p.workspace_bytes, dtype=torch.uint8, device=x.device)
    stats = torch.empty(B.TREE_STATS_INT64, dtype=torch.int64, device=x.device)
    B.fft_tree_exec(p.h, _ptr(x), _ptr(out), _ptr(ws), _ptr(stats), int(spin_limit), _stream(x.device))
    nproc = 1 << int(log2_procs)
    st = B.tree_stats_dict(stats.cpu().tolist(), nproc)
    mailbox = ws[n * 8:(1 + int(log2_procs)) * n * 8].view(torch.complex64).view(int(log2_procs), n)
    return out, st, mailbox
