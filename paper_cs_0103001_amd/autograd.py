"""Differentiable frequency-domain filter with a learnable real mask.

y = 2D-IDFT(m . 2D-DFT(x)) for a batch x [B][N][M] and a shared real mask
m [N][M].  Backward (PyTorch passes g = dL/dRe(y) + i dL/dIm(y)):

  dL/dm = sum_b Re( conj(X_b) . 2D-IDFT^H(g_b) ),   X_b = 2D-DFT(x_b),

computed by the adjoint column kernel with a fixed-order batch sum, and

  dL/dx = (m-filter)^H g = 2D-IDFT(m . 2D-DFT(g)),

since with a real mask the filter operator is self-adjoint (its scale is
1/(NM) under eq. 5 and the 2D-IDFT, and the unnormalised DFT matrix is
symmetric).
"""
import torch

from . import api


class FFTFilterFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, mask):
        y, spec = api.fft2d_filter(x, mask.detach(), spectrum=True)
        ctx.save_for_backward(spec, mask)
        ctx.x_real = x.dtype == torch.float32
        ctx.shape = x.shape
        return y

    @staticmethod
    def backward(ctx, g):
        spec, mask = ctx.saved_tensors
        g = g.contiguous()
        if g.dtype != torch.complex64:
            g = g.to(torch.complex64)
        gm = api.mask_grad(g, spec) if ctx.needs_input_grad[1] else None
        gx = None
        if ctx.needs_input_grad[0]:
            gx = api.fft2d_filter(g, mask.detach(), real_output=ctx.x_real)
        return gx, gm


def fft_filter(x, mask):
    """Filter x (float32 or complex64 [..., N, M]) with a learnable float32 mask [N, M]."""
    return FFTFilterFn.apply(x, mask)


class FFTFilterMSEFn(torch.autograd.Function):
    """L = mean over all pixels of |2D-IDFT(m . 2D-DFT(x)) - c|^2 for real x, c.

    Evaluated through the exact identity y - c = 2D-IDFT((m - 1) . X) + (x - c),
    so that neither the loss nor its mask gradient subtracts nearly equal
    float32 values where the filter is close to the identity (m near 1, the
    learnable mask's starting point).  The loss is taken in the frequency
    domain (Parseval's relation: sum |y - c|^2 = sum |(m - 1) X + R|^2 / (N M)
    for the unnormalised spectra X of x and R of x - c), and the forward also
    forms the per-bin sums the mask gradient needs, so the backward takes no
    transform; rows longer than 4096 points use the spatial-domain form.
    Backward:
      dL/dm = (2/K) sum_b [Re(conj X_b . R_b) + (m - 1)|X_b|^2] / (N M)
      dL/dx = (2/K) Re(filter_m(y - c)),   dL/dc = -(2/K)(y - c),
    with K = B N M and filter_m self-adjoint for a real mask.
    """

    @staticmethod
    def forward(ctx, x, clean, mask):
        if x.dtype != torch.float32 or clean.dtype != torch.float32:
            raise TypeError("fft_filter_mse takes float32 images")
        m = mask.detach().contiguous()
        x = x.contiguous()
        clean = clean.contiguous()
        K = clean.numel()
        try:
            loss, state = api.filter_mse_spectral(x, clean, m, 1.0 / K)
            ctx.spectral = True
        except api.B.FFTError as e:
            if e.code != api.B.FFT_ERR_UNSUPPORTED:
                raise
            loss, state = api.filter_mse(x, clean, m, 1.0 / K)
            ctx.spectral = False
        ctx.save_for_backward(state, x, clean, m)
        ctx.K = K
        return loss

    @staticmethod
    def backward(ctx, gL):
        state, x, clean, m = ctx.saved_tensors
        K = ctx.K
        gx = gc = gm = None
        if ctx.needs_input_grad[2]:
            if ctx.spectral:
                gm = api.mse_spectral_grad(x, state, m, 2.0 / K) * gL
            else:
                gm = api.mse_grad(x, clean, state, m, 2.0 / K) * gL
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            r = api.fft2d_filter(x, m) - clean  # y - c (only for the image gradients)
            if ctx.needs_input_grad[0]:
                gx = api.fft2d_filter(r, m, real_output=True) * (2.0 / K * gL)
            if ctx.needs_input_grad[1]:
                gc = r.real * (-2.0 / K * gL)
        return gx, gc, gm


def fft_filter_mse(noisy, clean, mask):
    """Mean squared error between the filtered noisy batch and clean (both float32
    [..., N, M]) with a learnable float32 mask [N, M]; differentiable in all three."""
    return FFTFilterMSEFn.apply(noisy, clean, mask)
