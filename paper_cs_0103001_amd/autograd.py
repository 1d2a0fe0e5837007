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
