"""fft2d_filter_noalloc (the filter with its intermediate in the library's
static scratch array) against fft2d_filter with a caller workspace, through the
C-ABI: two calls in a row, the second on a smaller input, each bit-identical to
the workspace form (same kernels, same arguments but the workspace address)
and within the parity tolerance of the FP64 oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _run(B, torch, x, dims, flags, mask, padded=False):
    """out_ws, out_noalloc for one plan (f32 in, c64 or f32 out)."""
    batch = x.shape[0]
    h = B.fft_plan_padded(dims, batch, flags) if padded else B.fft_plan(2, dims, batch, flags)
    try:
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        xd = to_dev(x)
        odt = torch.float32 if flags & B.FFT_OUT_REAL_F32 else torch.complex64
        out_ws = torch.full(x.shape, float("nan"), dtype=odt, device="cuda")
        out_na = torch.full(x.shape, float("nan"), dtype=odt, device="cuda")
        ws = torch.empty(max(B.fft_workspace_size(h), 1), dtype=torch.uint8, device="cuda")
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        B.fft2d_filter(h, p(xd), p(out_ws), mask, p(ws), st)
        B.fft2d_filter_noalloc(h, p(xd), p(out_na), mask, st)
        return to_host(out_ws), to_host(out_na)
    finally:
        B.fft_plan_destroy(h)


def test_noalloc_matches_workspace_form_twice_shrinking():
    import torch
    from paper_cs_0103001_amd import _binding as B
    f32c64 = B.FFT_IN_REAL_F32
    butter = B.make_mask("butterworth", cutoff=0.15, order=4)
    gauss = B.make_mask("gaussian", sigma_f=0.1)
    # first call: the full 4096^2 image (one chunk, the largest the scratch holds)
    announce("noalloc 4096x4096 butterworth (first call)")
    img = synth.image_4096()[None]
    a, b = _run(B, torch, img, (4096, 4096), f32c64, butter)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    rows = [0, 1, 2047, 4095]
    ref = oracle.filter2(img[0], oracle.mask_butterworth(4096, 4096, 0.15, 4))
    assert rel_l2(b[0][rows], ref[rows], 1) < TOL
    # second call, smaller input: batch of 3 at 256^2 on the same scratch,
    # whose head still holds the 4096^2 intermediate of the first call
    announce("noalloc 3 x 256x256 gaussian (second call, smaller)")
    small = np.stack([synth.small_256(), synth.small_256()[::-1].copy(), synth.small_256()[:, ::-1].copy()])
    a, b = _run(B, torch, small, (256, 256), f32c64, gauss)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    mk = oracle.mask_gaussian(256, 256, 0.1)
    for i in range(3):
        assert rel_l2(b[i], oracle.filter2(small[i], mk), 2) < TOL


def test_noalloc_padded_and_real_out():
    import torch
    from paper_cs_0103001_amd import _binding as B
    announce("noalloc padded 460x506 disc b=340, f32 out")
    img = synth.star_field(460, 506, 300, 1.5, seed=11)[None]
    flags = B.FFT_IN_REAL_F32 | B.FFT_OUT_REAL_F32
    disc = B.make_mask("disc", b=340.0, c1=256.0, c2=256.0)
    a, b = _run(B, torch, img, (460, 506), flags, disc, padded=True)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    ref = oracle.filter2_padded(img[0], oracle.mask_disc(512, 512, 340.0, 256.0, 256.0))
    assert rel_l2(b[0], ref.real, 2) < TOL


def test_noalloc_refuses_plans_beyond_scratch():
    import torch
    from paper_cs_0103001_amd import _binding as B
    announce("noalloc refuses 8192^2")
    h = B.fft_plan(2, (8192, 8192), 1, B.FFT_IN_REAL_F32)
    try:
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        x = torch.zeros((8192, 8192), dtype=torch.float32, device="cuda")
        out = torch.zeros((8192, 8192), dtype=torch.complex64, device="cuda")
        rc = B.lib().fft2d_filter_noalloc(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), None, st)
        assert rc == B.FFT_ERR_SCRATCH
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0  # nothing was launched
    finally:
        B.fft_plan_destroy(h)
    # a plan of another kind is refused as such
    h = B.fft_plan(1, (1024,), 4, 0)
    try:
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        assert B.lib().fft2d_filter_noalloc(h, None, None, None, st) == B.FFT_ERR_STATE
    finally:
        B.fft_plan_destroy(h)


def test_noalloc_tensor_mask_long_columns():
    """A tensor mask on a plan with 2048-point columns: its transposed copy
    also lives in the scratch (2048 x 1024: 16 MiB intermediate + 8 MiB);
    4096 x 4096 with a tensor mask needs 192 MiB and is refused."""
    import torch
    from paper_cs_0103001_amd import _binding as B
    announce("noalloc tensor mask 2048x1024")
    img = np.stack([synth.star_field(2048, 1024, 6000, 1.5, seed=12)])
    mask = np.random.default_rng(13).uniform(0.2, 1.2, (2048, 1024)).astype(np.float32)
    md = to_dev(mask)
    mk = B.make_mask("tensor", data_ptr=md.data_ptr())
    a, b = _run(B, torch, img, (2048, 1024), B.FFT_IN_REAL_F32, mk)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert rel_l2(b[0], oracle.filter2(img[0], mask.astype(np.float64)), 2) < TOL
    h = B.fft_plan(2, (4096, 4096), 1, B.FFT_IN_REAL_F32)
    try:
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        m4 = torch.ones((4096, 4096), dtype=torch.float32, device="cuda")
        x = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda")
        out = torch.zeros((4096, 4096), dtype=torch.complex64, device="cuda")
        mk4 = B.make_mask("tensor", data_ptr=m4.data_ptr())
        rc = B.lib().fft2d_filter_noalloc(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.byref(mk4), st)
        assert rc == B.FFT_ERR_SCRATCH
    finally:
        B.fft_plan_destroy(h)
