"""2D transforms and the Section-6 filter on the GPU against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _api():
    from paper_cs_0103001_amd import api
    return api


SHAPES = [(1, 1), (2, 2), (1, 16), (16, 1), (4, 8), (16, 16), (32, 64), (64, 32), (256, 256), (128, 1024),
          (1024, 128), (64, 4096), (4096, 64), (8192, 16), (16, 8192), (16384, 16), (16, 16384)]


@pytest.mark.parametrize("N,M", SHAPES)
def test_fft2_ifft2_vs_oracle(N, M):
    api = _api()
    from paper_cs_0103001_amd import _binding as B
    x = synth.uniform_complex((2, N, M), (21, N, M))
    xd = to_dev(x)
    announce("fft2 %dx%d" % (N, M))
    ref = oracle.fft2(x)
    assert rel_l2(to_host(api.fft2(xd)), ref, 2) < TOL
    announce("ifft2 %dx%d" % (N, M))
    refi = oracle.ifft2(x)
    assert rel_l2(to_host(api.ifft2(xd)), refi, 2) < TOL
    assert rel_l2(to_host(api.fft2(xd, norm="numpy")), ref * N, 2) < TOL
    assert rel_l2(to_host(api.ifft2(xd, norm="numpy")), refi / N, 2) < TOL
    # adjoints: (eq. 5)^H = (1/N) F^*; (2D-IDFT)^H = (1/M) F
    assert rel_l2(to_host(api.transform(xd, 2, B.FFT_ADJ_FORWARD)), refi * (M / float(N)), 2) < TOL
    assert rel_l2(to_host(api.transform(xd, 2, B.FFT_ADJ_INVERSE)), ref * (N / float(M)), 2) < TOL
    xr = x.real.copy()
    assert rel_l2(to_host(api.fft2(to_dev(xr))), oracle.fft2(xr), 2) < TOL
    got = to_host(api.ifft2(xd, real_output=True))
    assert got.dtype == np.float32 and rel_l2(got, refi.real, 2) < TOL


def test_small_256_gaussian_workload():
    """256x256 star field, Gaussian sigma_f = 0.1 (the small parity workload)."""
    api = _api()
    img = synth.small_256()
    announce("filter small_256 gaussian")
    out = to_host(api.fft2d_filter(to_dev(img), dict(kind="gaussian", sigma_f=0.1)))
    ref = oracle.filter2(img, oracle.mask_gaussian(256, 256, 0.1))
    assert rel_l2(out, ref, 2) < TOL
    # an even mask keeps a real image real
    assert np.max(np.abs(out.imag)) < 1e-4 * np.max(np.abs(out.real))


@pytest.mark.parametrize("N,M,kind", [(512, 512, "butterworth"), (64, 256, "butterworth"), (256, 64, "gaussian"),
                                      (512, 512, "disc"), (32, 32, "tensor"), (1024, 1024, "tensor"),
                                      (16, 16, "gaussian"), (4, 8, "butterworth"), (1, 1, "gaussian"),
                                      (32, 16384, "butterworth"), (16384, 32, "gaussian"),
                                      (2048, 512, "tensor"), (4096, 64, "tensor")])
@pytest.mark.parametrize("complex_in", [False, True])
def test_filter_kinds_vs_oracle(N, M, kind, complex_in):
    api = _api()
    import torch
    B_ = 3
    rng = np.random.default_rng(N * 7 + M)
    x = np.stack([synth.star_field(N, M, max(1, N * M // 300), 1.5, (31, N, M, b)) for b in range(B_)])
    if complex_in:
        x = x.astype(np.complex64) + 1j * rng.uniform(-5, 5, x.shape).astype(np.float32)
    if kind == "butterworth":
        spec = dict(kind="butterworth", cutoff=0.15, order=4)
        mask = oracle.mask_butterworth(N, M, 0.15, 4)
    elif kind == "gaussian":
        spec = dict(kind="gaussian", sigma_f=0.1)
        mask = oracle.mask_gaussian(N, M, 0.1)
    elif kind == "disc":
        spec = dict(kind="disc", b=340.0)   # Section 6's parameter for a 512x512 padded image
        mask = oracle.mask_disc(N, M, 340.0)
    else:
        mask = rng.uniform(0, 1, (N, M)).astype(np.float32)
        spec = to_dev(mask)
        mask = mask.astype(np.float64)
    announce("filter %s %dx%d complex_in=%s" % (kind, N, M, complex_in))
    out = to_host(api.fft2d_filter(to_dev(x), spec))
    ref = oracle.filter2(x, mask)
    assert rel_l2(out, ref, 2) < TOL
    outr = to_host(api.fft2d_filter(to_dev(x), spec, real_output=True))
    assert outr.dtype == np.float32 and rel_l2(outr, ref.real, 2) < TOL
    del torch


def test_filter_paper_and_numpy_norm_agree():
    api = _api()
    x = to_dev(synth.star_field(128, 256, 50, 1.5, 41))
    spec = dict(kind="butterworth", cutoff=0.2, order=2)
    a = to_host(api.fft2d_filter(x, spec))
    b = to_host(api.fft2d_filter(x, spec, norm="numpy"))
    assert rel_l2(a, b, 2) < 1e-6


def test_image_4096_butterworth_full_size():
    """The 4096x4096 headline workload, in the launch configuration the
    benchmark times, against the full FP64 oracle."""
    api = _api()
    img = synth.image_4096(0)
    announce("filter image_4096 butterworth")
    out = to_host(api.fft2d_filter(to_dev(img), dict(kind="butterworth", cutoff=0.15, order=4)))
    ref = oracle.filter2(img, oracle.mask_butterworth(4096, 4096, 0.15, 4))
    err = rel_l2(out, ref, 2)
    print("image_4096 relL2 = %.3e" % err)
    assert err < TOL


def test_image_4096_batch_matches_single_images():
    """Batch of 8 (the batched workload): every image equals its own
    single-image result bit for bit (images are independent), and image 7 is
    checked against the oracle."""
    api = _api()
    import torch
    imgs = np.stack([synth.image_4096(i) for i in (0, 7)])
    spec = dict(kind="butterworth", cutoff=0.15, order=4)
    announce("filter image_4096 batch")
    batch = torch.empty((8, 4096, 4096), dtype=torch.float32, device="cuda")
    batch[0] = to_dev(imgs[0])
    batch[7] = to_dev(imgs[1])
    for i in range(1, 7):
        batch[i] = batch[0] * (i + 1)
    outb = api.fft2d_filter(batch, spec)
    single7 = to_host(api.fft2d_filter(to_dev(imgs[1]), spec))
    np.testing.assert_array_equal(to_host(outb[7]), single7)
    ref7 = oracle.filter2(imgs[1], oracle.mask_butterworth(4096, 4096, 0.15, 4))
    assert rel_l2(single7, ref7, 2) < TOL
    # linearity across the batch: image i = (i+1) * image 0 gives (i+1) * output 0
    o0 = to_host(outb[0])
    for i in (1, 6):
        assert rel_l2(to_host(outb[i]), o0 * (i + 1), 2) < TOL


def test_filter_in_place_and_deterministic():
    api = _api()
    x = to_dev(synth.star_field(256, 512, 100, 1.5, 51).astype(np.complex64))
    spec = dict(kind="gaussian", sigma_f=0.1)
    a = to_host(api.fft2d_filter(x, spec))
    b = to_host(api.fft2d_filter(x, spec))
    np.testing.assert_array_equal(a, b)


def test_largest_plane_16384_separable():
    """16384 x 16384, the largest rank-2 plan (its blocked workspace, 2.15 GB,
    is above 2^31 bytes).  A separable image f = g h^T (integers, so every
    product is exact in float32) filtered by the separable Gaussian mask gives
    y = a b^T with a, b the 1D filters of g and h (eq. 5 and the 2D-IDFT
    factor into row and column sums); a, b come from the FP64 oracle's 1D
    transforms and masks.  Every element is compared."""
    import torch
    from paper_cs_0103001_amd import api
    N = M = 16384
    rng = np.random.default_rng(16384)
    g = rng.integers(-2048, 2049, N).astype(np.float64)
    h = rng.integers(-2048, 2049, M).astype(np.float64)
    sig = 0.05
    gu = oracle.mask_gaussian(N, 1, sig)[:, 0]
    gv = oracle.mask_gaussian(1, M, sig)[0]
    a = oracle.ifft(gu * oracle.fft(g, threads=8), threads=8)
    b = oracle.ifft(gv * oracle.fft(h, threads=8), threads=8)
    x = torch.from_numpy(g.astype(np.float32)).cuda()[:, None] * torch.from_numpy(h.astype(np.float32)).cuda()[None, :]
    announce("filter 16384^2 separable")
    y = api.fft2d_filter(x, dict(kind="gaussian", sigma_f=sig))
    torch.cuda.synchronize()
    del x
    num = den = 0.0
    for r0 in range(0, N, 1024):
        got = y[r0:r0 + 1024].cpu().numpy().astype(np.complex128)
        ref = np.outer(a[r0:r0 + 1024], b)
        num += float(np.sum(np.abs(got - ref) ** 2))
        den += float(np.sum(np.abs(ref) ** 2))
    err = (num / den) ** 0.5
    print("16384^2 separable filter relL2 %.3e" % err)
    assert err < TOL


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_non_finite_input_propagates(bad):
    """A NaN or Inf pixel spreads through the transforms (every bin of its
    image's spectrum takes it) without an error status or a fault; the other
    images of the batch stay finite and equal to their oracle results."""
    from paper_cs_0103001_amd import api
    N = M = 256
    x = np.stack([synth.star_field(N, M, 50, 1.5, (97, b)) for b in range(3)])
    x[1, 17, 33] = bad
    announce("non-finite input %s" % bad)
    y = to_host(api.fft2d_filter(to_dev(x), dict(kind="butterworth", cutoff=0.15, order=4)))
    assert not np.isfinite(y[1]).any()
    m = oracle.mask_butterworth(N, M, 0.15, 4)
    for b in (0, 2):
        assert np.isfinite(y[b]).all()
        assert rel_l2(y[b], oracle.filter2(x[b], m), 2) < TOL
    yr = to_host(api.fft2d_filter(to_dev(x), None, real_even=True, real_output=True))
    assert not np.isfinite(yr[1]).any() and np.isfinite(yr[0]).all() and np.isfinite(yr[2]).all()


def test_tensor_mask_long_columns_stages_and_fused_mse():
    """Tensor masks on plans with columns of 2048 points or more (read from a
    transposed copy made per call): the three stages run one by one equal the
    whole filter bit for bit, and the fused filter + MSE loss and gradient
    match the oracle."""
    import torch
    from paper_cs_0103001_amd import _binding as B
    from paper_cs_0103001_amd import api
    from paper_cs_0103001_amd.autograd import fft_filter_mse
    N, M, Bn = 4096, 64, 2
    x = np.stack([synth.star_field(N, M, 800, 1.5, (33, b)) for b in range(Bn)])
    mask = np.random.default_rng(41).uniform(0.2, 1.2, (N, M)).astype(np.float32)
    xd, md = to_dev(x), to_dev(mask)
    announce("tensor mask %dx%d stages" % (N, M))
    whole = to_host(api.fft2d_filter(xd, md))
    assert rel_l2(whole, oracle.filter2(x, mask.astype(np.float64)), 2) < TOL
    plan = api.get_plan(2, (N, M), Bn, B.FFT_IN_REAL_F32, xd.device)
    ws = plan.workspace()
    out = torch.empty((Bn, N, M), dtype=torch.complex64, device="cuda")
    mk = B.make_mask("tensor", data_ptr=md.data_ptr())
    for s_ in (0, 1, 2):
        B.fft2d_filter_stage(plan.h, s_, api._ptr(xd), api._ptr(out), mk, api._ptr(ws), api._stream(xd.device))
    assert np.array_equal(to_host(out).view(np.uint32), whole.view(np.uint32))
    announce("tensor mask %dx%d fused mse" % (N, M))
    clean = (x - np.float32(3.0)).astype(np.float32)
    m = md.clone().requires_grad_(True)
    L = fft_filter_mse(xd, to_dev(clean), m)
    L.backward()
    _, L_ref, g_ref = oracle.loss_grad(x, clean, mask)
    assert abs(float(L.detach()) - L_ref) / L_ref < 1e-5
    assert rel_l2(to_host(m.grad), g_ref, 2) < TOL
