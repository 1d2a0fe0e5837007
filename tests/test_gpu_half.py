"""The half-spectrum path for real images and even masks (FFT_REAL_EVEN):
the same filtered image as the full transform, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _mask(kind, N, M):
    if kind == "gaussian":
        return dict(kind="gaussian", sigma_f=0.1), oracle.mask_gaussian(N, M, 0.1)
    if kind == "butterworth":
        return dict(kind="butterworth", cutoff=0.15, order=4), oracle.mask_butterworth(N, M, 0.15, 4)
    if kind == "disc":
        return dict(kind="disc", b=0.3 * N), oracle.mask_disc(N, M, 0.3 * N)
    return None, np.ones((N, M))


@pytest.mark.parametrize("B,N,M,kind", [(1, 32, 4, "gaussian"), (2, 64, 64, "butterworth"), (1, 256, 128, "disc"),
                                        (3, 128, 512, "none"), (1, 1024, 1024, "gaussian"), (2, 32, 8192, "gaussian"),
                                        (1, 8192, 16, "butterworth")])
def test_half_spectrum_filter_vs_oracle(B, N, M, kind):
    from paper_cs_0103001_amd import api
    x = np.stack([synth.star_field(N, M, max(1, N * M // 300), 1.5, (93, b, N, M)) for b in range(B)])
    spec, m64 = _mask(kind, N, M)
    ref = oracle.filter2(x, m64, threads=4)
    announce("half spectrum B=%d %dx%d %s" % (B, N, M, kind))
    y = to_host(api.fft2d_filter(to_dev(x), spec, real_even=True))
    assert rel_l2(y, ref, 2) < TOL
    assert not np.any(y.imag)
    yr = to_host(api.fft2d_filter(to_dev(x), spec, real_even=True, real_output=True))
    assert rel_l2(yr, ref.real, 2) < TOL


def test_half_spectrum_full_size_image_4096():
    from paper_cs_0103001_amd import api
    img = synth.image_4096(0)
    spec = dict(synth.CONFIGS["image_4096"]["mask"])
    announce("half spectrum 4096^2")
    y = to_host(api.fft2d_filter(to_dev(img), spec, real_even=True, real_output=True))
    ref = oracle.filter2(img, oracle.mask_butterworth(4096, 4096, 0.15, 4)).real
    assert rel_l2(y, ref, 2) < TOL


def test_half_spectrum_rejects_odd_masks():
    import torch
    from paper_cs_0103001_amd import api
    from paper_cs_0103001_amd import _binding as B
    x = to_dev(np.ones((64, 64), np.float32))
    with pytest.raises(B.FFTError):
        api.fft2d_filter(x, torch.ones((64, 64), device="cuda"), real_even=True)
    with pytest.raises(B.FFTError):
        api.fft2d_filter(x, dict(kind="disc", b=10.0, c1=5.0, c2=7.0), real_even=True)
    # a disc centred at bin 0 is not even on the raw bin grid: bin (1, 1) lies
    # inside, bin (63, 63) outside, so the half spectrum would be wrong
    for c1, c2 in ((0.0, 0.0), (32.0, 0.0), (0.0, 32.0)):
        with pytest.raises(B.FFTError):
            api.fft2d_filter(x, dict(kind="disc", b=10.0, c1=c1, c2=c2), real_even=True)


def test_disc_centred_at_zero_full_path_vs_oracle():
    """The same disc on the full path (which has no evenness requirement)."""
    from paper_cs_0103001_amd import api
    N = M = 64
    x = synth.star_field(N, M, 20, 1.5, (95, N))
    announce("disc at 0, full path")
    y = to_host(api.fft2d_filter(to_dev(x), dict(kind="disc", b=10.0, c1=0.0, c2=0.0)))
    assert rel_l2(y, oracle.filter2(x, oracle.mask_disc(N, M, 10.0, 0.0, 0.0)), 2) < TOL
