"""Section 6's front end on the GPU: images of any size zero-padded to powers
of two, filtered, cropped back; and the spectrum magnitude.  Against the FP64
oracle (pad2 / filter2_padded / spectrum_padded)."""
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
    if kind == "disc":
        return dict(kind="disc", b=340.0), oracle.mask_disc(N, M, 340.0)
    if kind == "gaussian":
        return dict(kind="gaussian", sigma_f=0.1), oracle.mask_gaussian(N, M, 0.1)
    return dict(kind="butterworth", cutoff=0.15, order=4), oracle.mask_butterworth(N, M, 0.15, 4)


@pytest.mark.parametrize("B,n0,m0,kind", [(1, 460, 506, "disc"), (2, 100, 200, "butterworth"),
                                          (1, 3, 5, "gaussian"), (1, 1, 1, "gaussian"),
                                          (2, 17, 64, "gaussian"), (1, 64, 33, "butterworth")])
def test_padded_filter_vs_oracle(B, n0, m0, kind):
    from paper_cs_0103001_amd import api
    imgs = np.stack([synth.star_field(n0, m0, max(1, n0 * m0 // 300), 1.5, (90, b, n0, m0)) for b in range(B)])
    N, M = oracle.next_pow2(n0), oracle.next_pow2(m0)
    spec, m64 = _mask(kind, N, M)
    announce("padded filter B=%d %dx%d %s" % (B, n0, m0, kind))
    y = to_host(api.fft2d_filter(to_dev(imgs), spec))
    assert y.shape == (B, n0, m0)
    ref = oracle.filter2_padded(imgs, m64, threads=4)
    assert rel_l2(y, ref, 2) < TOL
    yr = to_host(api.fft2d_filter(to_dev(imgs), spec, real_output=True))
    assert rel_l2(yr, ref.real, 2) < TOL


def test_padded_complex_input():
    from paper_cs_0103001_amd import api
    x = synth.uniform_complex((2, 37, 70), (91, 0))
    spec, m64 = _mask("gaussian", 64, 128)
    announce("padded complex 37x70")
    y = to_host(api.fft2d_filter(to_dev(x), spec))
    assert rel_l2(y, oracle.filter2_padded(x, m64, threads=4), 2) < TOL


@pytest.mark.parametrize("n0,m0", [(460, 506), (64, 64), (5, 3), (1, 1)])
def test_spectrum_vs_oracle(n0, m0):
    from paper_cs_0103001_amd import api
    img = synth.star_field(n0, m0, max(1, n0 * m0 // 300), 1.5, (92, n0, m0))
    announce("spectrum %dx%d" % (n0, m0))
    s = to_host(api.spectrum(to_dev(img)))
    ref = oracle.spectrum_padded(img, threads=4)
    assert s.shape == ref.shape
    assert rel_l2(s, ref, 2) < TOL
