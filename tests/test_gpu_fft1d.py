"""1D transforms on the GPU against the FP64 oracle (eq. E2 forward with 1/N,
eq. E3 inverse unscaled), every power-of-two length up to 2^22."""
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


SINGLE = list(range(0, 15))          # one LDS pass
FOURSTEP = [15, 16, 17, 18, 20]       # two strided passes


@pytest.mark.parametrize("lg", SINGLE + FOURSTEP)
def test_forward_inverse_vs_oracle(lg):
    api = _api()
    n = 1 << lg
    batch = 5 if lg < 16 else 2        # 5 rows: the last workgroup is partly empty
    x = synth.uniform_complex((batch, n), (11, lg))
    announce("fft1d n=%d batch=%d" % (n, batch))
    X = to_host(api.fft(to_dev(x)))
    assert rel_l2(X, oracle.fft(x, threads=4), 1) < TOL
    announce("ifft1d n=%d batch=%d" % (n, batch))
    f = to_host(api.ifft(to_dev(x)))
    assert rel_l2(f, oracle.ifft(x, threads=4), 1) < TOL


@pytest.mark.parametrize("lg", [0, 3, 10, 12, 14, 16])
def test_norms_adjoints_and_real_io(lg):
    api = _api()
    from paper_cs_0103001_amd import _binding as B
    n = 1 << lg
    x = synth.uniform_complex((3, n), (12, lg))
    xd = to_dev(x)
    ref_f = oracle.fft(x, threads=4)
    ref_i = oracle.ifft(x, threads=4)
    announce("fft1d norms n=%d" % n)
    assert rel_l2(to_host(api.fft(xd, norm="numpy")), ref_f * n, 1) < TOL
    assert rel_l2(to_host(api.ifft(xd, norm="numpy")), ref_i / n, 1) < TOL
    # adjoint of the forward (1/N) F^H and of the inverse F
    assert rel_l2(to_host(api.transform(xd, 1, B.FFT_ADJ_FORWARD)), ref_i / n, 1) < TOL
    assert rel_l2(to_host(api.transform(xd, 1, B.FFT_ADJ_INVERSE)), ref_f * n, 1) < TOL
    if lg <= 14:
        xr = x.real.copy()
        assert rel_l2(to_host(api.fft(to_dev(xr))), oracle.fft(xr, threads=4), 1) < TOL
        got = to_host(api.ifft(xd, real_output=True))
        assert got.dtype == np.float32
        assert rel_l2(got, ref_i.real, 1) < TOL


def test_empty_batch():
    api = _api()
    import torch
    x = torch.empty((0, 256), dtype=torch.complex64, device="cuda")
    assert api.fft(x).shape == (0, 256)


@pytest.mark.parametrize("lg", [10, 14, 16, 22])
def test_full_sweep_batch_sampled_rows(lg):
    """The 256 MiB batch of the 1D sweep, in the launch shape the benchmark
    times; sampled rows are checked against the oracle, and the round trip
    against the input."""
    api = _api()
    n = 1 << lg
    batch = synth.sweep_1d_batch(lg)
    x = synth.sweep_1d(lg, batch)
    announce("fft1d sweep n=%d batch=%d" % (n, batch))
    xd = to_dev(x)
    X = api.fft(xd)
    back = api.ifft(X)
    rows = sorted({0, batch // 3, batch - 1})
    Xh = to_host(X[rows])
    assert rel_l2(Xh, oracle.fft(x[rows], threads=8), 1) < TOL
    assert rel_l2(to_host(back), x, 1) < TOL


def test_deterministic():
    api = _api()
    x = to_dev(synth.uniform_complex((64, 4096), 5))
    a = to_host(api.fft(x))
    b = to_host(api.fft(x))
    np.testing.assert_array_equal(a, b)
