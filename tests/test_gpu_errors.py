"""The error of every result of the five workloads against the FP64 oracle,
measured at the workloads' own sizes and printed as one line per result
("[error] ..."), each held to relative L2 <= 1e-5 per image or signal.

  small_256     256x256 star field, Gaussian sigma_f 0.1
  sweep_1d      N = 2^10 .. 2^22, 256 MiB batches: forward (sampled rows) and
                forward + inverse round trip (sampled rows)
  image_4096    4096x4096 star field, Butterworth order 4, cutoff 0.15 (plain
                and half-spectrum paths)
  ragged_512    the 512-image ragged batch, two images of every side
  learn_1024    batch of 1024x1024 pairs: loss and mask gradient of the fused
                filter + MSE at mask = 1 and at a random mask
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, announce, need_gpu, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _report(name, err):
    print("[error] %-58s max relL2 = %.2e" % (name, err), flush=True)
    assert err < TOL, name


def test_error_small_256():
    from paper_cs_0103001_amd import api
    img = synth.small_256()
    out = to_host(api.fft2d_filter(to_dev(img), dict(kind="gaussian", sigma_f=0.1)))
    _report("small_256 filter (c64 out)", rel_l2(out, oracle.filter2(img, oracle.mask_gaussian(256, 256, 0.1)), 2))


@pytest.mark.parametrize("lg", list(range(10, 23)))
def test_error_sweep_1d(lg):
    import torch
    from paper_cs_0103001_amd import api
    batch = synth.sweep_1d_batch(lg)
    announce("sweep 2^%d x %d" % (lg, batch))
    x = synth.sweep_1d(lg, batch)
    xd = to_dev(x)
    X = api.fft(xd)
    back = api.ifft(X)
    rows = [0, batch - 1]
    Xs = to_host(X[rows])
    bs = to_host(back[rows])
    del X, back, xd
    torch.cuda.empty_cache()
    ref = np.stack([oracle.fft(x[r], threads=oracle.default_threads()) for r in rows])
    _report("sweep_1d N=2^%d forward (rows 0, last of %d)" % (lg, batch), rel_l2(Xs, ref, 1))
    _report("sweep_1d N=2^%d forward+inverse round trip" % lg, rel_l2(bs, x[rows], 1))


def test_error_image_4096_plain_and_half():
    from paper_cs_0103001_amd import api
    img = synth.image_4096(0)
    mask = dict(kind="butterworth", cutoff=0.15, order=4)
    ref = oracle.filter2(img, oracle.mask_butterworth(4096, 4096, 0.15, 4))
    xd = to_dev(img)
    _report("image_4096 filter, plain path (c64 out)", rel_l2(to_host(api.fft2d_filter(xd, mask)), ref, 2))
    _report("image_4096 filter, half-spectrum path (f32 out)",
            rel_l2(to_host(api.fft2d_filter(xd, mask, real_output=True, real_even=True)), ref.real, 2))


def test_error_ragged_512():
    from paper_cs_0103001_amd import api
    sizes = synth.ragged_sizes()
    flat = synth.ragged_batch(sizes, workers=8)
    rmask = dict(synth.CONFIGS["ragged_512"]["mask"])
    out = to_host(api.filter_ragged(to_dev(flat), sizes, rmask))
    offs = np.concatenate([[0], np.cumsum([s * s for s in sizes])])
    worst = 0.0
    for s in sorted(set(sizes)):
        for i in [k for k, t in enumerate(sizes) if t == s][:2]:
            img = flat[offs[i]:offs[i + 1]].reshape(s, s)
            ref = oracle.filter2(img, oracle.mask_gaussian(s, s, rmask["sigma_f"]))
            worst = max(worst, rel_l2(out[offs[i]:offs[i + 1]].reshape(s, s), ref, 2))
    _report("ragged_512 filter, 2 images of every side (c64 out)", worst)


@pytest.mark.parametrize("at_one", [True, False])
def test_error_learn_1024(at_one):
    import torch
    from paper_cs_0103001_amd.autograd import fft_filter_mse
    B, N, M = 8, 1024, 1024
    noisy, clean = zip(*[synth.learn_pair(b) for b in range(B)])
    noisy, clean = np.stack(noisy), np.stack(clean)
    mask = (np.ones((N, M), np.float32) if at_one
            else np.random.default_rng(5).uniform(0.2, 1.2, (N, M)).astype(np.float32))
    m = to_dev(mask).requires_grad_(True)
    L = fft_filter_mse(to_dev(noisy), to_dev(clean), m)
    L.backward()
    _, L_ref, g_ref = oracle.loss_grad(noisy, clean, mask)
    tag = "mask = 1" if at_one else "random mask"
    _report("learn_1024 (batch 8) loss, %s" % tag, abs(float(L.detach()) - L_ref) / L_ref)
    _report("learn_1024 (batch 8) mask gradient, %s" % tag, rel_l2(to_host(m.grad), g_ref, 2))
    del torch
