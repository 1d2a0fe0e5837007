"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random inputs and holds the workload parameters; it
contains none of the transform or filter arithmetic, so the GPU path and the
FP64 oracle can both be fed from it without sharing any of the method.

Star fields stand in for the paper's astronomical image (Section 6 filters a
460x506 photograph of NGC5194, which is not available): a flat sky background,
point sources with a Gaussian PSF and additive Gaussian read noise, cast to
float32 once.  Recipe (fixed here, used everywhere):

  * SeedSequence(seed).spawn(4) gives four independent streams, drawn in the
    order x positions, y positions, fluxes, noise.
  * Exactly n_stars sources, positions uniform on [0, M) x [0, N) (x along a
    row, y down the rows), i.e. a Poisson process conditioned on its count.
  * Integrated flux 10^U(lo, hi); the PSF is flux / (2 pi s^2) exp(-d^2 / 2 s^2)
    evaluated at integer pixel centres inside a (2R+1)^2 window, R = ceil(5 s),
    clipped at the image edges.
  * Background + PSFs + N(0, noise_sigma^2), in float64, then float32.
"""
import math

import numpy as np

# Workload parameters (sizes, seeds, filter parameters).  Mask parameters are
# data only; each side evaluates the mask with its own code.
CONFIGS = {
    "small_256": dict(N=256, M=256, n_stars=200, psf_sigma=1.5, seed=0,
                      mask=dict(kind="gaussian", sigma_f=0.1)),
    "sweep_1d": dict(log2_sizes=list(range(10, 23)), batch_bytes=256 << 20, seed=1),
    "image_4096": dict(N=4096, M=4096, n_stars=20000, psf_sigma=2.0, seed=2,
                       mask=dict(kind="butterworth", cutoff=0.15, order=4), batched=8),
    "ragged_512": dict(count=512, sizes=[64, 128, 256, 512, 1024, 2048], seed=3,
                       psf_sigma=1.5, stars_per_256sq=200, mask=dict(kind="gaussian", sigma_f=0.1)),
    "learn_1024": dict(B=64, N=1024, M=1024, n_stars=3200, psf_sigma=1.5, seed=4,
                       extra_noise_sigma=10.0),
}


def star_field(N, M, n_stars, psf_sigma, seed, background=100.0, noise_sigma=5.0,
               log10_flux=(2.0, 4.0)) -> np.ndarray:
    """One [N][M] float32 star field (recipe in the module docstring)."""
    ss = np.random.SeedSequence(seed)
    s_x, s_y, s_f, s_n = ss.spawn(4)
    xs = np.random.default_rng(s_x).uniform(0.0, M, n_stars)
    ys = np.random.default_rng(s_y).uniform(0.0, N, n_stars)
    flux = 10.0 ** np.random.default_rng(s_f).uniform(log10_flux[0], log10_flux[1], n_stars)
    img = np.full(N * M, background, np.float64)
    R = int(math.ceil(5.0 * psf_sigma))
    off = np.arange(-R, R + 1)
    norm = flux / (2.0 * math.pi * psf_sigma * psf_sigma)
    chunk = 4096
    for s in range(0, n_stars, chunk):
        cx = np.rint(xs[s:s + chunk]).astype(np.int64)
        cy = np.rint(ys[s:s + chunk]).astype(np.int64)
        px = cx[:, None, None] + off[None, None, :]          # columns
        py = cy[:, None, None] + off[None, :, None]          # rows
        px, py = np.broadcast_arrays(px, py)
        dx = px - xs[s:s + chunk, None, None]
        dy = py - ys[s:s + chunk, None, None]
        val = norm[s:s + chunk, None, None] * np.exp(-(dx * dx + dy * dy) / (2.0 * psf_sigma * psf_sigma))
        ok = (px >= 0) & (px < M) & (py >= 0) & (py < N)
        idx = (py * M + px)[ok]
        img += np.bincount(idx, weights=val[ok], minlength=N * M)
    img += np.random.default_rng(s_n).normal(0.0, noise_sigma, N * M)
    return img.reshape(N, M).astype(np.float32)


def uniform_complex(shape, seed) -> np.ndarray:
    """complex64 array with real and imaginary parts i.i.d. U[-1, 1] (float32)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    n = int(np.prod(shape))
    re = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    im = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    out = np.empty(n, np.complex64)
    out.real = re
    out.imag = im
    return out.reshape(shape)


# ------------------------------------------------------------ named workloads
def small_256() -> np.ndarray:
    """256x256 field, 200 stars, PSF 1.5 px, seed 0."""
    c = CONFIGS["small_256"]
    return star_field(c["N"], c["M"], c["n_stars"], c["psf_sigma"], c["seed"])


def image_4096(index: int = 0) -> np.ndarray:
    """4096x4096 field, 20000 stars, PSF 2.0 px; image i of the batch uses seed 2 + i."""
    c = CONFIGS["image_4096"]
    return star_field(c["N"], c["M"], c["n_stars"], c["psf_sigma"], c["seed"] + index)


def sweep_1d_batch(log2n: int) -> int:
    """Batch that makes one complex64 batch of length-2^log2n signals 256 MiB."""
    return CONFIGS["sweep_1d"]["batch_bytes"] // (8 << log2n)


def sweep_1d(log2n: int, batch: int = None) -> np.ndarray:
    """[batch][2^log2n] complex64 signals from seed (1, log2n)."""
    if batch is None:
        batch = sweep_1d_batch(log2n)
    return uniform_complex((batch, 1 << log2n), (CONFIGS["sweep_1d"]["seed"], log2n))


def ragged_sizes(count: int = None) -> list:
    """Square image sizes drawn uniformly from {64..2048} with seed 3."""
    c = CONFIGS["ragged_512"]
    count = c["count"] if count is None else count
    rng = np.random.default_rng(np.random.SeedSequence(c["seed"]))
    return [int(s) for s in rng.choice(c["sizes"], size=c["count"])[:count]]


def ragged_image(i: int, size: int) -> np.ndarray:
    """Image i of the ragged batch: density of 200 stars per 256^2, PSF 1.5, seed (3, i)."""
    c = CONFIGS["ragged_512"]
    n_stars = int(round(c["stars_per_256sq"] * (size / 256.0) ** 2))
    return star_field(size, size, n_stars, c["psf_sigma"], (c["seed"], i))


def _ragged_one(args):
    i, size = args
    return ragged_image(i, size)


def ragged_batch(sizes, workers: int = 1) -> np.ndarray:
    """Images 0..len(sizes)-1 of the ragged batch packed back to back (float32,
    image i row-major at offset sum_{j<i} sizes[j]^2).  workers > 1 generates
    them on a thread pool (numpy releases the interpreter lock in the heavy
    steps; no child processes; same values)."""
    total = sum(int(s) * int(s) for s in sizes)
    out = np.empty(total, dtype=np.float32)
    jobs = list(enumerate(int(s) for s in sizes))
    if workers > 1 and len(jobs) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            imgs = list(ex.map(_ragged_one, jobs))
    else:
        imgs = [_ragged_one(j) for j in jobs]
    off = 0
    for (i, s), im in zip(jobs, imgs):
        out[off:off + s * s] = im.reshape(-1)
        off += s * s
    return out


def learn_pair(b: int, N: int = None, M: int = None):
    """(noisy, clean) float32 images b of the learnable-mask batch.

    clean: star field (PSF 1.5, sky noise 5) from seed (4, b); noisy = clean +
    N(0, 10^2) from seed (4, b, 1).  Star count scales with area (3200 at 1024^2).
    """
    c = CONFIGS["learn_1024"]
    N = c["N"] if N is None else N
    M = c["M"] if M is None else M
    n_stars = int(round(c["n_stars"] * (N * M) / float(c["N"] * c["M"])))
    clean = star_field(N, M, n_stars, c["psf_sigma"], (c["seed"], b))
    rng = np.random.default_rng(np.random.SeedSequence((c["seed"], b, 1)))
    noisy = (clean.astype(np.float64) + rng.normal(0.0, c["extra_noise_sigma"], (N, M))).astype(np.float32)
    return noisy, clean
