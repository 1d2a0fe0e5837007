"""Seeded synthetic inputs: determinism and the statistics of the recipe."""
import numpy as np

import synth


def test_star_field_deterministic_and_typed():
    a = synth.star_field(64, 32, 10, 1.5, 7)
    b = synth.star_field(64, 32, 10, 1.5, 7)
    assert a.dtype == np.float32 and a.shape == (64, 32)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, synth.star_field(64, 32, 10, 1.5, 8))


def test_star_field_statistics():
    # no stars: background 100 plus N(0, 5^2) noise
    sky = synth.star_field(256, 256, 0, 1.5, 0).astype(np.float64)
    assert abs(sky.mean() - 100.0) < 0.1
    assert abs(sky.std() - 5.0) < 0.1
    # one star well inside: the PSF window integrates to the flux
    one = synth.star_field(128, 128, 1, 1.5, 3, noise_sigma=0.0).astype(np.float64)
    flux = one.sum() - 100.0 * 128 * 128
    rng = np.random.default_rng(np.random.SeedSequence(3).spawn(4)[2])
    assert abs(flux - 10.0 ** rng.uniform(2, 4, 1)[0]) / flux < 1e-3


def test_small_256_workload():
    img = synth.small_256()
    assert img.shape == (256, 256) and img.dtype == np.float32
    assert img.max() > 150.0  # bright stars present


def test_ragged_sizes_and_sweep():
    s = synth.ragged_sizes()
    assert len(s) == 512 and set(s) <= {64, 128, 256, 512, 1024, 2048}
    assert synth.ragged_sizes() == s
    assert synth.sweep_1d_batch(10) == 32768 and synth.sweep_1d_batch(22) == 8
    x = synth.sweep_1d(10, batch=4)
    assert x.dtype == np.complex64 and x.shape == (4, 1024)
    assert np.all(np.abs(x.real) <= 1) and np.all(np.abs(x.imag) <= 1)


def test_learn_pair():
    noisy, clean = synth.learn_pair(0, 64, 64)
    assert noisy.dtype == np.float32 and clean.dtype == np.float32
    assert 8.0 < np.std(noisy.astype(np.float64) - clean) < 12.0
