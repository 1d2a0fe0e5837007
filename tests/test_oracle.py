"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself only: each check ties it to a
library routine (numpy's pocketfft), a closed form, an identity the paper
states, the paper's worked 8-point example or its Table 1, or exact finite
differences of a quadratic loss.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import complexity

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(12345)


def crand(*shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def relerr(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# --------------------------------------------------------------- definition
@pytest.mark.parametrize("n", list(range(1, 33)) + [64, 100, 128])
def test_direct_dft_matches_library(n):
    # eq. (E2): H = (1/N) DFT; numpy's fft is the unscaled sum with e^{-2 pi i kj/N}
    f = crand(n)
    assert relerr(oracle.dft_direct(f), np.fft.fft(f) / n) < 1e-13
    # + sign, unit scale: numpy ifft is (1/N) sum e^{+...}
    assert relerr(oracle.dft_direct(f, sign=+1, scale=1.0), np.fft.ifft(f) * n) < 1e-13


def test_direct_dft_hand_values():
    # worked by hand: f = [1,2,3,4] -> (1/4)[10, -2+2i, -2, -2-2i]
    h = oracle.dft_direct([1, 2, 3, 4])
    np.testing.assert_allclose(h, [2.5, -0.5 + 0.5j, -0.5, -0.5 - 0.5j], atol=1e-15)
    h2 = oracle.dft_direct([3.0, 1.0])
    np.testing.assert_allclose(h2, [2.0, 1.0], atol=1e-15)


# ------------------------------------------------------------ Section 2 tree
POW2 = [1 << m for m in range(0, 13)]


@pytest.mark.parametrize("n", POW2)
def test_tree_fft_closed_forms(n):
    j = np.arange(n)
    for k0 in sorted({0, 1 % n, n // 3, n - 1}):
        # a single exponential e^{+2 pi i k0 j/N} has H = delta_{k,k0}, exactly 1
        e = np.exp(2j * np.pi * k0 * j / n)
        H = oracle.fft(e)
        ref = np.zeros(n, complex)
        ref[k0] = 1.0
        assert np.max(np.abs(H - ref)) < 1e-12 * max(1, np.log2(n))
    for j0 in sorted({0, 1 % n, n // 2, n - 1}):
        # delta at j0: H[k] = (1/N) e^{-2 pi i k j0/N}; |H| = 1/N everywhere, phase steps by -2 pi j0/N
        d = np.zeros(n, complex)
        d[j0] = 1.0
        H = oracle.fft(d)
        assert np.max(np.abs(np.abs(H) - 1.0 / n)) < 1e-15
        if n > 1:
            ratio = H[1:] / H[:-1]
            assert np.max(np.abs(ratio - np.exp(-2j * np.pi * j0 / n))) < 1e-12
    c = 2.5 - 1.25j
    H = oracle.fft(np.full(n, c))
    ref = np.zeros(n, complex)
    ref[0] = c
    assert np.max(np.abs(H - ref)) < 1e-14


@pytest.mark.parametrize("n", POW2 + [1 << 14, 1 << 16])
def test_tree_fft_matches_library_and_parseval(n):
    f = crand(3, n)
    H = oracle.fft(f)
    assert relerr(H, np.fft.fft(f, axis=-1) / n) < 1e-14
    # Parseval under 1/N: sum |H|^2 = (1/N) sum |f|^2
    np.testing.assert_allclose(np.sum(np.abs(H) ** 2, -1), np.sum(np.abs(f) ** 2, -1) / n, rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64, 256, 1024])
def test_tree_fft_matches_direct_definition(n):
    f = crand(n)
    assert relerr(oracle.fft(f), oracle.dft_direct(f)) < 1e-13


@pytest.mark.parametrize("n", POW2 + [1 << 15])
def test_inverse_section3(n):
    c = crand(2, n)
    f = oracle.ifft(c)
    # eq. (E3): f_j = sum_k c_k e^{+2 pi i jk/N} = N * numpy.ifft
    assert relerr(f, np.fft.ifft(c, axis=-1) * n) < 1e-14
    # round trip: the exponential polynomial p interpolates f at x_j (eq. E3)
    g = crand(n)
    assert relerr(oracle.ifft(oracle.fft(g)), g) < 1e-14


def test_inverse_contrary_order_identity():
    # Section 3: p(2 pi - x_k) = N FFT(c)[k] with the boundary k=0 -> 0 (2 pi periodicity)
    n = 16
    c = crand(n)
    f = oracle.ifft(c)
    G = n * (np.fft.fft(c) / n)
    for k in range(n):
        assert abs(f[(n - k) % n] - G[k]) < 1e-12


def _gold_tree():
    rows = {}
    with open(os.path.join(GOLD, "tree_n8.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                key, *vals = line.split()
                rows[key] = vals
    return rows


def test_worked_example_tree_structure():
    """Paper, Section 2: N=8 leaves in bit-reversed order, and each tree node
    P_r^(n) (a block of 2^n positions after level n) holds the unscaled DFT of
    the data items that node interpolates."""
    g = _gold_tree()
    f = crand(8)
    leaves = [int(v) for v in g["leaves"]]
    np.testing.assert_array_equal(oracle.tree_partial(f, 0), f[leaves])
    for lev in (1, 2, 3):
        out = oracle.tree_partial(f, lev)
        nodes = g["level%d" % lev]
        blk = 1 << lev
        assert len(nodes) * blk == 8
        for pos, node in enumerate(nodes):
            items = [int(v) for v in node.split(":")[1].split(",")]
            ref = np.fft.fft(f[items])
            assert relerr(out[pos * blk:(pos + 1) * blk], ref) < 1e-14
    # each processor's branch (up to level m1 = 1) is the set j = idproc (mod nproc)
    for b in g["branch"]:
        p, items = b.split(":")
        assert sorted(int(v) for v in items.split(",")) == [j for j in range(8) if j % 4 == int(p)]
    # after level m1 the upper half sends to the lower half (nproc_sup = nproc/2)
    assert all(int(s.split(":")[0]) - 2 == int(s.split(":")[1]) for s in g["send"])


def test_oracle_rejects_non_power_of_two():
    with pytest.raises(oracle.OracleError):
        oracle.fft(np.ones(12))
    with pytest.raises(oracle.OracleError):
        oracle.fft2(np.ones((8, 6)))


# ------------------------------------------------------------------ 2D, eq. 5
SHAPES2 = [(1, 1), (1, 8), (8, 1), (2, 2), (4, 8), (8, 4), (16, 32), (32, 16), (32, 32), (64, 128)]


@pytest.mark.parametrize("N,M", SHAPES2)
def test_fft2_eq5_and_inverse(N, M):
    f = crand(2, N, M)
    F = oracle.fft2(f, threads=2)
    # eq. (5) carries 1/N (rows), not 1/(NM)
    assert relerr(F, np.fft.fft2(f) / N) < 1e-14
    # 2D-IDFT carries 1/M: f = (1/M) sum F e^{+...} = (N M / M) numpy.ifft2 = N ifft2
    assert relerr(oracle.ifft2(F, threads=2), f) < 1e-14
    assert relerr(oracle.ifft2(f, threads=2), np.fft.ifft2(f) * N) < 1e-14
    # Parseval under eq. (5): sum |F|^2 = (M/N) sum |f|^2
    np.testing.assert_allclose(np.sum(np.abs(F) ** 2), (M / N) * np.sum(np.abs(f) ** 2), rtol=1e-13)


def test_fft2_separable_rows_then_columns():
    # Section 5: F(x,v) = M FFT_M(row x) then a 1/N FFT down each column
    f = crand(8, 16)
    Fx = np.stack([16 * oracle.fft(r) for r in f])
    F = np.stack([oracle.fft(Fx[:, v]) for v in range(16)], axis=1)
    assert relerr(oracle.fft2(f), F) < 1e-14


def test_fft2_threads_do_not_change_bits():
    f = crand(64, 32)
    np.testing.assert_array_equal(oracle.fft2(f, threads=1), oracle.fft2(f, threads=7))


# ---------------------------------------------------------------- Section 6
@pytest.mark.parametrize("N,M", [(8, 8), (16, 32), (64, 64)])
def test_filter_identities(N, M):
    f = crand(N, M)
    ones = np.ones((N, M))
    assert relerr(oracle.filter2(f, ones, threads=2), f) < 1e-14
    dc = np.zeros((N, M))
    dc[0, 0] = 1.0
    out = oracle.filter2(f, dc, threads=2)
    assert np.max(np.abs(out - f.mean())) < 1e-13
    # a mask that is 1 only at +-(u0, v0) passes exactly that cosine
    u0, v0 = 3 % N, 5 % M
    x, y = np.meshgrid(np.arange(N), np.arange(M), indexing="ij")
    cosw = np.cos(2 * np.pi * (u0 * x / N + v0 * y / M))
    other = np.cos(2 * np.pi * (1 * x / N + 2 * y / M)) + 0.5
    sel = np.zeros((N, M))
    sel[u0, v0] = 1.0
    sel[(-u0) % N, (-v0) % M] = 1.0
    out = oracle.filter2(cosw + other, sel, threads=2)
    assert np.max(np.abs(out - cosw)) < 1e-12


def test_masks_against_fftfreq():
    N, M = 32, 16
    fu = np.fft.fftfreq(N)[:, None]
    fv = np.fft.fftfreq(M)[None, :]
    r2 = fu ** 2 + fv ** 2
    g = oracle.mask_gaussian(N, M, 0.1)
    assert g[0, 0] == 1.0
    np.testing.assert_allclose(g, np.exp(-r2 / 0.02), rtol=1e-13)
    b = oracle.mask_butterworth(N, M, 0.15, 4)
    assert b[0, 0] == 1.0
    np.testing.assert_allclose(b, 1.0 / (1.0 + (r2 / 0.15 ** 2) ** 4), rtol=1e-13)
    # radial and even: H(u,v) = H(-u,-v) (so real images stay real)
    for m in (g, b):
        np.testing.assert_array_equal(m, np.roll(np.flip(m, (0, 1)), (1, 1), (0, 1)))
    # at r = cutoff the Butterworth gain is exactly 1/2
    bb = oracle.mask_butterworth(1, 20, 0.15, 4)  # fftfreq(20)[3] = 0.15
    assert abs(bb[0, 3] - 0.5) < 1e-12


def test_disc_mask_paper_application():
    # Section 6: 512x512 padded image, b = 340, centre = image centre; count the
    # lattice points inside the closed disc with integer arithmetic
    m = oracle.mask_disc(512, 512, 340.0)
    u = np.arange(512)[:, None] - 256
    v = np.arange(512)[None, :] - 256
    inside = (u * u + v * v) <= 340 * 340
    np.testing.assert_array_equal(m == 0.0, inside)
    assert int(inside.sum()) == 512 * 512 - 1997
    assert np.all(oracle.mask_disc(8, 8, 100.0) == 0.0)


# ------------------------------------------------------------ learnable mask
@pytest.mark.parametrize("B,N,M", [(2, 8, 8), (1, 4, 8), (2, 8, 4)])
def test_mask_gradient_exact_finite_differences(B, N, M):
    # L is quadratic in the mask, so central differences are exact up to rounding
    x = rng.standard_normal((B, N, M))
    c = rng.standard_normal((B, N, M))
    m = rng.uniform(0.5, 1.5, (N, M))
    _, L0, g = oracle.loss_grad(x, c, m, threads=1)
    eps = 1e-3
    for (u, v) in [(0, 0), (1, 2), (N - 1, M - 1), (N // 2, M // 2)]:
        mp = m.copy()
        mp[u, v] += eps
        mm = m.copy()
        mm[u, v] -= eps
        Lp = oracle.loss_grad(x, c, mp, threads=1)[1]
        Lm = oracle.loss_grad(x, c, mm, threads=1)[1]
        assert abs((Lp - Lm) / (2 * eps) - g[u, v]) < 1e-11 * max(1.0, abs(g[u, v]))
    # directional derivative along a random direction
    d = rng.standard_normal((N, M))
    Lp = oracle.loss_grad(x, c, m + eps * d, threads=1)[1]
    Lm = oracle.loss_grad(x, c, m - eps * d, threads=1)[1]
    assert abs((Lp - Lm) / (2 * eps) - np.sum(g * d)) < 1e-10 * max(1.0, abs(np.sum(g * d)))


def test_loss_grad_forward_values():
    B, N, M = 2, 8, 16
    x = rng.standard_normal((B, N, M))
    c = rng.standard_normal((B, N, M))
    m = np.ones((N, M))
    y, L, _ = oracle.loss_grad(x, c, m, threads=1)
    # all-ones mask: y = x exactly (round trip), so L = mean (x - c)^2
    assert relerr(y, x) < 1e-14
    assert abs(L - np.mean((x - c) ** 2)) < 1e-12
    m2 = rng.uniform(0, 1, (N, M))
    y2, _, _ = oracle.loss_grad(x, c, m2, threads=1)
    assert relerr(y2, np.fft.ifft2(m2 * np.fft.fft2(x))) < 1e-14


# -------------------------------------------------------------- Section 4
def test_table1_complexity_model():
    with open(os.path.join(GOLD, "table1.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 4
    for N, n2, nlog, pfp, rsp in rows:
        N = int(N)
        m = N.bit_length() - 1
        assert complexity.direct_products(m) == int(n2)
        assert complexity.sequential_products(m) == int(nlog)
        assert complexity.parallel_products(m, 2) == int(pfp)
        assert round(complexity.speedup(m, 2), 2) == float(rsp)
    # the worked example: N=8, nproc=4 -> m=3, m1=1
    assert complexity.parallel_products(3, 0) == complexity.sequential_products(3)


# ------------------------------------------------- Section 6 padding/cropping
def test_pad2_appends_zero_rows_and_columns():
    f = np.arange(460 * 506, dtype=np.float64).reshape(460, 506)
    g = oracle.pad2(f)
    assert g.shape == (512, 512)
    assert np.array_equal(g[:460, :506], f)
    assert not g[460:, :].any() and not g[:, 506:].any()
    h = np.ones((2, 16, 32))
    assert np.array_equal(oracle.pad2(h), h)
    assert [oracle.next_pow2(n) for n in (1, 2, 3, 5, 16, 17, 460)] == [1, 2, 4, 8, 16, 32, 512]


def test_padded_filter_pins():
    rng = np.random.default_rng(21)
    f = rng.standard_normal((2, 13, 20))
    N, M = 16, 32
    # powers of two: nothing to pad, the plain filter
    g = rng.standard_normal((16, 32))
    m = rng.uniform(0, 1, (16, 32))
    assert np.allclose(oracle.filter2_padded(g, m), oracle.filter2(g, m), rtol=0, atol=1e-12)
    # an all-ones mask is the identity on the original region
    assert np.allclose(oracle.filter2_padded(f, np.ones((N, M))), f, rtol=0, atol=1e-12)
    # a DC-only mask gives the mean over the padded N x M array (eq. 5's 1/N,
    # the 2D-IDFT's 1/M)
    dc = np.zeros((N, M))
    dc[0, 0] = 1.0
    out = oracle.filter2_padded(f, dc)
    for b in range(2):
        assert np.allclose(out[b], f[b].sum() / (N * M), rtol=0, atol=1e-12)


def test_padded_spectrum_pins():
    rng = np.random.default_rng(22)
    f = rng.standard_normal((11, 6))
    S = oracle.spectrum_padded(f)
    N, M = 16, 8
    assert S.shape == (N, M)
    assert abs(S[0, 0] - abs(f.sum()) / N) < 1e-12
    # Parseval under eq. 5: sum |F|^2 = (M / N) sum |f|^2 (zeros add nothing)
    assert abs((S ** 2).sum() - M / N * (f ** 2).sum()) < 1e-9 * (f ** 2).sum()
