"""Pins of the degree-3 transform for any PSF (kind "F3", a reading: the paper defines no
degree-3 transform).  What fixes it: its columns are T_F's except the frequency +-1 pair;
the columns with eigenvalue z(0) span all cubics, so the model A = T diag(d) T^{-1}
multiplies every sampled cubic by sum h (for any PSF, as T_F does for quadratics); the
cosine column is an exact eigenvector of the convolution with a symmetric PSF away from
the boundary, with eigenvalue z(x_1); real signals have real coefficients on the two new
columns and conjugate pairs elsewhere; the model restores noise-free cubics exactly."""

import numpy as np
import pytest

from oracle import tikhonov as tk
from oracle import transforms as tr


def rand_psf(rng, m, center):
    h = rng.random(2 * m + 1) + 0.05
    return h / h.sum(), center


@pytest.mark.parametrize("n", [7, 12, 33])
def test_structure(n):
    T3 = tr.transform_matrix("F3", n).astype(np.complex128)
    TF = tr.transform_matrix("F", n).astype(np.complex128)
    keep = [c for c in range(n) if c not in (2, n - 2)]
    assert np.array_equal(T3[:, keep], TF[:, keep])
    N = n - 2
    x = 2 * np.pi * (np.arange(1, n + 1) - 2) / N
    assert np.abs(T3[:, 2] - np.sqrt(2.0 / N) * np.cos(x)).max() < 1e-15
    c = x * (x - np.pi) * (x - 2 * np.pi)
    assert np.abs(T3[:, n - 2] - c / np.linalg.norm(c)).max() < 1e-15
    assert np.linalg.cond(T3) < 1e4


@pytest.mark.parametrize("n", [9, 24, 50])
def test_cubics_are_multiplied_by_z0_for_any_psf(n):
    rng = np.random.default_rng(n)
    h, c = rand_psf(rng, 2, 1)           # one-sided, nonsymmetric
    h = h * 1.7                           # sum h != 1
    A3 = tr.blur_matrix("F3", n, h, c).astype(np.complex128)
    AF = tr.blur_matrix("F", n, h, c).astype(np.complex128)
    x = np.arange(n, dtype=np.float64)
    for deg in range(4):
        f = np.polyval(rng.standard_normal(deg + 1), x / n)
        assert np.abs(A3 @ f - h.sum() * f).max() < 1e-12 * np.abs(f).max()
    cubic = (x / n) ** 3
    assert np.abs(AF @ cubic - h.sum() * cubic).max() > 1e-6   # T_F keeps quadratics only


def test_cosine_column_eigen_relation_for_symmetric_psf():
    n = 40
    N = n - 2
    h = np.array([1.0, 3.0, 5.0, 3.0, 1.0]) / 13.0
    c = 2
    d = tr.blur_eigs("F3", n, h, c)
    col = tr.transform_matrix("F3", n)[:, 2].real.astype(np.float64)
    g = np.convolve(col, h, mode="valid")          # rows c .. n-1-c, away from the boundary
    assert np.abs(g - d[2].real * col[c:n - c]).max() < 1e-15
    z1 = np.sum(h * np.cos(2 * np.pi / N * (np.arange(5) - c)))
    assert abs(d[2] - z1) < 1e-15 and d[2].imag == 0
    assert d[n - 2] == pytest.approx(1.0, abs=1e-15) and d[0] == d[-1] == pytest.approx(1.0, abs=1e-15)


def test_real_signals_and_eigenvalue_pairs():
    n = 30
    rng = np.random.default_rng(3)
    h, c = rand_psf(rng, 3, 2)
    y = rng.standard_normal(n)
    xh = tr.inverse("F3", y)
    assert abs(xh[2].imag) < 1e-13 and abs(xh[n - 2].imag) < 1e-13
    N = n - 2
    # remaining core pairs (frequencies k and N - k, k = 2 .. N-2): conjugate
    for k in range(2, N // 2 + 1):
        assert abs(xh[1 + k] - np.conj(xh[1 + N - k])) < 1e-12
    d = tr.blur_eigs("F3", n, h, c)
    for k in range(2, N // 2 + 1):
        assert abs(d[1 + k] - np.conj(d[1 + N - k])) < 1e-14
    s = tr.smooth_eigs("F3", n, "D2")
    fc = tr.forward("F3", tk.tikhonov_filter(xh, d, s, 1e-2))   # complex arithmetic
    assert np.abs(fc.imag).max() < 1e-12 * np.abs(fc.real).max()


@pytest.mark.parametrize("mu", [1e-4, 1e-1])
def test_noise_free_cubic_restored_exactly(mu):
    n = 48
    rng = np.random.default_rng(11)
    h, c = rand_psf(rng, 4, 3)
    x = np.linspace(0.0, 1.0, n)
    P = np.polyval(rng.standard_normal(4), x)
    f = tk.restore_spectral("F3", P, h, c, "D2", mu)
    assert np.abs(f - P).max() < 1e-11 * np.abs(P).max()
    s = tr.smooth_eigs("F3", n, "D2")
    assert s[n - 2] == 0 and s[2] == pytest.approx(2 - 2 * np.cos(2 * np.pi / (n - 2)), abs=1e-15)
