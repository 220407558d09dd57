"""Pins of the exact GCV functional (eq. gcv, oracle.tikhonov.gcv_exact_values) against
routes that do not use its T (sigma ghat) form:

* antireflective: ||g - A f||^2 / trace(I - A (A A + mu L L)^{-1} A)^2 with A assembled
  from the boundary rule (symmetric PSF: the reblurring matrix is A itself) and L the
  second-difference matrix of eq. L -- no transform at all;
* every kind of the paper and the DST family: the dense evaluation of eq. gcv as printed
  (A = T D T^{-1}, the trace of the dense influence matrix, f_reg by the transforms);
* periodic and reflective bases are unitary, so eq. gcv equals eq. gcv2 there (the
  statement of Section 4.2 for A_P and A_R).
"""

import numpy as np
import pytest

from oracle import bc
from oracle import tikhonov as tk
from oracle import transforms as tr


def rand_sym_psf(rng, m):
    h = rng.random(m + 1) + 0.1
    full = np.concatenate([h[:0:-1], h])
    return full / full.sum(), m


@pytest.mark.parametrize("norm", ["I", "D2"])
@pytest.mark.parametrize("n", [17, 40])
def test_antireflective_exact_gcv_from_boundary_matrices(norm, n):
    rng = np.random.default_rng(n)
    h, c = rand_sym_psf(rng, 3)
    g = rng.standard_normal(n)
    A = bc.blur_matrix_bc("antireflective", n, h, c)
    L = bc.second_difference_ar(n) if norm == "D2" else np.eye(n)
    mus = [1e-4, 3e-3, 0.1, 2.0]
    G = tk.gcv_exact_values("AR", tr.inverse("AR", g), tr.blur_eigs("AR", n, h, c), tr.smooth_eigs("AR", n, norm), mus)
    for k, mu in enumerate(mus):
        M = A @ A + mu * (L @ L)
        f = np.linalg.solve(M, A @ g)
        H = A @ np.linalg.solve(M, A)
        ref = np.sum((g - A @ f) ** 2) / np.trace(np.eye(n) - H) ** 2
        assert abs(G[k] - ref) < 1e-9 * ref, (mu, G[k], ref)


@pytest.mark.parametrize("kind", ["C", "F", "AR", "DST2", "DST3"])
def test_exact_gcv_equals_dense_eq_gcv(kind):
    n = 24
    rng = np.random.default_rng(3)
    if kind == "F":
        h, c = rng.random(6) + 0.05, 2
        h /= h.sum()
    else:
        h, c = rand_sym_psf(rng, 3)
    g = rng.standard_normal(n)
    for norm in ("I", "D2"):
        d = tr.blur_eigs(kind, n, h, c)
        s = tr.smooth_eigs(kind, n, norm)
        mus = [1e-3, 5e-2]
        G = tk.gcv_exact_values(kind, tr.inverse(kind, g), d, s, mus)
        for k, mu in enumerate(mus):
            ref = tk.exact_gcv(kind, g, h, c, norm, mu)
            assert abs(G[k] - ref) < 1e-9 * ref, (kind, norm, mu)


@pytest.mark.parametrize("kind", ["P", "R"])
def test_exact_equals_approximation_for_unitary_bases(kind):
    n = 20
    rng = np.random.default_rng(8)
    h, c = rand_sym_psf(rng, 2)
    ghat = tr.inverse(kind, rng.standard_normal(n))
    d = tr.blur_eigs(kind, n, h, c)
    s = tr.smooth_eigs(kind, n, "D2")
    s = np.where(s == 0, 1.0, s)   # keep sigma finite where the Laplacian vanishes
    mus = [1e-3, 1e-1]
    assert np.allclose(tk.gcv_exact_values(kind, ghat, d, s, mus), tk.gcv_values(ghat, d, s, mus), rtol=1e-12)


def test_exact_differs_from_approximation_for_tc():
    """T_C is not unitary, so eq. gcv and its approximation differ (not a pin: the size of
    the difference on one seeded case)."""
    n = 64
    rng = np.random.default_rng(1)
    h, c = rand_sym_psf(rng, 4)
    ghat = tr.inverse("C", rng.standard_normal(n))
    d = tr.blur_eigs("C", n, h, c)
    s = np.ones(n)
    mus = np.logspace(-6, 0, 16)
    Ge = tk.gcv_exact_values("C", ghat, d, s, mus)
    Ga = tk.gcv_values(ghat, d, s, mus)
    assert np.max(np.abs(Ge / Ga - 1)) > 1e-3


# ------------------------------------------------------------------------------- 2D

def _ar_extend(X, m):
    def rows(v):
        n = v.shape[0]
        out = np.empty((n + 2 * m,) + v.shape[1:])
        out[m:m + n] = v
        for j in range(1, m + 1):
            out[m - j] = 2 * v[0] - v[j]
            out[m + n - 1 + j] = 2 * v[n - 1] - v[n - 1 - j]
        return out
    return rows(rows(X.T).T)


@pytest.mark.parametrize("norm", ["I", "D2"])
def test_2d_antireflective_exact_gcv_from_boundary_matrices(norm):
    """2D eq. gcv of a separable even PSF against the 2D antireflective blurring matrix
    assembled pixel by pixel from the boundary rule, with the Laplacian L0 (x) I + I (x) L1
    of eq. L, by dense solves (no transform)."""
    from oracle import twod
    n0, n1, m = 7, 8, 2
    rng = np.random.default_rng(12)
    h0, c0 = rand_sym_psf(rng, m)
    h1, c1 = rand_sym_psf(rng, m)
    N = n0 * n1
    A = np.zeros((N, N))
    for col in range(N):
        E = np.zeros(N)
        E[col] = 1.0
        Xe = _ar_extend(E.reshape(n0, n1), m)
        G = np.zeros((n0, n1))
        for a in range(2 * m + 1):
            for b in range(2 * m + 1):
                s0, s1 = m - (a - c0), m - (b - c1)   # g[p, q] += h0_a h1_b f[p - (a-c0), q - (b-c1)]
                G += h0[a] * h1[b] * Xe[s0:s0 + n0, s1:s1 + n1]
        A[:, col] = G.ravel()
    if norm == "D2":
        L = np.kron(bc.second_difference_ar(n0), np.eye(n1)) + np.kron(np.eye(n0), bc.second_difference_ar(n1))
    else:
        L = np.eye(N)
    g = rng.standard_normal((n0, n1))
    D = twod.eigs2d_separable("AR", "AR", n0, n1, h0, c0, h1, c1)
    S = twod.smooth2d("AR", "AR", n0, n1, norm)
    ghat = twod.inverse2d("AR", "AR", g)
    mus = [1e-3, 0.05, 1.0]
    Gx = twod.gcv2d_exact_values("AR", "AR", ghat, D, S, mus)
    gv = g.ravel()
    for k, mu in enumerate(mus):
        M = A @ A + mu * (L @ L)
        f = np.linalg.solve(M, A @ gv)
        H = A @ np.linalg.solve(M, A)
        ref = np.sum((gv - A @ f) ** 2) / np.trace(np.eye(N) - H) ** 2
        assert abs(Gx[k] - ref) < 1e-9 * ref, (mu, Gx[k], ref)


@pytest.mark.parametrize("kind", ["P", "R"])
def test_2d_exact_equals_approximation_for_unitary_bases(kind):
    from oracle import twod
    n0, n1 = 9, 10
    rng = np.random.default_rng(2)
    ghat = twod.inverse2d(kind, kind, rng.standard_normal((n0, n1)))
    h, c = rand_sym_psf(rng, 2)
    D = twod.eigs2d_separable(kind, kind, n0, n1, h, c, h, c)
    S = twod.smooth2d(kind, kind, n0, n1, "I")
    mus = [1e-3, 1e-1]
    assert np.allclose(twod.gcv2d_exact_values(kind, kind, ghat, D, S, mus),
                       tk.gcv_values(ghat.ravel(), D.ravel(), S.ravel(), mus), rtol=1e-12)


def test_2d_exact_of_a_row_image_is_the_1d_functional_scaled():
    """Separability check: an image whose coefficients live on the constant axis-0 column
    of T_C (index 1) reduces to the 1D functional of axis 1 times the squared norm of that
    column (the trace sums only over the entries that are not masked)."""
    from oracle import twod
    n0, n1 = 8, 11
    rng = np.random.default_rng(4)
    g1 = tr.inverse("C", rng.standard_normal(n1))
    ghat = np.zeros((n0, n1))
    ghat[1] = g1
    D = np.ones((n0, n1))
    D[1] = rng.random(n1) + 0.2
    S = np.zeros((n0, n1))
    S[1] = 1.0
    mus = [1e-2, 0.3]
    col = tr.transform_matrix("C", n0)[:, 1].astype(np.float64)
    G2 = twod.gcv2d_exact_values("C", "C", ghat, D, S, mus)
    G1 = tk.gcv_exact_values("C", g1, D[1], S[1], mus)
    assert np.allclose(G2, G1 * np.sum(col ** 2), rtol=1e-12)
