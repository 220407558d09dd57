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
