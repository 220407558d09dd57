"""Pins of the general 2D eigenvalue routine (oracle.twod.eigs2d_general, Section 6's
three steps) against references that do not use it:

* 2D blurring matrices assembled by brute force from the boundary conditions (each
  boundary condition applied along both axes, then the direct 2D convolution of the
  extended image, one mask tap at a time): the 2D antireflective matrix of a mask even in
  each axis is diagonalised exactly by T_AR (x) T_AR (the antireflective algebra, Section
  3 of the paper's reference ADS08); the 2D reflective matrix of order (n0-2, n1-2) by the
  DCT-II pair, whose eigenvalues are the inner entries for T_C (eq. Ac in each axis); the
  2D periodic matrix of order (n0-2, n1-2) by the DFT pair for any mask (eq. Af);
* the convolution of a basis image t0_i (x) t1_j with the mask at the pixels where the
  mask stays inside the field of view (the eigen relation itself) for edge columns;
* a closed form (the 5-point mask) and the separable case (the outer product of the
  pinned 1D eigenvalues).
"""

import numpy as np
import pytest

from oracle import bc
from oracle import transforms as tr
from oracle import twod
from paper_0906_2704_amd import synth


def _extend(X, m0, m1, rule):
    """Samples outside the field of view by a boundary condition along axis 1, then axis 0
    (the 2D extension of Section 6 is the tensor product of the 1D ones)."""
    if rule == "reflective":
        return np.pad(X, ((m0, m0), (m1, m1)), mode="symmetric")   # f_{1-j} = f_j
    if rule == "periodic":
        return np.pad(X, ((m0, m0), (m1, m1)), mode="wrap")        # f_{1-j} = f_{n+1-j}

    def ar_rows(v, m):  # antireflective along axis 0: f_{1-j} = 2 f_1 - f_{1+j}
        n = v.shape[0]
        out = np.empty((n + 2 * m,) + v.shape[1:])
        out[m:m + n] = v
        for j in range(1, m + 1):
            out[m - j] = 2 * v[0] - v[j]
            out[m + n - 1 + j] = 2 * v[n - 1] - v[n - 1 - j]
        return out
    return ar_rows(ar_rows(X.T, m1).T, m0)


def _blur(X, H, c0, c1, rule):
    """g[p, q] = sum_{a,b} H[a, b] f[p - (a - c0), q - (b - c1)] with f outside the view
    given by ``rule`` (the convolution of eq. mod_cont in 2D)."""
    n0, n1 = X.shape
    m0, m1 = synth.mask_halfwidths(H, c0, c1)
    Xe = _extend(X, m0, m1, rule)
    G = np.zeros((n0, n1), dtype=np.result_type(X, H))
    for a in range(H.shape[0]):
        for b in range(H.shape[1]):
            s0, s1 = m0 - (a - c0), m1 - (b - c1)
            G = G + H[a, b] * Xe[s0:s0 + n0, s1:s1 + n1]
    return G


def _bc_matrix(n0, n1, H, c0, c1, rule):
    A = np.zeros((n0 * n1, n0 * n1))
    for col in range(n0 * n1):
        E = np.zeros(n0 * n1)
        E[col] = 1.0
        A[:, col] = _blur(E.reshape(n0, n1), H, c0, c1, rule).ravel()
    return A


def even_mask(rng, m0, m1):
    """Random mask even in each axis but not separable (rank > 1)."""
    Q = rng.random((m0 + 1, m1 + 1)) + 0.05
    H = np.concatenate([Q[:0:-1], Q])
    H = np.concatenate([H[:, :0:-1], H], axis=1)
    return H / H.sum(), m0, m1


def test_mask_helpers_are_what_they_claim():
    H, c0, c1 = synth.disk_psf(2.5)
    assert twod._even_in_axis(H, c0, 0) and twod._even_in_axis(H, c1, 1)
    assert np.linalg.matrix_rank(H) > 1
    M, a, b = synth.motion_psf(4, 30)
    assert not twod._even_in_axis(M, a, 0) and not twod._even_in_axis(M, b, 1)
    # the extension rules against the 1D brute-force matrices of oracle.bc
    rng = np.random.default_rng(1)
    h, c = rng.random(5), 2
    h /= h.sum()
    for rule, name in (("reflective", "reflective"), ("periodic", "periodic"), ("ar", "antireflective")):
        n = 9
        A1 = bc.blur_matrix_bc(name, n, h, c)
        A = _bc_matrix(1, n, h[None, :], 0, c, rule)
        assert np.abs(A - A1).max() < 1e-15


@pytest.mark.parametrize("n0,n1,mask", [(9, 10, "disk"), (10, 9, "even"), (11, 8, "even2")])
def test_ar_2d_matrix_is_diagonalised_with_3step_eigenvalues(n0, n1, mask):
    rng = np.random.default_rng(n0 * 10 + n1)
    if mask == "disk":
        H, c0, c1 = synth.disk_psf(2.2)
    elif mask == "even":
        H, c0, c1 = even_mask(rng, 2, 3)
    else:
        H, c0, c1 = even_mask(rng, 1, 2)
    assert np.linalg.matrix_rank(H) > 1
    A = _bc_matrix(n0, n1, H, c0, c1, "ar")
    T2 = twod.kron_transform("AR", "AR", n0, n1).astype(np.float64)
    D = twod.eigs2d_general("AR", "AR", n0, n1, H, c0, c1)
    assert D.dtype == np.float64
    assert np.abs(T2 @ np.diag(D.ravel()) @ np.linalg.inv(T2) - A).max() < 1e-13


@pytest.mark.parametrize("n0,n1", [(10, 12), (13, 9)])
def test_TC_inner_entries_are_2d_reflective_of_order_n_minus_2(n0, n1):
    H, c0, c1 = synth.disk_psf(2.9)
    N0, N1 = n0 - 2, n1 - 2
    A_R = _bc_matrix(N0, N1, H, c0, c1, "reflective")
    C = np.kron(tr.dct2_matrix(N0), tr.dct2_matrix(N1)).astype(np.float64)
    M = C @ A_R @ C.T
    assert np.abs(M - np.diag(np.diag(M))).max() < 1e-14
    D = twod.eigs2d_general("C", "C", n0, n1, H, c0, c1)
    assert np.abs(D[1:-1, 1:-1].ravel() - np.diag(M)).max() < 1e-14


@pytest.mark.parametrize("length,angle", [(3, 30), (4, 120), (3, 0)])
def test_TF_inner_entries_are_2d_periodic_of_order_n_minus_2(length, angle):
    """Any mask (here one-sided motion blur): R2 grid /(n-2) and R4 (z(-x)) in both axes."""
    H, c0, c1 = synth.motion_psf(length, angle)
    n0, n1 = 11, 12
    N0, N1 = n0 - 2, n1 - 2
    A_P = _bc_matrix(N0, N1, H, c0, c1, "periodic")
    F = np.kron(tr.dft_matrix(N0), tr.dft_matrix(N1)).astype(np.complex128)
    M = F @ A_P @ F.conj().T
    assert np.abs(M - np.diag(np.diag(M))).max() < 1e-14
    D = twod.eigs2d_general("F", "F", n0, n1, H, c0, c1)
    assert D.dtype == np.complex128
    assert np.abs(D[1:-1, 1:-1].ravel() - np.diag(M)).max() < 1e-14


@pytest.mark.parametrize("kind", ["C", "F", "DST2", "AR"])
def test_edges_act_on_polynomial_times_basis_images(kind):
    """Edge entries: an image that is a preserved polynomial along one axis (degree <= 1;
    the constant for F, whose masks need not be even) times a core column along the other
    is, under the model T2 diag(d) T2^{-1}, multiplied by the edge eigenvalue -- and the
    plain 2D convolution with the mask multiplies it by the same number at every pixel
    where the mask stays inside the view (the eigen relation needs no boundary rule there).
    A bilinear (constant, for F) image gets the corner value sum H."""
    n0, n1 = 14, 13
    if kind == "F":
        H, c0, c1 = synth.motion_psf(4, 60)
    else:
        H, c0, c1 = synth.disk_psf(2.5)
    m0, m1 = synth.mask_halfwidths(H, c0, c1)
    D = twod.eigs2d_general(kind, kind, n0, n1, H, c0, c1)
    T2 = twod.kron_transform(kind, kind, n0, n1).astype(np.complex128)
    A2 = T2 @ np.diag(D.ravel().astype(np.complex128)) @ np.linalg.inv(T2)
    T0 = tr.transform_matrix(kind, n0).astype(np.complex128)
    T1 = tr.transform_matrix(kind, n1).astype(np.complex128)
    poly0, num0, _ = tr.eigen_grid(kind, n0)
    poly1, num1, _ = tr.eigen_grid(kind, n1)
    rng = np.random.default_rng(3)
    slope = 0.0 if kind == "F" else 1.0
    l0 = 0.4 + slope * rng.standard_normal() * np.arange(n0) / n0
    l1 = -0.7 + slope * rng.standard_normal() * np.arange(n1) / n1
    win = (slice(m0, n0 - m0), slice(m1, n1 - m1))
    inner0 = [i for i in range(n0) if not poly0[i] and num0[i] != 0]
    inner1 = [j for j in range(n1) if not poly1[j] and num1[j] != 0]
    cases = [(np.outer(l0, T1[:, j]), D[0, j]) for j in inner1[::3]]
    cases += [(np.outer(T0[:, i], l1), D[i, n1 - 1]) for i in inner0[::3]]
    cases += [(np.outer(l0, l1), H.sum())]
    for X, lam in cases:
        assert np.abs(A2 @ X.ravel() - lam * X.ravel()).max() < 1e-12 * np.abs(X).max()
        G = _blur(X, H, c0, c1, "periodic")   # the rule only matters outside the window
        assert np.abs(G[win] - lam * X[win]).max() < 1e-13 * np.abs(X).max()
    # both edges of a line carry the same value
    assert np.array_equal(D[0], D[-1]) and np.array_equal(D[:, 0], D[:, -1])


def test_five_point_mask_closed_form():
    H = np.array([[0, 1, 0], [1, 4, 1], [0, 1, 0]], dtype=np.float64) / 8.0
    n0, n1 = 12, 9
    D = twod.eigs2d_general("C", "C", n0, n1, H, 1, 1)
    t = np.pi * (np.arange(1, n0 + 1) - 2) / (n0 - 2)
    u = np.pi * (np.arange(1, n1 + 1) - 2) / (n1 - 2)
    inner = (4 + 2 * np.cos(t[1:-1])[:, None] + 2 * np.cos(u[1:-1])[None, :]) / 8.0
    assert np.abs(D[1:-1, 1:-1] - inner).max() < 1e-15
    assert np.abs(D[[0, -1], 1:-1] - (6 + 2 * np.cos(u[1:-1])) / 8.0).max() < 1e-15   # marginal (1, 6, 1)/8
    assert np.abs(D[1:-1, [0, -1]].T - (6 + 2 * np.cos(t[1:-1])) / 8.0).max() < 1e-15
    assert np.all(D[[0, 0, -1, -1], [0, -1, 0, -1]] == 1.0)


@pytest.mark.parametrize("kind,sym", [("C", True), ("AR", True), ("DST3", True), ("F", False)])
def test_separable_mask_gives_outer_product(kind, sym):
    rng = np.random.default_rng(9)
    if sym:
        h0, c0 = synth.gaussian_psf(3, 1.2)
        h1, c1 = synth.box_psf(2)
    else:
        h0, c0 = synth.gaussian_psf(3, 1.2, shift=0.7)
        h1, c1 = rng.random(4), 1
    h1 = h1 * 1.3   # factor sums other than 1
    n0, n1 = 13, 17
    D = twod.eigs2d_general(kind, kind, n0, n1, np.outer(h0, h1), c0, c1)
    S = twod.eigs2d_separable(kind, kind, n0, n1, h0, c0, h1, c1)
    assert np.abs(D - S).max() < 1e-15 * np.abs(S).max() * 4


def test_contract():
    H, c0, c1 = synth.motion_psf(3, 30)
    with pytest.raises(ValueError, match="even"):
        twod.eigs2d_general("C", "C", 12, 12, H, c0, c1)
    with pytest.raises(ValueError, match="both axes"):
        twod.eigs2d_general("C", "F", 12, 12, np.ones((3, 3)) / 9, 1, 1)
    Hd, d0, d1 = synth.disk_psf(4.0)                 # 9 x 9: needs n - 2 >= 9
    with pytest.raises(ValueError, match="too wide"):
        twod.eigs2d_general("C", "C", 10, 20, Hd, d0, d1)
    twod.eigs2d_general("C", "C", 11, 11, Hd, d0, d1)
