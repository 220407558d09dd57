"""The multidimensional case by tensor product (ORACLE, test infrastructure).

Section 6: T^(2) = T_{n0} (x) T_{n1}.  Images are row-major arrays X[i0, i1]; with the
row-major vectorisation, (T0 (x) T1) vec(X) = vec(T0 X T1^T), i.e. a 1D transform of every
column followed by a 1D transform of every row (the order does not matter).

Eigenvalues (R12, R20): ``eigs2d_general`` follows the 3-step algorithm of Section 6 for
any mask; for a separable PSF h = h0 (x) h1 it reduces to the outer product d0 (x) d1 of
``eigs2d_separable`` (edge entries use the marginal 1D PSFs, whose symbols at 0 are the
factors' sums).  The 2D Laplacian (R11) is L0 (x) I + I (x) L1, with
spectrum s0_i + s1_j; L = I has s = 1.
"""

import numpy as np

from . import transforms as tr
from . import tikhonov as tk


def forward2d(kind0, kind1, X, wide=True):
    """wide=False: float64 products (large images)."""
    fwd = tr.forward if wide else tr.forward_f64
    Y = fwd(kind1, X)                   # rows (axis 1)
    return fwd(kind0, Y.T).T            # columns (axis 0)


def inverse2d(kind0, kind1, Y, refine_steps=3):
    """refine_steps=0: plain float64 LU solves (large images)."""
    X = tr.inverse(kind1, Y, refine_steps)
    return tr.inverse(kind0, X.T, refine_steps).T


def eigs2d_separable(kind0, kind1, n0, n1, h0, c0, h1, c1):
    d0 = tr.blur_eigs(kind0, n0, h0, c0)
    d1 = tr.blur_eigs(kind1, n1, h1, c1)
    return np.multiply.outer(d0, d1)


def _even_in_axis(H, c, axis):
    """True when the mask H (tap offset index - c along ``axis``) is even along that axis."""
    H = np.moveaxis(np.asarray(H, dtype=np.float64), axis, 0)
    m = max(c, H.shape[0] - 1 - c)
    full = np.zeros((2 * m + 1,) + H.shape[1:])
    full[m - c:m - c + H.shape[0]] = H
    return bool(np.array_equal(full, full[::-1]))


def eigs2d_general(kind0, kind1, n0, n1, H, c0, c1):
    """Eigenvalues d[i, j] for a general (non-separable) 2D PSF mask, in the basis
    T_{n0} (x) T_{n1}, by the three steps of Section 6.

    H[a, b] is the tap at offset (a - c0, b - c1) (axis 0 first).
      1. Marginal 1D masks: h0 = the sum of the columns of H (a vector along axis 0) and
         h1 = the sum of its rows (along axis 1).
      2. Edges: the 1D eigenvalues of h0 on axis 0 fill the columns j whose axis-1 basis
         vector is a preserved polynomial (the vertical edges of the array), those of h1 on
         axis 1 the rows i with a polynomial axis-0 vector (the horizontal edges); the four
         corners are sum H either way.
      3. Inner entries: the 2D transform of the mask at the two axes' grid frequencies --
         for the real kinds the 2D cosine sum, sum H[a,b] cos((a-c0) t_i) cos((b-c1) u_j),
         for F the 2D Fourier sum at (-t_i, -u_j) (the convolution model, as in 1D).
    Real kinds need H even in each axis (ValueError otherwise, as for 1D masks), so that
    products of per-axis cosine columns are eigenvectors; both axes must be real or both
    complex.  Width: 2 m_a + 1 <= n_a - 2 per axis (checked by the 1D routine).
    Products in long double with exactly reduced angles."""
    H = np.asarray(H, dtype=np.float64)
    if H.ndim != 2:
        raise ValueError("H must be a 2D mask")
    cplx = tr.is_complex(kind0)
    if cplx != tr.is_complex(kind1):
        raise ValueError("both axes real or both complex")
    if not cplx and not (_even_in_axis(H, c0, 0) and _even_in_axis(H, c1, 1)):
        raise ValueError("real kinds need a mask even in each axis")
    HL = H.astype(tr.LD)
    # step 1
    h0 = np.sum(HL, axis=1).astype(np.float64)
    h1 = np.sum(HL, axis=0).astype(np.float64)
    # step 2
    d0 = tr.blur_eigs(kind0, n0, h0, c0)
    d1 = tr.blur_eigs(kind1, n1, h1, c1)
    # step 3
    poly0, num0, den0 = tr.eigen_grid(kind0, n0)
    poly1, num1, den1 = tr.eigen_grid(kind1, n1)
    if cplx:
        num0, num1 = -num0, -num1
    k0 = np.arange(H.shape[0], dtype=np.int64) - int(c0)
    k1 = np.arange(H.shape[1], dtype=np.int64) - int(c1)
    C0, S0 = tr.cos_sin_pi(np.outer(num0, k0), den0)
    C1, S1 = tr.cos_sin_pi(np.outer(num1, k1), den1)
    if cplx:
        E0 = C0.astype(tr.CLD) + 1j * S0.astype(tr.CLD)
        E1 = C1.astype(tr.CLD) + 1j * S1.astype(tr.CLD)
        D = (E0 @ HL.astype(tr.CLD) @ E1.T).astype(np.complex128)
    else:
        D = (C0 @ HL @ C1.T).astype(np.float64)
    D[:, poly1] = d0[:, None]
    D[poly0, :] = d1[None, :]
    return D


def gcv2d_exact_values(kind0, kind1, ghat, d, s, mus, wide=True):
    """Eq. gcv for an image: ||T^(2) (sigma ghat)||^2 / (sum sigma)^2 per grid value, the
    residual norm of eq. gcnum with T^(2) = T_{n0} (x) T_{n1} applied exactly (long-double
    products; float64 products with wide=False, for large images), on the scale of eq. gcv2
    (the factors mu^2 cancel; R21 in 2D)."""
    ghat = np.asarray(ghat)
    d = np.asarray(d)
    s2 = np.asarray(s, dtype=np.float64) ** 2
    d2 = np.abs(d) ** 2
    out = np.empty(len(mus), dtype=np.float64)
    for k, mu in enumerate(mus):
        sigma = s2 / (d2 + mu * s2)
        Y = forward2d(kind0, kind1, sigma * ghat, wide=wide)
        out[k] = np.sum(np.abs(Y) ** 2) / np.sum(sigma) ** 2
    return out


def smooth2d(kind0, kind1, n0, n1, norm):
    if norm == "I":
        return np.ones((n0, n1))
    s0 = tr.smooth_eigs(kind0, n0, "D2")
    s1 = tr.smooth_eigs(kind1, n1, "D2")
    return np.add.outer(s0, s1)


def kron_transform(kind0, kind1, n0, n1):
    """Full (n0 n1) x (n0 n1) Kronecker matrix (tiny sizes only)."""
    return np.kron(tr.transform_matrix(kind0, n0), tr.transform_matrix(kind1, n1))


def restore2d(kind0, kind1, G, h0, c0, h1, c1, norm, mu):
    n0, n1 = G.shape
    d = eigs2d_separable(kind0, kind1, n0, n1, h0, c0, h1, c1)
    s = smooth2d(kind0, kind1, n0, n1, norm)
    ghat = inverse2d(kind0, kind1, G)
    fhat = tk.tikhonov_filter(ghat, d, s, mu)
    f = forward2d(kind0, kind1, fhat)
    return f.real if np.iscomplexobj(f) else f


def gcv2d(kind0, kind1, G, h0, c0, h1, c1, norm, mus):
    n0, n1 = G.shape
    d = eigs2d_separable(kind0, kind1, n0, n1, h0, c0, h1, c1)
    s = smooth2d(kind0, kind1, n0, n1, norm)
    ghat = inverse2d(kind0, kind1, G)
    return tk.gcv_scan(ghat.ravel(), d.ravel(), s.ravel(), mus)
