"""The multidimensional case by tensor product (ORACLE, test infrastructure).

Section 6: T^(2) = T_{n0} (x) T_{n1}.  Images are row-major arrays X[i0, i1]; with the
row-major vectorisation, (T0 (x) T1) vec(X) = vec(T0 X T1^T), i.e. a 1D transform of every
column followed by a 1D transform of every row (the order does not matter).

Eigenvalues (R12): for a separable PSF h = h0 (x) h1 with unit-sum factors the 3-step
algorithm of Section 6 gives the outer product d0 (x) d1 (edge entries use the marginal
1D PSFs, whose symbols at 0 are 1).  The 2D Laplacian (R11) is L0 (x) I + I (x) L1, with
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
