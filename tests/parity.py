"""Tolerances shared by the GPU parity tests.

Float64 vectors (coefficients, restorations, eigenvalues) are compared normwise:
max_i |a_i - b_i| / max_i |b_i| <= 1e-12.

GCV values G_k = N_k / D_k^2 depend on the coefficient vector ghat through
N_k = sum_i sigma_ik^2 |ghat_i|^2.  A normwise perturbation |dghat_i| <= delta max|ghat|
changes G_k by at most kappa_k delta relatively, with
    kappa_k = 2 max|ghat| sum_i sigma_ik^2 |ghat_i| / sum_i sigma_ik^2 |ghat_i|^2,
which is large when G_k is dominated by coefficients far below max|ghat| (noise-level
high frequencies).  Any float64 FFT-based transform carries a normwise error of a few
tens of ulp (delta = 64 eps), so the bound on G_k is 1e-12 + kappa_k delta; kappa_k comes
from the oracle's own quantities only.
"""

import numpy as np

TOL = 1e-12
DELTA = 64 * np.finfo(np.float64).eps


def rel_normwise(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gcv_kappa(ghat, d, s, mus):
    g = np.abs(np.asarray(ghat, dtype=np.complex128))
    d2 = np.abs(np.asarray(d, dtype=np.complex128)) ** 2
    s2 = np.asarray(s, dtype=np.float64) ** 2
    gmax = g.max()
    out = np.empty(len(mus))
    for k, mu in enumerate(mus):
        with np.errstate(divide="ignore", invalid="ignore"):
            sig = np.where(s2 > 0, s2 / (d2 + mu * s2), 0.0)
        w = sig * sig
        out[k] = 2.0 * gmax * np.sum(w * g) / np.sum(w * g * g)
    return out


def assert_gcv_close(G, Gw, ghat_oracle, d, s, mus, what=""):
    G = np.asarray(G)
    Gw = np.asarray(Gw)
    bound = TOL + gcv_kappa(ghat_oracle, d, s, mus) * DELTA
    rel = np.abs(G - Gw) / np.abs(Gw)
    bad = np.nonzero(rel > bound)[0]
    assert bad.size == 0, (what, int(bad[0]), float(rel[bad[0]]), float(bound[bad[0]]))
    return float(np.max(rel))
