"""Reblurred Tikhonov filtering and the GCV choice of mu (ORACLE, test infrastructure).

Section 4 of the paper.  With A = T diag(d) T^{-1}, A' = T diag(conj d) T^{-1} (the PSF
rotated by 180 degrees) and L = T diag(s) T^{-1}:

* eq. nerebl  (A'A + mu L'L) f_reg = A' g
* eq. freg    f_reg = T Phi D^{-1} T^{-1} g, Phi_i = |d_i|^2 / (|d_i|^2 + mu |s_i|^2),
              evaluated as conj(d_i) ghat_i / (|d_i|^2 + mu |s_i|^2) (R5: no 0/0 where d_i=0)
* eqs. gcv2 / mugcv  G(mu) = sum_i |sigma_i ghat_i|^2 / (sum_i sigma_i)^2,
              sigma_i = |s_i|^2 / (|d_i|^2 + mu |s_i|^2), ghat = T^{-1} g; mu_GCV is the
              minimiser over the caller's grid, the first one on ties (R9), and the modulus
              is taken for complex coefficients (R6).
* eq. gcv     the exact functional ||g - A f_reg||^2 / trace(I - A T Phi D^{-1} T^{-1})^2.
              The residual is g - A f_reg = T (I - Phi) ghat (eq. gcnum before its
              approximation) and the trace is sum_i (1 - Phi_i) = mu sum_i sigma_i (R8), so
              eq. gcv = ||T (sigma ghat)||^2 / (sum_i sigma_i)^2: eq. gcv2 with the norm of
              T applied to sigma ghat instead of the norm of sigma ghat (``gcv_exact_values``).
"""

import numpy as np
import scipy.linalg as sla

from . import transforms as tr

LD = np.longdouble


def tikhonov_filter(ghat, d, s, mu):
    """fhat = Phi D^{-1} ghat of eq. freg, long-double evaluation."""
    ghat = np.asarray(ghat)
    cplx = np.iscomplexobj(ghat) or np.iscomplexobj(d)
    gl = ghat.astype(np.clongdouble if cplx else LD)
    dl = np.asarray(d).astype(np.clongdouble if np.iscomplexobj(d) else LD)
    sl = np.asarray(s).astype(LD)
    den = (dl * np.conj(dl)).real + LD(mu) * sl * sl
    out = np.conj(dl) * gl / den
    return out.astype(np.complex128 if cplx else np.float64)


def gcv_values(ghat, d, s, mus, wide=True):
    """G(mu_k) for every mu_k of the grid (eq. mugcv), long-double sums (float64 sums with
    wide=False, for million-entry images)."""
    R, C = (LD, np.clongdouble) if wide else (np.float64, np.complex128)
    gl = np.asarray(ghat).astype(C)
    dl = np.asarray(d).astype(C)
    s2 = np.asarray(s).astype(R) ** 2
    d2 = (dl * np.conj(dl)).real
    g2 = (gl * np.conj(gl)).real
    out = np.empty(len(mus), dtype=np.float64)
    for k, mu in enumerate(mus):
        sigma = s2 / (d2 + R(mu) * s2)
        out[k] = np.float64(np.sum(sigma * sigma * g2) / np.sum(sigma) ** 2)
    return out


def gcv_exact_values(kind, ghat, d, s, mus):
    """Eq. gcv for every mu_k of the grid: ||T (sigma ghat)||^2 / (sum_i sigma_i)^2 with the
    dense transform T of the kind (long double), i.e. the exact residual norm of eq. gcnum
    instead of its approximation, on the same scale as ``gcv_values`` (the factors mu^2 of
    numerator and denominator cancel).  1D, any kind; O(n^2) per grid value."""
    n = len(ghat)
    T = tr.transform_matrix(kind, n).astype(np.clongdouble)
    gl = np.asarray(ghat).astype(np.clongdouble)
    dl = np.asarray(d).astype(np.clongdouble)
    s2 = np.asarray(s).astype(LD) ** 2
    d2 = (dl * np.conj(dl)).real
    out = np.empty(len(mus), dtype=np.float64)
    for k, mu in enumerate(mus):
        sigma = s2 / (d2 + LD(mu) * s2)
        r = T @ (sigma * gl)
        out[k] = np.float64(np.sum((r * np.conj(r)).real) / np.sum(sigma) ** 2)
    return out


def gcv_argmin(G):
    """Index of the first minimum of G; raises on a non-finite value (R9)."""
    G = np.asarray(G)
    if not np.all(np.isfinite(G)):
        raise FloatingPointError("non-finite GCV value")
    return int(np.argmin(G))  # numpy returns the first occurrence


def gcv_scan(ghat, d, s, mus):
    G = gcv_values(ghat, d, s, mus)
    k = gcv_argmin(G)
    return G, k, float(mus[k])


def restore_spectral(kind, g, h, center, norm, mu):
    """f_reg by eq. freg: T^{-1} g, filter, T (dense transforms with refinement)."""
    n = len(g)
    d = tr.blur_eigs(kind, n, h, center)
    s = tr.smooth_eigs(kind, n, norm)
    ghat = tr.inverse(kind, g)
    f = tr.forward(kind, tikhonov_filter(ghat, d, s, mu))
    return f.real if not np.iscomplexobj(g) else f


def solve_normal_equations(A, Ap, L, g, mu):
    """f with (A'A + mu L'L) f = A' g (eq. nerebl), dense LU + long-double refinement."""
    A = np.asarray(A)
    Ap = np.asarray(Ap)
    L = np.asarray(L)
    M = Ap @ A + LD(mu) * (L @ L)
    rhs = Ap @ np.asarray(g).astype(M.dtype)
    cplx = np.iscomplexobj(M)
    lu = sla.lu_factor(M.astype(np.complex128 if cplx else np.float64))
    x = sla.lu_solve(lu, rhs.astype(np.complex128 if cplx else np.float64)).astype(M.dtype)
    for _ in range(3):
        r = rhs - M @ x
        x = x + sla.lu_solve(lu, r.astype(np.complex128 if cplx else np.float64)).astype(M.dtype)
    return x


def restore_normal_equations(kind, g, h, center, norm, mu):
    """f_reg by assembling A, A' (PSF rotated 180 degrees) and L densely (eq. nerebl).

    Here L' = L because s is real; the rotated PSF has taps h_{-j}."""
    n = len(g)
    h = np.asarray(h, dtype=np.float64)
    A = tr.blur_matrix(kind, n, h, center)
    Ap = tr.blur_matrix(kind, n, h[::-1], h.size - 1 - center)
    L = tr.smoothing_matrix(kind, n, norm)
    f = solve_normal_equations(A, Ap, L, g, mu)
    return f


def exact_gcv(kind, g, h, center, norm, mu):
    """Eq. gcv evaluated densely (diagnostic only)."""
    n = len(g)
    T = tr.transform_matrix(kind, n)
    A = tr.blur_matrix(kind, n, h, center)
    d = tr.blur_eigs(kind, n, h, center).astype(np.clongdouble)
    s = tr.smooth_eigs(kind, n, norm).astype(LD)
    Tinv = tr._dense_inverse(kind, n)
    phi_dinv = np.conj(d) / ((d * np.conj(d)).real + LD(mu) * s * s)
    H = A @ (T * phi_dinv[None, :]) @ Tinv
    f = tr.forward(kind, tikhonov_filter(tr.inverse(kind, g), tr.blur_eigs(kind, n, h, center),
                                         tr.smooth_eigs(kind, n, norm), mu))
    res = np.asarray(g).astype(np.clongdouble) - A @ f.astype(np.clongdouble)
    num = np.sum((res * np.conj(res)).real)
    tr_ = np.trace(np.eye(n) - H)
    return float(num / (tr_ * np.conj(tr_)).real)
