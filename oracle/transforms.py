"""Dense transforms and spectra of the high-order boundary condition models (ORACLE).

Test infrastructure: only the tests, the smoke check and the CPU-baseline leg of the
benchmark may use this module.

Notation (1-based as in the paper): n = signal length, N = n - 2 = order of the
trigonometric core, PSF taps h_j, symbol z(t) = sum_j h_j e^{i j t} (eq. symbol).

Kinds of transform built here, every entry from its defining formula, with every angle
reduced exactly as an integer multiple of pi before the trigonometric call:

* ``"AR"``   antireflective transform T = [p | Q padded with zero rows | Jp]      (eq. ART)
* ``"C"``    T_C: quadratic q, Jq and the cosine columns on the extended grid     (eq. Tc)
* ``"F"``    T_F: quadratic q, Jq and the exponential columns on the extended grid (eq. Tf)
* ``"DST2"``, ``"DST3"``  degree-2 / degree-3 extension of the antireflective transform:
             the lowest d-1 sine columns are replaced by unit-norm polynomial "bubbles"
             vanishing at both ends (the paper's conclusion suggests higher order
             boundary conditions; this construction is the reading adopted for degree 3)
* ``"P"``, ``"R"``  periodic F^(n) and reflective C^(n) bases of order n (eqs. permat,
             refm), used as comparators and to pin the GCV formula.
* ``"F3"``   degree 3 for any PSF (not in the paper; the reading adopted here): T_F with
             its conjugate pair of frequency +-1 (columns 3 and n-1, 1-based) replaced by
             two real columns, sqrt(2) cos x / sqrt(N) (the pair's real part) and the
             unit-norm samples of the cubic x (x - pi)(x - 2 pi) on the extended grid, so
             that the columns with eigenvalue z(0) span all cubics.  The cosine column
             carries Re z(x_1) (the part of the mask even about its centre, as for the real
             kinds), the cubic z(0).

A kind's matrix T has the eigenvectors of the blurring matrix A = T diag(d) T^{-1} as
columns; ``blur_eigs`` returns d and ``smooth_eigs`` the spectrum s of the smoothing
operator L = T diag(s) T^{-1} (Section 4, eq. L and the definitions of L_C, L_F).

Readings of the paper taken here (each is tested):
* R1  p is normalised to unit 2-norm: the printed factor sqrt(n(2n-1)/(6(n-1))) is the
      norm of (1 - (i-1)/(n-1))_i, so p divides by it (eq. ART says ||p||_2 = 1).
* R2  the core grid of A_F is 2 pi (i-2)/(n-2) (the circulant of order n-2), not /n.
* R4  with the convolution model g_i = sum_j h_j f_{i-j} the exponential columns
      e^{i k x} carry the eigenvalue z(-k 2pi/N) = conj(z(k 2pi/N)) for a real PSF; this
      is what the paper's first-column formula for eq. permat gives.
* R7  the eigenvalue of the preserved polynomials is z(0) = sum_j h_j.
"""

from fractions import Fraction
from functools import lru_cache

import numpy as np
import scipy.linalg as sla

LD = np.longdouble
CLD = np.clongdouble
PI = 4 * np.arctan(LD(1))

KINDS = ("AR", "C", "F", "DST2", "DST3", "P", "R", "F3")
COMPLEX_KINDS = ("F", "P", "F3")


def degree_of(kind):
    """Degree of the polynomials the model preserves with eigenvalue z(0)."""
    return {"AR": 1, "C": 2, "F": 2, "DST2": 2, "DST3": 3, "P": 0, "R": 0, "F3": 3}[kind]


def is_complex(kind):
    return kind in COMPLEX_KINDS


def cos_sin_pi(num, den):
    """cos and sin of pi*num/den in long double, num reduced exactly modulo 2*den."""
    r = np.mod(np.asarray(num, dtype=np.int64), 2 * den)
    ang = PI * r.astype(LD) / LD(den)
    return np.cos(ang), np.sin(ang)


def _unit(v):
    v = np.asarray(v, dtype=LD)
    return v / np.sqrt(np.sum(v * v))


# ----------------------------------------------------------------------------------------
# the preserved-polynomial columns
# ----------------------------------------------------------------------------------------

def ar_p(n):
    """p of eq. ART: p_i = (1 - (i-1)/(n-1)) / sqrt(n(2n-1)/(6(n-1))), i = 1..n (R1)."""
    i = np.arange(1, n + 1, dtype=np.int64)
    raw = LD(1) - (i - 1).astype(LD) / LD(n - 1)
    return raw / np.sqrt(LD(n * (2 * n - 1)) / LD(6 * (n - 1)))


def _extended_grid_over_pi(kind, n):
    """Grid points x_i / pi, i = 0..n-1, and the interval end b / pi (exact rationals).

    C: x_i = (2i-1) pi / (2n-4), b = (2n-3) pi / (2n-4)            (eqs. ints, points)
    F: x_i = (i-1) 2 pi / (n-2), b = 2 pi                            (eqs. intn, pointn)
    """
    if kind == "C":
        xs = [Fraction(2 * i - 1, 2 * n - 4) for i in range(n)]
        b = Fraction(2 * n - 3, 2 * n - 4)
    elif kind == "F":
        xs = [Fraction(2 * (i - 1), n - 2) for i in range(n)]
        b = Fraction(2)
    else:
        raise ValueError(kind)
    return xs, b


def quad_q(kind, n):
    """q = q~/||q~||, q~_{i+1} = (b - x_i)^2, i = 0..n-1, on the kind's extended grid."""
    xs, b = _extended_grid_over_pi(kind, n)
    # the common factor pi^2 cancels in the normalisation
    qt = [(b - x) * (b - x) for x in xs]
    return _unit(np.array([LD(fr.numerator) / LD(fr.denominator) for fr in qt], dtype=LD))


def dst_bubbles(n, degree):
    """Unit-norm samplings of x(pi-x) and (x-pi/2) x (pi-x) at x_i = i pi/(n-1), i=1..n-2.

    They vanish at the ends x = 0 and x = pi of the antireflective grid, so together with
    p and Jp they span all polynomials of degree <= 3 sampled on that grid."""
    N = n - 2
    cols = []
    for c in range(degree - 1):
        vals = []
        for i in range(1, N + 1):
            x = Fraction(i, n - 1)  # x / pi
            v = x * (1 - x)
            if c == 1:
                v = v * (x - Fraction(1, 2))
            vals.append(LD(v.numerator) / LD(v.denominator))
        cols.append(_unit(np.array(vals, dtype=LD)))
    return cols


# ----------------------------------------------------------------------------------------
# dense transform matrices
# ----------------------------------------------------------------------------------------

def cubic_f3(n):
    """Unit-norm samples of x (x - pi)(x - 2 pi) at the T_F grid x_r = (r-2) 2 pi/(n-2),
    r = 1..n (exact rationals in units of pi)."""
    N = n - 2
    vals = []
    for r in range(1, n + 1):
        t = Fraction(2 * (r - 2), N)  # x / pi
        v = t * (t - 1) * (t - 2)
        vals.append(LD(v.numerator) / LD(v.denominator))
    return _unit(np.array(vals, dtype=LD))


@lru_cache(maxsize=16)
def transform_matrix(kind, n):
    """Dense n x n matrix of the kind's transform, long double (complex for F, P, F3)."""
    if kind not in KINDS:
        raise ValueError(kind)
    if kind == "F3":
        T = transform_matrix("F", n).copy()
        T[:, 2] = np.sqrt(LD(2)) * T[:, 2].real   # (e^{ix} + e^{-ix}) / sqrt(2 N)
        T[:, n - 2] = cubic_f3(n)
        return T
    if kind in ("P", "R"):
        return _comparator_matrix(kind, n)
    if n < 5:
        raise ValueError("n must be at least 5")
    N = n - 2
    if kind in ("AR", "DST2", "DST3"):
        T = np.zeros((n, n), dtype=LD)
        p = ar_p(n)
        T[:, 0] = p
        T[:, n - 1] = p[::-1]
        i = np.arange(1, N + 1, dtype=np.int64)
        _, s = cos_sin_pi(np.outer(i, i), n - 1)
        T[1:n - 1, 1:n - 1] = np.sqrt(LD(2) / LD(n - 1)) * s  # Q_ij, Section 2.2
        if kind != "AR":
            for c, bub in enumerate(dst_bubbles(n, degree_of(kind))):
                T[1:n - 1, 1 + c] = bub
        return T
    q = quad_q(kind, n)
    r = np.arange(1, n + 1, dtype=np.int64)  # row r samples the grid point x_{r-1}
    j = np.arange(1, N + 1, dtype=np.int64)
    if kind == "C":
        # middle column j: sqrt((2 - delta_j1)/N) cos((j-1) x), x = (2(r-1)-1) pi / (2N)
        c, _ = cos_sin_pi(np.outer(2 * (r - 1) - 1, j - 1), 2 * N)
        w = np.where(j == 1, np.sqrt(LD(1) / LD(N)), np.sqrt(LD(2) / LD(N)))
        T = np.zeros((n, n), dtype=LD)
        T[:, 1:n - 1] = c * w[None, :]
    else:
        # middle column j: exp(i (j-1) x) / sqrt(N), x = (r-2) 2 pi / N
        c, s = cos_sin_pi(np.outer(2 * (r - 2), j - 1), N)
        T = np.zeros((n, n), dtype=CLD)
        T[:, 1:n - 1] = (c + 1j * s) / np.sqrt(LD(N))
    T[:, 0] = q
    T[:, n - 1] = q[::-1]
    return T


def dct2_matrix(n):
    """C^(n)_{ij} = sqrt((2 - delta_{i,1})/n) cos((i-1)(2j-1) pi / (2n))   (Section 2.1)."""
    i = np.arange(1, n + 1, dtype=np.int64)
    c, _ = cos_sin_pi(np.outer(i - 1, 2 * i - 1), 2 * n)
    w = np.where(i == 1, np.sqrt(LD(1) / LD(n)), np.sqrt(LD(2) / LD(n)))
    return c * w[:, None]


def dft_matrix(n):
    """F^(n)_{ij} = exp(-i 2 pi (i-1)(j-1) / n) / sqrt(n)                 (Section 2.1)."""
    i = np.arange(n, dtype=np.int64)
    c, s = cos_sin_pi(-2 * np.outer(i, i), n)
    return (c + 1j * s) / np.sqrt(LD(n))


def dst1_matrix(N):
    """Q_{ij} = sqrt(2/(N+1)) sin(i j pi / (N+1)), i, j = 1..N               (Section 2.2)."""
    i = np.arange(1, N + 1, dtype=np.int64)
    _, s = cos_sin_pi(np.outer(i, i), N + 1)
    return np.sqrt(LD(2) / LD(N + 1)) * s


def _comparator_matrix(kind, n):
    if kind == "P":  # A_P = F^H diag F: eigenvectors are the columns of F^H (eq. permat)
        return np.conj(dft_matrix(n)).T.copy()
    return dct2_matrix(n).T.copy()  # A_R = C^T diag C (eq. refm)


# ----------------------------------------------------------------------------------------
# spectra
# ----------------------------------------------------------------------------------------

def eigen_grid(kind, n):
    """Per column of T: (is_poly, num, den) with frequency t = pi*num/den.

    AR   y_i = (i-1) pi/(n-1), i = 1..n-1, y_n = 0                          (eq. jcf)
    C    x_i = (i-2) pi/(n-2), i = 2..n-1, x_1 = x_n = 0                    (eq. Ac)
    F    x_i = (i-2) 2 pi/(n-2), i = 2..n-1, x_1 = x_n = 0                  (eq. Af, R2)
    DSTd as AR, with columns 2..d also carrying z(0) (the replaced columns)
    P    x_i = 2 (i-1) pi / n                                               (eq. permat)
    R    x_i = (i-1) pi / n                                                 (eq. refm)
    F3   as F, with column n-1 (the cubic) also carrying z(0)
    """
    i = np.arange(1, n + 1, dtype=np.int64)
    poly = np.zeros(n, dtype=bool)
    if kind in ("P", "R"):
        num = 2 * (i - 1) if kind == "P" else i - 1
        return poly, num, n
    poly[0] = poly[n - 1] = True
    if kind in ("AR", "DST2", "DST3"):
        poly[1:degree_of(kind)] = True
        num, den = i - 1, n - 1
    elif kind == "C":
        num, den = i - 2, n - 2
    else:
        num, den = 2 * (i - 2), n - 2
        if kind == "F3":
            poly[n - 2] = True
    num = np.where(poly, 0, num)
    return poly, num, den


def symbol(h, center, num, den):
    """z(t) = sum_j h_j e^{i j t} at t = pi*num/den (eq. symbol), direct summation in
    long double with exactly reduced angles."""
    h = np.asarray(h, dtype=np.float64)
    j = np.arange(h.size, dtype=np.int64) - int(center)
    c, s = cos_sin_pi(np.outer(np.asarray(num, dtype=np.int64), j), den)
    hl = h.astype(LD)
    return (c @ hl) + 1j * (s @ hl)


def psf_is_symmetric(h, center):
    h = np.asarray(h, dtype=np.float64)
    m = max(center, h.size - 1 - center)
    full = np.zeros(2 * m + 1)
    full[m - center:m - center + h.size] = h
    return bool(np.array_equal(full, full[::-1]))


def psf_halfwidth(h, center):
    h = np.asarray(h)
    return max(int(center), h.size - 1 - int(center))


def blur_eigs(kind, n, h, center):
    """d: eigenvalues of the blurring matrix in the kind's basis (eqs. jcf, Ac, Af, permat,
    refm).  Real (float64) for the symmetric-PSF kinds, complex128 for F and P.

    The spectral models of AR, C, DST2, DST3, R are defined for symmetric PSFs only
    (Sections 2-3); a nonsymmetric PSF raises ValueError.  Requires 2m+1 <= n-2 for the
    kinds with a core of order n-2 (eq. jcf)."""
    m = psf_halfwidth(h, center)
    core = n if kind in ("P", "R") else n - 2
    if 2 * m + 1 > core:
        raise ValueError("PSF too wide: need 2m+1 <= %d" % core)
    if kind not in COMPLEX_KINDS and not psf_is_symmetric(h, center):
        raise ValueError("kind %s needs a symmetric PSF" % kind)
    poly, num, den = eigen_grid(kind, n)
    if kind in ("F", "P", "F3"):
        num = -num  # R4: exponential column e^{ikx} carries z(-kx) under convolution
    z = symbol(h, center, num, den)
    if kind == "F3":
        z[2] = z[2].real  # the cosine column: Re z(x_1)
    z[poly] = np.sum(np.asarray(h, dtype=np.float64).astype(LD))  # R7: z(0) = sum h_j
    if kind in COMPLEX_KINDS:
        return z.astype(np.complex128)
    return z.real.astype(np.float64)


def smooth_eigs(kind, n, norm):
    """s: spectrum of the smoothing operator L (Section 4).

    norm "I": L = I, s = 1.  norm "D2": s(x) = 2 - 2 cos(x) on the kind's grid, which is
    zero on the preserved polynomials (eq. L and the definitions of L_C, L_F)."""
    if norm == "I":
        return np.ones(n, dtype=np.float64)
    if norm != "D2":
        raise ValueError(norm)
    poly, num, den = eigen_grid(kind, n)
    c, _ = cos_sin_pi(num, den)
    s = LD(2) - LD(2) * c
    s[poly] = 0
    return s.astype(np.float64)


# ----------------------------------------------------------------------------------------
# products with T and T^{-1}
# ----------------------------------------------------------------------------------------

@lru_cache(maxsize=8)
def _lu(kind, n):
    T = transform_matrix(kind, n)
    T64 = T.astype(np.complex128 if is_complex(kind) else np.float64)
    return sla.lu_factor(T64, check_finite=False)


def forward(kind, x):
    """y = T x (the "direct transform"), long-double accumulation. x: (..., n)."""
    x = np.asarray(x)
    n = x.shape[-1]
    T = transform_matrix(kind, n)
    xl = x.astype(CLD if np.iscomplexobj(x) or is_complex(kind) else LD)
    y = np.einsum("ij,...j->...i", T, xl)
    return _round(y, kind, x)


def forward_f64(kind, x):
    """y = T x with a float64 product (used as the reference at sizes where the long-double
    product is too slow; its error, about 1e-15 relative, is far below what it checks)."""
    T = transform_matrix(kind, np.asarray(x).shape[-1])
    T64 = T.astype(np.complex128 if is_complex(kind) else np.float64)
    y = np.asarray(x) @ T64.T
    return y if (is_complex(kind) or np.iscomplexobj(x)) else y.real


def _round(y, kind, x):
    if is_complex(kind) or np.iscomplexobj(x):
        return y.astype(np.complex128)
    return y.astype(np.float64)


def inverse(kind, y, refine_steps=3):
    """x = T^{-1} y (the "inverse transform") by dense LU of T with iterative refinement,
    residuals y - T x evaluated in long double.  y: (n,) or (batch, n).  refine_steps=0 is
    the plain float64 LU solve (about 1e-12 relative at n = 2048)."""
    y = np.asarray(y)
    squeeze = y.ndim == 1
    Y = np.atleast_2d(y)
    n = Y.shape[-1]
    T = transform_matrix(kind, n)
    lu = _lu(kind, n)
    cplx = is_complex(kind) or np.iscomplexobj(y)
    Yl = Y.astype(CLD if cplx else LD)
    X = sla.lu_solve(lu, Y.astype(np.complex128 if cplx else np.float64).T).T.astype(Yl.dtype)
    for _ in range(refine_steps):
        R = Yl - np.einsum("ij,bj->bi", T, X)
        dX = sla.lu_solve(lu, R.astype(np.complex128 if cplx else np.float64).T).T
        X = X + dX.astype(Yl.dtype)
    out = X.astype(np.complex128 if cplx else np.float64)
    return out[0] if squeeze else out


def blur_matrix(kind, n, h, center):
    """Dense A_X = T diag(d) T^{-1} (eqs. jcf, Ac, Af), long-double products."""
    T = transform_matrix(kind, n)
    d = blur_eigs(kind, n, h, center)
    Tinv = _dense_inverse(kind, n)
    A = (T * d.astype(CLD if np.iscomplexobj(d) else LD)[None, :]) @ Tinv
    return A


def smoothing_matrix(kind, n, norm):
    T = transform_matrix(kind, n)
    s = smooth_eigs(kind, n, norm).astype(LD)
    return (T * s[None, :]) @ _dense_inverse(kind, n)


@lru_cache(maxsize=8)
def _dense_inverse(kind, n):
    eye = np.eye(n)
    return inverse(kind, eye.astype(np.complex128 if is_complex(kind) else np.float64)).T.astype(
        CLD if is_complex(kind) else LD)


def row_of_T(kind, n, i, rowwise=None):
    """Row i (0-based) of T.  With rowwise (the default for n > 2048) the row is computed
    on its own from the entry formulas in O(n) (for sampled checks at sizes where the dense
    matrix is too large); otherwise it is read from transform_matrix."""
    if rowwise is None:
        rowwise = n > 2048
    if not rowwise:
        return transform_matrix(kind, n)[i]
    if kind in ("P", "R"):
        k = np.arange(n, dtype=np.int64)
        if kind == "P":  # column k of F^H: exp(+2 pi i (row) k / n) / sqrt(n)
            c, s = cos_sin_pi(2 * i * k, n)
            return (c + 1j * s) / np.sqrt(LD(n))
        c, _ = cos_sin_pi(k * (2 * i + 1), 2 * n)  # column k of C^T: row k of C
        return c * np.where(k == 0, np.sqrt(LD(1) / LD(n)), np.sqrt(LD(2) / LD(n)))
    N = n - 2
    j = np.arange(1, N + 1, dtype=np.int64)  # core column j (1-based), matrix column j
    if kind in ("AR", "DST2", "DST3"):
        row = np.zeros(n, dtype=LD)
        p = ar_p(n)
        row[0], row[n - 1] = p[i], p[n - 1 - i]
        if 0 < i < n - 1:
            _, s = cos_sin_pi(i * j, n - 1)  # Q_{ij}, rows of Q sit on rows 2..n-1 of T
            row[1:n - 1] = np.sqrt(LD(2) / LD(n - 1)) * s
            if kind != "AR":
                for c, bub in enumerate(dst_bubbles(n, degree_of(kind))):
                    row[1 + c] = bub[i - 1]
        return row
    kq = "C" if kind == "C" else "F"
    q = quad_q(kq, n)
    r = i + 1  # 1-based row: the grid point x_{r-1}
    if kind == "C":
        c, _ = cos_sin_pi((2 * (r - 1) - 1) * (j - 1), 2 * N)
        w = np.where(j == 1, np.sqrt(LD(1) / LD(N)), np.sqrt(LD(2) / LD(N)))
        row = np.zeros(n, dtype=LD)
        row[1:n - 1] = c * w
    else:
        c, s = cos_sin_pi(2 * (r - 2) * (j - 1), N)
        row = np.zeros(n, dtype=CLD)
        row[1:n - 1] = (c + 1j * s) / np.sqrt(LD(N))
        if kind == "F3":  # column 3: sqrt(2/N) cos x; column n-1: the unit-norm cubic
            row[2] = np.sqrt(LD(2)) * row[2].real
            row[n - 2] = cubic_f3(n)[i]
    row[0], row[n - 1] = q[i], q[n - 1 - i]
    return row
