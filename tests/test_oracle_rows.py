"""Pins of the oracle's row-by-row evaluation of T (oracle.transforms.row_of_T), which is
the reference of the sampled-row GPU checks at the largest sizes (n > 2048, where the dense
matrix is not built).

* At sizes where the dense matrix exists, every row computed on its own equals the dense
  matrix's row, for every kind.
* At n = 4099 (and the maximum n = 8192) sampled rows equal a 30-digit evaluation of the
  entry formulas as the paper prints them (eq. ART with the normalised p of R1 and the DST-I
  block of Section 2.2; eq. Tc with the cosine columns on x_i = (2i-3) pi / (2N) and
  q~_i = (b - x_i)^2, b = (2n-3) pi / (2n-4); eq. Tf with the exponential columns on
  x_i = (i-2) 2 pi / N and b = 2 pi (R2); the bubbles of the degree-2/3 extension, R10;
  the F3 columns of R23; the comparator bases F^H and C^T of eqs. permat, refm), computed
  with mpmath's own sine, cosine and pi, no exact angle reduction: an independent route.
"""

import mpmath as mpm
import numpy as np
import pytest

from oracle import transforms as tr

mpm.mp.dps = 30


@pytest.mark.parametrize("kind", tr.KINDS)
@pytest.mark.parametrize("n", [9, 257, 1031, 2048])
def test_rowwise_equals_dense_rows(kind, n):
    T = tr.transform_matrix(kind, n)
    rows = range(n) if n <= 257 else sorted(set([0, 1, 2, 3, n // 3, n // 2, n - 4, n - 3, n - 2, n - 1]
                                                + list(np.random.default_rng(n).integers(0, n, 24))))
    for i in rows:
        r = tr.row_of_T(kind, n, int(i), rowwise=True)
        # exact for every kind except P, whose dense form conjugates F (angle reduced from
        # the other side: one long-double rounding)
        tol = 0.0 if kind != "P" else 4e-19
        assert np.max(np.abs(r - T[i])) <= tol, (kind, n, i)


def _unit(v):
    nrm = mpm.sqrt(mpm.fsum(abs(x) ** 2 for x in v))
    return [x / nrm for x in v]


def _q(kind, n):
    """q = q~ / ||q~|| on the kind's extended grid (eqs. Tc, Tf), 0-based rows."""
    N = n - 2
    if kind == "C":
        x = [(2 * (i + 1) - 3) * mpm.pi / (2 * N) for i in range(n)]
        b = (2 * n - 3) * mpm.pi / (2 * n - 4)
    else:
        x = [((i + 1) - 2) * 2 * mpm.pi / N for i in range(n)]
        b = 2 * mpm.pi
    return _unit([(b - xi) ** 2 for xi in x])


def _bubbles(n, degree):
    xs = [i * mpm.pi / (n - 1) for i in range(1, n - 1)]
    cols = [_unit([x * (mpm.pi - x) for x in xs])]
    if degree == 3:
        cols.append(_unit([(x - mpm.pi / 2) * x * (mpm.pi - x) for x in xs]))
    return cols


def mp_row(kind, n, i, cache):
    """Row i (0-based) of T from the printed entry formulas, 30 digits."""
    N = n - 2
    r = i + 1  # 1-based row
    if kind == "P":
        return [mpm.exp(1j * 2 * mpm.pi * i * k / n) / mpm.sqrt(n) for k in range(n)]
    if kind == "R":
        return [mpm.sqrt(mpm.mpf(1 if k == 0 else 2) / n) * mpm.cos(k * (2 * i + 1) * mpm.pi / (2 * n))
                for k in range(n)]
    row = [mpm.mpf(0)] * n
    if kind in ("AR", "DST2", "DST3"):
        scale = mpm.sqrt(mpm.mpf(n * (2 * n - 1)) / (6 * (n - 1)))
        p = lambda k: (1 - mpm.mpf(k - 1) / (n - 1)) / scale  # p_k, k = 1..n
        row[0], row[n - 1] = p(r), p(n + 1 - r)
        if 1 < r < n:
            for j in range(1, N + 1):
                row[j] = mpm.sqrt(mpm.mpf(2) / (n - 1)) * mpm.sin((r - 1) * j * mpm.pi / (n - 1))
            if kind != "AR":
                if "bub" not in cache:
                    cache["bub"] = _bubbles(n, tr.degree_of(kind))
                for c, bub in enumerate(cache["bub"]):
                    row[1 + c] = bub[r - 2]
        return row
    if "q" not in cache:
        cache["q"] = _q("C" if kind == "C" else "F", n)
    q = cache["q"]
    if kind == "C":
        x = (2 * r - 3) * mpm.pi / (2 * N)
        for j in range(1, N + 1):
            row[j] = mpm.sqrt(mpm.mpf(1 if j == 1 else 2) / N) * mpm.cos((j - 1) * x)
    else:
        x = (r - 2) * 2 * mpm.pi / N
        for j in range(1, N + 1):
            row[j] = mpm.exp(1j * (j - 1) * x) / mpm.sqrt(N)
        if kind == "F3":
            row[2] = mpm.sqrt(mpm.mpf(2) / N) * mpm.cos(x)
            if "cubic" not in cache:
                xs = [((k + 1) - 2) * 2 * mpm.pi / N for k in range(n)]
                cache["cubic"] = _unit([t * (t - mpm.pi) * (t - 2 * mpm.pi) for t in xs])
            row[n - 2] = cache["cubic"][i]
    row[0], row[n - 1] = q[i], q[n - 1 - i]
    return row


@pytest.mark.parametrize("kind", tr.KINDS)
@pytest.mark.parametrize("n", [4099, 8192])
def test_rowwise_against_printed_formulas(kind, n):
    rng = np.random.default_rng(n + len(kind))
    rows = sorted(set([0, 1, 2, n // 3, n // 2, n - 3, n - 2, n - 1] + list(rng.integers(0, n, 3))))
    cache = {}
    for i in rows:
        got = tr.row_of_T(kind, n, int(i))  # the default path at this size: rowwise
        want = np.array([complex(v) for v in mp_row(kind, n, int(i), cache)])
        err = float(np.max(np.abs(got.astype(np.clongdouble) - want)))
        # entries are O(n^-1/2); long-double rounding of the reduced angles and the
        # normalisations stays far below float64 resolution
        assert err < 1e-17, (kind, n, i, err)
