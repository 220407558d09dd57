"""Blurring matrices assembled directly from boundary conditions (ORACLE, test infrastructure).

The observed sample is g_i = sum_j h_j f_{i-j}, i = 1..n (the discretised convolution of
eq. mod_cont; the PSF is the blur of a single pixel, Section 1), where samples of f outside
the field of view 1..n are replaced by the boundary condition:

* periodic       f_{1-j} = f_{n+1-j},       f_{n+j} = f_j             (Section 2.1)
* reflective     f_{1-j} = f_j,             f_{n+j} = f_{n+1-j}       (Section 2.1)
* antireflective f_{1-j} = 2 f_1 - f_{j+1}, f_{n+j} = 2 f_n - f_{n-j} (Section 2.2)

These matrices are built by brute force, one PSF tap at a time, and never use a transform.
They are the independent references that pin the spectral constructions in ``transforms``.

PSF convention: ``h`` is a 1D array and ``center`` the index of the tap h_0, so that
h[idx] is the tap h_{idx-center}.
"""

import numpy as np


def _taps(h, center):
    h = np.asarray(h, dtype=np.float64)
    return [(idx - center, h[idx]) for idx in range(h.size)]


def _add_sample(A, i, l, w, bc, n):
    """Add weight w times the (possibly out-of-view) sample f_l to row i (1-based)."""
    if 1 <= l <= n:
        A[i - 1, l - 1] += w
        return
    if bc == "periodic":
        _add_sample(A, i, (l - 1) % n + 1, w, bc, n)
    elif bc == "reflective":
        if l < 1:  # f_{1-j} = f_j with j = 1 - l
            _add_sample(A, i, 1 - l, w, bc, n)
        else:  # f_{n+j} = f_{n+1-j}
            j = l - n
            _add_sample(A, i, n + 1 - j, w, bc, n)
    elif bc == "antireflective":
        if l < 1:  # f_{1-j} = 2 f_1 - f_{j+1}
            j = 1 - l
            _add_sample(A, i, 1, 2.0 * w, bc, n)
            _add_sample(A, i, j + 1, -w, bc, n)
        else:  # f_{n+j} = 2 f_n - f_{n-j}
            j = l - n
            _add_sample(A, i, n, 2.0 * w, bc, n)
            _add_sample(A, i, n - j, -w, bc, n)
    else:
        raise ValueError(bc)


def blur_matrix_bc(bc, n, h, center):
    """Dense n x n blurring matrix for boundary condition ``bc`` (Section 2).

    Parity: pinned by the hand-computed fixture tests/golden/ar_n5_n7.txt and by the
    closed-form eigen-decompositions of eqs. permat / refm / jcf (tests)."""
    A = np.zeros((n, n), dtype=np.float64)
    for i in range(1, n + 1):
        for j, hj in _taps(h, center):
            _add_sample(A, i, i - j, hj, bc, n)
    return A


def second_difference_ar(n):
    """The matrix of eq. L: rows 2..n-1 hold the stencil (-1, 2, -1), rows 1 and n are zero."""
    L = np.zeros((n, n), dtype=np.float64)
    for i in range(1, n - 1):
        L[i, i - 1] = -1.0
        L[i, i] = 2.0
        L[i, i + 1] = -1.0
    return L
