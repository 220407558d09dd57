"""Learned choice of mu (ORACLE, test infrastructure): the feature definition and the
certificate rule, written out plainly.  Not part of the paper: an accelerator of its GCV
step (eq. mugcv), judged by it.

Features of one signal (72 numbers): with N = n-2 core coefficients ghat_1..ghat_N (the
two polynomial entries excluded) and the core blur eigenvalues d_1..d_N, the means of
log10(|ghat_j|^2 + 1e-20) over 64 bands and of log10(|d_j|^2 + 1e-20) over 8 bands of the
normalised frequency; band b of B holds the 0-based core indices j with floor(B j / N) = b.
The floor 1e-20 keeps the logarithms well conditioned where the blur spectrum vanishes
(there |d_j| is only known to about 1e-16 absolutely).

Certificate: the grid index k^ nearest (in log10 mu, first on ties) to the prediction;
G on the bracket [k^-4, k^+4] clipped to the grid; k_m its first minimum; accept if
G(k^) <= 1.05 G(k_m) and k_m is not an edge of the bracket that lies inside the grid; the
chosen index is then k_m, otherwise the full scan's first minimum.
"""

import numpy as np


def features(ghat, d):
    ghat = np.asarray(ghat)
    d = np.asarray(d)
    n = ghat.size
    N = n - 2
    core_g = np.abs(ghat[1:n - 1]) ** 2
    core_d = np.abs(d[1:n - 1]) ** 2
    out = []
    for vals, B in ((core_g, 64), (core_d, 8)):
        logs = np.log10(vals + 1e-20)
        band = (B * np.arange(N)) // N
        for b in range(B):
            out.append(logs[band == b].mean())
    return np.array(out)


def nearest_index(mus, pred):
    lm = np.log10(np.asarray(mus, dtype=np.float64))
    return int(np.argmin(np.abs(lm - float(pred))))


def certify(G, khat, half=8, slack=1.05):
    """(chosen index, fell back?) for the GCV curve G of one signal."""
    G = np.asarray(G)
    K = G.size
    lo, hi = max(0, khat - half), min(K - 1, khat + half)
    km = lo + int(np.argmin(G[lo:hi + 1]))
    edge = (km == lo and lo > 0) or (km == hi and hi < K - 1)
    if not edge and G[khat] <= slack * G[km]:
        return km, False
    return int(np.argmin(G)), True
