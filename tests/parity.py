"""Tolerances shared by the GPU parity tests, and the log of measured errors.

Float64 vectors (coefficients, restorations, eigenvalues) are compared normwise:
max_i |a_i - b_i| / max_i |b_i| <= 1e-12.

GCV values G_k = N_k / D_k^2 are checked two ways:

* against the oracle's G evaluated on the GPU's own coefficients (when the test has them):
  this isolates the scan's arithmetic, and the bound is the flat 1e-12;
* against the oracle's G on the oracle's coefficients: G_k depends on ghat through
  N_k = sum_i sigma_ik^2 |ghat_i|^2, so a normwise perturbation |dghat_i| <= delta max|ghat|
  changes G_k by at most kappa_k delta relatively, with
      kappa_k = 2 max|ghat| sum_i sigma_ik^2 |ghat_i| / sum_i sigma_ik^2 |ghat_i|^2,
  large when G_k is dominated by coefficients far below max|ghat| (noise-level high
  frequencies).  delta is the measured normwise coefficient error of the same run where
  the test has the GPU's coefficients, else DELTA_FFT (a few ulp: the normwise error of a
  float64 FFT-based transform of these lengths); the bound 1e-12 + kappa_k delta is capped
  at CAP_G = 1e-11.  kappa_k comes from the oracle's own quantities only.

Every check records its measured error and bound through `record` (printed, and appended as
JSON lines to the file named by HT_PARITY_LOG when that is set).
"""

import json
import os

import numpy as np

TOL = 1e-12
EPS = np.finfo(np.float64).eps
DELTA_FFT = 8 * EPS
CAP_G = 1e-11


def record(what, err, bound, **extra):
    """Print and log one measured error next to the bound it is asserted against."""
    err = float(err)
    bound = float(bound)
    print("PARITY %s err=%.3e bound=%.3e" % (what, err, bound), flush=True)
    path = os.environ.get("HT_PARITY_LOG")
    if path:
        row = {"what": str(what), "err": err, "bound": bound}
        row.update({k: (float(v) if isinstance(v, (float, np.floating)) else v) for k, v in extra.items()})
        with open(path, "a") as fh:
            fh.write(json.dumps(row) + "\n")
    return err


def rel_normwise(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def check_normwise(a, b, what, bound=TOL):
    """Assert max|a - b| / max|b| <= bound and record the measured value."""
    err = rel_normwise(a, b)
    record(what, err, bound)
    assert err <= bound, (what, err, bound)
    return err


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


def assert_gcv_close(G, Gw, ghat_oracle, d, s, mus, what="", delta=None):
    """G (GPU) against Gw (oracle on the oracle's coefficients) within
    min(CAP_G, 1e-12 + kappa_k delta) per grid value; delta = the measured normwise
    coefficient error when given, else DELTA_FFT."""
    G = np.asarray(G)
    Gw = np.asarray(Gw)
    delta = DELTA_FFT if delta is None else max(float(delta), EPS)
    kappa = gcv_kappa(ghat_oracle, d, s, mus)
    bound = np.minimum(CAP_G, TOL + kappa * delta)
    rel = np.abs(G - Gw) / np.abs(Gw)
    worst = int(np.argmax(rel / bound))
    record("G %s" % (what,), rel[worst], bound[worst], max_err=float(np.max(rel)), kappa=float(kappa[worst]),
           delta=delta)
    bad = np.nonzero(rel > bound)[0]
    assert bad.size == 0, (what, int(bad[0]), float(rel[bad[0]]), float(bound[bad[0]]))
    return float(np.max(rel))


def assert_scan_arith(G, Gw_own, what=""):
    """G (GPU) against the oracle's G on the GPU's own coefficients: the scan's
    arithmetic alone, flat 1e-12."""
    rel = float(np.max(np.abs(np.asarray(G) - np.asarray(Gw_own)) / np.abs(np.asarray(Gw_own))))
    record("G-arith %s" % (what,), rel, TOL)
    assert rel <= TOL, (what, rel)
    return rel
