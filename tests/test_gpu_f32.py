"""GPU checks of the float32 chirp-z cores (ht_plan_set_precision(HT_PRECISION_F32)):
1D transforms of every kind against the float64 oracle, and the 512 x 512 T_F (x) T_F
restoration (Laplacian, 128-point GCV) with its error against the oracle per result.

The core works in float32 on float64 inputs (boundary solve, corrections, eigenvalues, GCV
sums and filter stay float64).  A float32 FFT convolution of length M has a normwise
relative error of order log2(M) u (u = 2^-24), about 1e-6, relative to the vector it
transforms: the signal's coefficients for the inverse, and for the forward the result,
stated against the norm of the output y (measured <= 5.5e-6)."""

import numpy as np
import pytest
import torch

from oracle import tikhonov as tk
from oracle import transforms as tr
from oracle import twod
from paper_0906_2704_amd import synth

from parity import record, rel_normwise

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL_CORE = 1e-5
TOL_F_2D = 1.3e-4  # twice the measured 6.4e-5 of the 512 x 512 T_F (x) T_F restoration


@pytest.fixture(scope="module")
def ht():
    from paper_0906_2704_amd import ht as _ht
    _ht.lib()
    return _ht


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("degree,sym,family,kind", [(2, True, "paper", "C"), (2, False, "paper", "F"),
                                                    (1, True, "paper", "AR"), (3, True, "paper+dst3", "DST3")])
@pytest.mark.parametrize("n", [5, 37, 200, 1000, 5000])
def test_f32_core_1d(ht, degree, sym, family, kind, n):
    plan = ht.Plan(n, degree, psf_symmetric=sym, family=family)
    assert plan.kinds == [kind]
    plan.set_precision("f32")
    assert plan.precision == "f32"
    rng = np.random.default_rng(n + degree)
    m = max(1, min(8, (n - 3) // 2))
    h, c = synth.gaussian_psf(m, max(m / 3.0, 0.5), shift=0.0 if sym else 0.5)
    Y = np.stack([synth.add_noise(rng, synth.observe_1d(synth.piecewise_poly(rng, n + 2 * m), h, c, n), 0.01)
                  for _ in range(12)])
    X = tr.inverse(kind, Y)
    Xg = ht.ht_transform_inv(plan, to_dev(Y)).cpu().numpy()
    e_inv = np.max(np.linalg.norm(Xg - X, axis=1) / np.linalg.norm(X, axis=1))
    Yf = tr.forward(kind, X)
    Yg = ht.ht_transform_fwd(plan, to_dev(X)).cpu().numpy()
    Yf = Yf.real if np.iscomplexobj(Yf) else Yf
    e_fwd = np.max(np.linalg.norm(Yg - Yf, axis=1) / np.linalg.norm(X, axis=1))
    e_fwd_y = np.max(np.linalg.norm(Yg - Yf, axis=1) / np.linalg.norm(Yf, axis=1))
    record("f32 inverse %s n=%d" % (kind, n), e_inv, TOL_CORE)
    record("f32 forward/||x|| %s n=%d" % (kind, n), e_fwd, TOL_CORE)
    record("f32 forward/||y|| %s n=%d" % (kind, n), e_fwd_y, TOL_CORE)
    assert e_inv < TOL_CORE
    assert e_fwd_y < TOL_CORE


def test_f32_2d_512(ht):
    p = synth.config1(0)
    n = p.g.shape[0]
    plan = ht.Plan((n, n), 2, psf_symmetric=False, max_batch=1)
    assert plan.kinds == ["F", "F"]
    plan.set_precision("f32")
    psf = to_dev(np.concatenate([p.h0, p.h1]))
    d, s = ht.ht_eigs(plan, psf, [len(p.h0), len(p.h1)], [p.c0, p.c1], "D2")
    ghat = ht.ht_transform_inv(plan, to_dev(p.g[None]))
    Gv, kb, mb = ht.ht_gcv_scan(plan, ghat, d, s, to_dev(p.mus))
    f = ht.ht_transform_fwd(plan, ht.ht_tikhonov_filter(plan, ghat, d, s, mb))
    gh_o = twod.inverse2d("F", "F", p.g)
    dd = twod.eigs2d_separable("F", "F", n, n, p.h0, p.c0, p.h1, p.c1)
    ss = twod.smooth2d("F", "F", n, n, "D2")
    G_o = tk.gcv_values(gh_o.ravel(), dd.ravel(), ss.ravel(), p.mus)
    k = int(kb.cpu()[0])
    ko = int(np.argmin(G_o))
    e_ghat = rel_normwise(ghat.cpu().numpy()[0], gh_o)
    e_G = float(np.max(np.abs(Gv.cpu().numpy()[0] - G_o) / G_o))
    fo = twod.forward2d("F", "F", tk.tikhonov_filter(gh_o, dd, ss, float(p.mus[k]))).real
    e_f = rel_normwise(f.cpu().numpy()[0], fo)
    rre = np.linalg.norm(f.cpu().numpy()[0] - p.f_true) / np.linalg.norm(p.f_true)
    rre_o = np.linalg.norm(fo - p.f_true) / np.linalg.norm(p.f_true)
    print("f32 512x512 T_F: ghat %.2e  G %.2e  k* %d (oracle %d)  f %.2e  RRE %.5f (oracle %.5f)"
          % (e_ghat, e_G, k, ko, e_f, rre, rre_o))
    # the restoration's error is the coefficients' error passed through the filter, whose
    # gain conj(d) / (|d|^2 + mu |s|^2) reaches max_i 1 / (2 sqrt(mu) |s_i|) on the high
    # frequencies where the blurred coefficients are smallest: it exceeds 1e-5 (measured
    # 6.4e-5, asserted at twice that); the derived first-order bound is printed beside it
    gain = np.abs(dd) / (np.abs(dd) ** 2 + float(p.mus[k]) * ss ** 2)
    e_f_derived = e_ghat * float(np.max(np.abs(gh_o)) * np.max(gain)) / float(np.max(np.abs(fo)))
    record("f32 2d512 ghat", e_ghat, TOL_CORE)
    record("f32 2d512 G", e_G, TOL_CORE)
    record("f32 2d512 f", e_f, TOL_F_2D, k=k, ko=ko, derived=e_f_derived)
    assert k == ko
    assert e_ghat < TOL_CORE
    assert e_G < TOL_CORE
    assert e_f < TOL_F_2D
