"""GPU checks of the split-precision matrix-core cores (ht_plan_set_precision): 1D and 2D
transforms against the float64 oracle at sizes that span several 128 x 128 tiles with
ragged tails, the error contract, and the 16-image 2048 x 2048 T_C (x) T_C restoration
(L = I, 128-point GCV) with its error against the oracle reported per result.

Tolerances (normwise, relative to the norm of the data the GEMMs consume: the signal for
the 1D inverse, the signal T x for the forward; the boundary terms are float64.  In 2D the
second pass's boundary solve amplifies the first pass's errors by the condition number of
T, which the coefficients carry as well, so the 2D inverse is measured relative to the
coefficients' norm): one split
product has a componentwise error of at most about 3 u^2 sum_k |a_ik||x_k| from the
dropped low-low term and the two-part representations (u = 2^-8 for bfloat16, u = 2^-11
for float16), plus float32 accumulation.  With orthonormal core rows and errors of random
sign this is of order 3 u^2 ||x|| = 4.6e-5 (bfloat16) in the worst aligned case and
several times smaller in practice; for float16, 3 u^2 = 7e-7 is comparable to the float32
accumulation over N terms, and the bound allows 2e-6.  The bounds are per 1D pass."""

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
TOL_PASS = {"bf16x3": 4.6e-5, "f16x3": 2e-6}
# The 16 x 2048^2 restoration, per result: twice the largest value measured over images 0
# and 15 (bfloat16: ghat 4.1e-8, G 1.6e-5, f 6.1e-4; float16: ghat 2.7e-8, G 1.25e-7,
# f 2.1e-5).  They sit well inside the first-order bounds derived above (per-pass bound,
# times the filter gain max d / (d^2 + mu) = 500 at mu = 1e-6, times ||g|| / ||f|| for f),
# which the test prints beside them.
TOL_16X2048 = {"bf16x3": {"ghat": 8.2e-8, "G": 3.2e-5, "f": 1.22e-3},
               "f16x3": {"ghat": 5.4e-8, "G": 2.5e-7, "f": 4.2e-5}}
CONFIGS = [(2, "paper", "C"), (1, "paper", "AR"), (2, "dst", "DST2"), (3, "paper+dst3", "DST3")]


@pytest.fixture(scope="module")
def ht():
    from paper_0906_2704_amd import ht as _ht
    _ht.lib()
    return _ht


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def signals(n, count, seed):
    rng = np.random.default_rng(seed)
    m = max(1, min(8, (n - 3) // 2))
    h, c = synth.gaussian_psf(m, max(m / 3.0, 0.5))
    Y = np.empty((count, n))
    for b in range(count):
        f = synth.piecewise_poly(rng, n + 2 * m)
        Y[b] = synth.add_noise(rng, synth.observe_1d(f, h, c, n), 0.01)
    return Y


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("degree,family,kind", CONFIGS)
@pytest.mark.parametrize("n", [5, 37, 130, 1000])
def test_split_core_1d(ht, prec, degree, family, kind, n):
    count = 150  # two row tiles, the second ragged
    plan = ht.Plan(n, degree, psf_symmetric=True, family=family, max_batch=count)
    assert plan.kinds == [kind]
    plan.set_precision(prec)
    assert plan.precision == prec
    Y = signals(n, count, 100 + n)
    X = tr.inverse(kind, Y)
    Xg = ht.ht_transform_inv(plan, to_dev(Y)).cpu().numpy()
    # boundary coefficients come from the float64 boundary solve
    assert np.max(np.abs(Xg[:, [0, -1]] - X[:, [0, -1]])) <= 1e-12 * np.max(np.abs(X))
    err_inv = np.linalg.norm(Xg - X, axis=1) / np.linalg.norm(Y, axis=1)
    Yf = tr.forward(kind, X)
    Yg = ht.ht_transform_fwd(plan, to_dev(X)).cpu().numpy()
    err_fwd = np.linalg.norm(Yg - Yf, axis=1) / np.linalg.norm(Yf, axis=1)
    print("%s %s n=%d  inverse max %.2e mean %.2e   forward max %.2e mean %.2e"
          % (prec, kind, n, err_inv.max(), err_inv.mean(), err_fwd.max(), err_fwd.mean()))
    assert err_inv.max() < TOL_PASS[prec]
    assert err_fwd.max() < TOL_PASS[prec]


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
@pytest.mark.parametrize("degree,kind", [(2, "C"), (1, "AR"), (3, "DST3")])
def test_split_core_2d(ht, prec, degree, kind):
    n0, n1, batch = 70, 133, 3
    plan = ht.Plan((n0, n1), degree, psf_symmetric=True, family="paper+dst3", max_batch=batch)
    assert plan.kinds == [kind, kind]
    plan.set_precision(prec)
    rng = np.random.default_rng(7 + degree)
    G = np.stack([synth.add_noise(rng, synth.observe_2d(synth.piecewise_poly_image(rng, (n0 + 8, n1 + 6)),
                                                        *synth.gaussian_psf(4, 1.5), *synth.gaussian_psf(3, 1.0),
                                                        (n0, n1)), 0.01) for _ in range(batch)])
    X = np.stack([twod.inverse2d(kind, kind, g) for g in G])
    Xg = ht.ht_transform_inv(plan, to_dev(G)).cpu().numpy()
    Yf = np.stack([twod.forward2d(kind, kind, x) for x in X])
    Yg = ht.ht_transform_fwd(plan, to_dev(X)).cpu().numpy()
    for b in range(batch):
        e_inv = rel_normwise(Xg[b], X[b])
        e_fwd = np.linalg.norm(Yg[b] - Yf[b]) / np.linalg.norm(Yf[b])
        print("%s %s 2D image %d  inverse %.2e  forward %.2e" % (prec, kind, b, e_inv, e_fwd))
        assert e_inv < 2 * TOL_PASS[prec]
        assert e_fwd < 2 * TOL_PASS[prec]


def test_split_core_contract(ht):
    plan = ht.Plan((40, 40), 2, psf_symmetric=False, max_batch=2)  # T_F (x) T_F
    with pytest.raises(ht.HTError, match="UNSUPPORTED|unsupported|real core"):
        plan.set_precision("bf16x3")
    assert plan.precision == "f64"
    plan = ht.Plan(64, 2, max_batch=4)
    plan.set_precision("f16x3")
    Y = to_dev(signals(64, 5, 3))
    with pytest.raises(ht.HTError, match="max_batch"):
        ht.ht_transform_inv(plan, Y)
    with pytest.raises(ht.HTError, match="overlap"):
        ht.ht_transform_inv(plan, Y[:4], out=Y[:4])
    # back to the float64 core: parity at 1e-12 again
    plan.set_precision("f64")
    Yh = Y.cpu().numpy()
    assert rel_normwise(ht.ht_transform_inv(plan, Y).cpu().numpy(), tr.inverse("C", Yh)) < 1e-12


# ------------------------------------------------------------- 16 x 2048 x 2048 (T_C)

BATCH3, N3, K3 = 16, 2048, 128


@pytest.fixture(scope="module")
def images3():
    return [synth.config3(i) for i in range(BATCH3)]


@pytest.fixture(scope="module")
def oracle3(images3):
    """Oracle results for the sampled images 0 and 15: plain float64 dense solves and
    products (about 1e-12 relative at this size), float64 GCV sums."""
    out = {}
    for i in (0, BATCH3 - 1):
        p = images3[i]
        ghat = twod.inverse2d("C", "C", p.g, refine_steps=0)
        d = twod.eigs2d_separable("C", "C", N3, N3, p.h0, p.c0, p.h1, p.c1)
        G = tk.gcv_values(ghat.ravel(), d.ravel(), np.ones(N3 * N3), p.mus, wide=False)
        out[i] = dict(ghat=ghat, d=d, G=G)
    return out


@pytest.mark.parametrize("prec", ["bf16x3", "f16x3"])
def test_mixed_precision_16x2048(ht, prec, images3, oracle3):
    p0 = images3[0]
    plan = ht.Plan((N3, N3), 2, psf_symmetric=True, max_batch=BATCH3)
    assert plan.kinds == ["C", "C"]
    plan.set_precision(prec)
    g = to_dev(np.stack([p.g for p in images3]))
    psf = to_dev(np.concatenate([p0.h0, p0.h1]))
    d, s = ht.ht_eigs(plan, psf, [len(p0.h0), len(p0.h1)], [p0.c0, p0.c1], "I")
    mus = to_dev(p0.mus)
    ghat = ht.ht_transform_inv(plan, g)
    Gv, kb, mb = ht.ht_gcv_scan(plan, ghat, d, s, mus)
    f = ht.ht_transform_fwd(plan, ht.ht_tikhonov_filter(plan, ghat, d, s, mb))
    torch.cuda.synchronize()
    for i in (0, BATCH3 - 1):
        o = oracle3[i]
        gh = ghat[i].cpu().numpy()
        e_ghat = rel_normwise(gh, o["ghat"])
        Gi = Gv[i].cpu().numpy()
        e_G = np.max(np.abs(Gi - o["G"]) / o["G"])
        k = int(kb[i])
        ko = int(np.argmin(o["G"]))
        assert k == ko, (k, ko)
        mu = float(p0.mus[k])
        fo = twod.forward2d("C", "C", tk.tikhonov_filter(o["ghat"], o["d"], np.ones((N3, N3)), mu), wide=False)
        e_f = rel_normwise(f[i].cpu().numpy(), fo)
        # the filter amplifies coefficient errors by at most max_i d_i / (d_i^2 + mu)
        amp = float(np.max(np.abs(o["d"]) / (o["d"] ** 2 + mu)))
        rre = np.linalg.norm(f[i].cpu().numpy() - images3[i].f_true) / np.linalg.norm(images3[i].f_true)
        rre_o = np.linalg.norm(fo - images3[i].f_true) / np.linalg.norm(images3[i].f_true)
        print("%s image %d: ghat %.2e  G %.2e  k* %d (oracle %d)  f %.2e (filter gain %.0f)  "
              "RRE %.5f (oracle %.5f)" % (prec, i, e_ghat, e_G, k, ko, e_f, amp, rre, rre_o))
        derived = 2 * TOL_PASS[prec] * amp * np.linalg.norm(images3[i].g) / np.linalg.norm(fo)
        tol = TOL_16X2048[prec]
        record("%s 16x2048 image %d ghat" % (prec, i), e_ghat, tol["ghat"])
        record("%s 16x2048 image %d G" % (prec, i), e_G, tol["G"], k=k, ko=ko)
        record("%s 16x2048 image %d f" % (prec, i), e_f, tol["f"], derived=derived)
        assert e_ghat < tol["ghat"]
        assert e_G < tol["G"]
        assert e_f < tol["f"]
