"""GPU parity of the comparator boundary conditions of Section 2.1 on the same path:
periodic (A_P = F^H diag(d) F, eq. permat, any PSF) and reflective (A_R = C^T diag(d) C,
eq. refm, symmetric PSF), cores of order n with no boundary columns, through the C ABI.

References: the oracle's dense transforms for n <= 1031; for the long signals (n = 4097
and 8192, where the FFT length 16384 takes the split path) scipy's orthonormal FFT and
DCT-II, the library routines these unitary transforms reduce to.  Restorations, G and k*
against the oracle, 1D and 2D (separable and general masks), and the restoration errors
of the four boundary models on the 1D workload."""

import numpy as np
import pytest
import scipy.fft as sfft
import torch

from oracle import tikhonov as tk
from oracle import transforms as tr
from oracle import twod
from paper_0906_2704_amd import synth

from parity import assert_gcv_close, rel_normwise

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-12


@pytest.fixture(scope="module")
def ht():
    from paper_0906_2704_amd import ht as _ht
    _ht.lib()
    return _ht


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def problem(kind, n, count, seed):
    rng = np.random.default_rng(seed)
    m = max(1, min(8, (n - 1) // 2))
    h, c = synth.gaussian_psf(m, max(m / 3, 0.6), shift=0.7 if kind == "P" else 0.0)
    Y = np.stack([synth.add_noise(rng, synth.observe_1d(synth.piecewise_poly(rng, n + 2 * m), h, c, n), 0.01)
                  for _ in range(count)])
    return Y, h, c


def reference_inverse(kind, Y):
    if Y.shape[-1] <= 1031:
        return np.stack([tr.inverse(kind, y) for y in Y])
    if kind == "P":   # T_P^{-1} = F, the unitary DFT with e^{-i ...}
        return sfft.fft(Y, axis=-1, norm="ortho")
    return sfft.dct(Y, type=2, axis=-1, norm="ortho")


def reference_forward(kind, X):
    if X.shape[-1] <= 1031:
        return np.stack([tr.forward(kind, x) for x in X])
    if kind == "P":
        return sfft.ifft(X, axis=-1, norm="ortho")
    return sfft.idct(X, type=2, axis=-1, norm="ortho")


@pytest.mark.parametrize("kind", ["P", "R"])
@pytest.mark.parametrize("n", [5, 64, 257, 1031, 4097, 8192])
def test_comparator_transforms_and_eigs(ht, kind, n):
    print("case", kind, n, flush=True)
    fam = "periodic" if kind == "P" else "reflective"
    plan = ht.Plan(n, 0, psf_symmetric=(kind == "R"), family=fam)
    assert plan.kinds == [kind]
    assert plan.is_complex == (kind == "P")
    Y, h, c = problem(kind, n, 3, n)
    X = reference_inverse(kind, Y)
    Xg = ht.ht_transform_inv(plan, to_dev(Y)).cpu().numpy()
    assert rel_normwise(Xg, X) < TOL
    Yg = ht.ht_transform_fwd(plan, ht.ht_transform_inv(plan, to_dev(Y))).cpu().numpy()
    assert rel_normwise(Yg, Y) < TOL
    Zr = reference_forward(kind, X)
    Zg = ht.ht_transform_fwd(plan, to_dev(X.astype(np.complex128) if kind == "P" else X)).cpu().numpy()
    assert rel_normwise(Zg, Zr.real) < TOL
    for norm in ("I", "D2"):
        d, s = ht.ht_eigs(plan, to_dev(h), [len(h)], [c], norm)
        if n <= 1031:
            do = tr.blur_eigs(kind, n, h, c)
            so = tr.smooth_eigs(kind, n, norm)
        else:   # z on the grid directly (eqs. permat, refm)
            k = np.arange(n)
            x = (2 * np.pi * k / n) if kind == "P" else (np.pi * k / n)
            taps = np.arange(len(h)) - c
            E = np.exp(1j * np.outer(-x if kind == "P" else x, taps))
            do = E @ h if kind == "P" else (E @ h).real
            so = np.ones(n) if norm == "I" else 2 - 2 * np.cos(x)
        assert np.abs(d.cpu().numpy()[0] - do).max() < 1e-13
        assert np.abs(s.cpu().numpy()[0] - so).max() < 1e-13


@pytest.mark.parametrize("kind", ["P", "R"])
@pytest.mark.parametrize("norm", ["I", "D2"])
def test_comparator_restoration_matches_oracle(ht, kind, norm):
    n = 300
    fam = "periodic" if kind == "P" else "reflective"
    plan = ht.Plan(n, 0, psf_symmetric=(kind == "R"), family=fam)
    Y, h, c = problem(kind, n, 4, 17)
    d, s = ht.ht_eigs(plan, to_dev(h), [len(h)], [c], norm)
    ghat = ht.ht_transform_inv(plan, to_dev(Y))
    mus = synth.mu_grid(-6.0, 0.0, 64)
    Gv, kb, mb = ht.ht_gcv_scan(plan, ghat, d, s, to_dev(mus))
    Gx, kx, mx = ht.ht_gcv_scan_exact(plan, ghat, d, s, to_dev(mus))   # unitary T: the same functional
    assert torch.equal(Gv, Gx) and torch.equal(kb, kx)
    f = ht.ht_transform_fwd(plan, ht.ht_tikhonov_filter(plan, ghat, d, s, mb)).cpu().numpy()
    do = tr.blur_eigs(kind, n, h, c)
    so = tr.smooth_eigs(kind, n, norm)
    for b in range(len(Y)):
        gh = tr.inverse(kind, Y[b])
        Gw, kw, muw = tk.gcv_scan(gh, do, so, mus)
        assert_gcv_close(Gv[b].cpu().numpy(), Gw, gh, do, so, mus, "%s %d" % (kind, b))
        assert int(kb[b]) == kw
        fw = tr.forward(kind, tk.tikhonov_filter(gh, do, so, muw)).real
        assert rel_normwise(f[b], fw) < TOL
        Ge = tk.gcv_exact_values(kind, gh, do, so, mus)
        assert_gcv_close(Gx[b].cpu().numpy(), Ge, gh, do, so, mus, "exact %s %d" % (kind, b))


@pytest.mark.parametrize("kind", ["P", "R"])
def test_comparator_2d(ht, kind):
    """Separable factors (ht_eigs) and a general mask (ht_eigs2d) on a 2D comparator plan."""
    n0, n1 = 72, 131
    fam = "periodic" if kind == "P" else "reflective"
    plan = ht.Plan((n0, n1), 0, psf_symmetric=(kind == "R"), family=fam, max_batch=2)
    assert plan.kinds == [kind, kind]
    rng = np.random.default_rng(4)
    if kind == "P":
        H, c0, c1 = synth.motion_psf(7, 25)
        h0, ch0 = synth.gaussian_psf(4, 1.3, shift=0.5)
    else:
        H, c0, c1 = synth.disk_psf(4.5)
        h0, ch0 = synth.gaussian_psf(4, 1.3)
    h1, ch1 = synth.gaussian_psf(3, 1.0)
    m0, m1 = synth.mask_halfwidths(H, c0, c1)
    Fx = synth.piecewise_poly_image(rng, (n0 + 2 * m0, n1 + 2 * m1))
    G = synth.add_noise(rng, synth.observe_2d_mask(Fx, H, c0, c1, (n0, n1)), 0.005)
    gh = twod.inverse2d(kind, kind, G)
    ghat = ht.ht_transform_inv(plan, to_dev(G[None]))
    assert rel_normwise(ghat.cpu().numpy()[0], gh) < TOL
    mus = synth.mu_grid(-6.0, 0.0, 32)
    s2 = twod.smooth2d(kind, kind, n0, n1, "D2")
    for layout in ("factors", "full"):
        if layout == "factors":
            d, s = ht.ht_eigs(plan, to_dev(np.concatenate([h0, h1])), [len(h0), len(h1)], [ch0, ch1], "D2")
            D = twod.eigs2d_separable(kind, kind, n0, n1, h0, ch0, h1, ch1)
        else:
            d, s = ht.ht_eigs2d(plan, to_dev(H), (c0, c1), "D2")
            D = twod.eigs2d_general(kind, kind, n0, n1, H, c0, c1)
            assert np.abs(d.cpu().numpy()[0] - D).max() < 1e-13
        Gv, kb, mb = ht.ht_gcv_scan(plan, ghat, d, s, to_dev(mus))
        Gw, kw, muw = tk.gcv_scan(gh.ravel(), D.ravel(), s2.ravel(), mus)
        assert_gcv_close(Gv[0].cpu().numpy(), Gw, gh.ravel(), D.ravel(), s2.ravel(), mus, layout)
        assert int(kb[0]) == kw
        f = ht.ht_transform_fwd(plan, ht.ht_tikhonov_filter(plan, ghat, d, s, mb)).cpu().numpy()[0]
        fw = twod.forward2d(kind, kind, tk.tikhonov_filter(gh, D, s2, muw)).real
        assert rel_normwise(f, fw) < TOL


def test_comparator_contract(ht):
    with pytest.raises(ht.HTError, match="degree 0"):
        ht.Plan(64, 1, family="periodic")
    with pytest.raises(ht.HTError, match="symmetric"):
        ht.Plan(64, 0, psf_symmetric=False, family="reflective")
    plan = ht.Plan(64, 0, family="reflective")
    with pytest.raises(ht.HTError, match="comparator|UNSUPPORTED"):
        plan.set_precision("bf16x3")
    # the core has order n: a mask of width n fits, n + 2 does not
    h = np.full(63, 1.0 / 63)
    ht.ht_eigs(plan, to_dev(h), [63], [31], "I")
    with pytest.raises(ht.HTError, match="PSF_TOO_WIDE"):
        ht.ht_eigs(plan, to_dev(np.full(65, 1.0 / 65)), [65], [32], "I")
    plan.set_precision("f32")   # the float32 chirp core works for the comparators too
    Y, h5, c5 = problem("R", 64, 2, 3)
    X = np.stack([tr.inverse("R", y) for y in Y])
    assert rel_normwise(ht.ht_transform_inv(plan, to_dev(Y)).cpu().numpy(), X) < 1e-5


def test_boundary_models_on_the_1d_workload(ht):
    """Restoration errors of the four boundary models (and the DST degree 3) at their GCV
    mu on the 1D workload (n = 256, Gaussian m = 8 sigma = 2, 1% noise), L = D2 and L = I:
    the structure of the paper's comparisons (Section 5) on synthetic data."""
    count = 64
    G_host, F, h, c, mus = synth.config0_batch(count)
    n = G_host.shape[1]
    models = [("P", 0, "periodic"), ("R", 0, "reflective"), ("AR", 1, "paper"), ("C", 2, "paper"),
              ("DST3", 3, "dst")]
    g = to_dev(G_host)
    out = {}
    for norm in ("D2", "I"):
        for kind, deg, fam in models:
            plan = ht.Plan(n, deg, psf_symmetric=True, family=fam)
            assert plan.kinds == [kind]
            d, s = ht.ht_eigs(plan, to_dev(h), [len(h)], [c], norm)
            ghat = ht.ht_transform_inv(plan, g)
            _, kb, mb = ht.ht_gcv_scan(plan, ghat, d, s, to_dev(mus))
            f = ht.ht_transform_fwd(plan, ht.ht_tikhonov_filter(plan, ghat, d, s, mb)).cpu().numpy()
            rre = np.linalg.norm(f - F, axis=1) / np.linalg.norm(F, axis=1)
            out[(kind, norm)] = rre.mean()
            # oracle check of one signal per model
            gh = tr.inverse(kind, G_host[0])
            do = tr.blur_eigs(kind, n, h, c)
            so = tr.smooth_eigs(kind, n, norm)
            _, kw, muw = tk.gcv_scan(gh, do, so, mus)
            assert int(kb[0]) == kw
    print("mean RRE at mu_GCV over %d signals:" % count)
    for norm in ("D2", "I"):
        print("  L=%s  " % norm + "  ".join("%s %.4f" % (k, out[(k, norm)]) for k, _, _ in models))
    # periodic boundary conditions ring at the edges of a non-periodic signal
    assert out[("P", "D2")] > out[("AR", "D2")]
