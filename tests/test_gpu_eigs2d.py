"""GPU parity of the general 2D eigenvalues (ht_eigs2d, the three steps of Section 6) and
of the filter and GCV scan on full [n0][n1] spectra, against the CPU oracle, through the
C ABI: out-of-focus (disk) and random even masks on the real kinds, one-sided motion
masks on T_F, at shapes that span several 64 x 64 tiles with ragged tails.

Tolerance: the entries are direct sums of len0 * len1 taps with exactly reduced angles;
their float64 rounding is a few units of 2^-52 times sum |H| * len, well under
1e-13 * sum |H|.  The restorations follow the 1e-12 contract of the separable path."""

import numpy as np
import pytest
import torch

from oracle import tikhonov as tk
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


def even_mask(rng, m0, m1):
    Q = rng.random((m0 + 1, m1 + 1)) + 0.05
    H = np.concatenate([Q[:0:-1], Q])
    H = np.concatenate([H[:, :0:-1], H], axis=1)
    return H / H.sum(), m0, m1


def masks(kind, seed):
    """Two masks of one shape (one ht_eigs2d call takes a batch of equal shapes)."""
    rng = np.random.default_rng(seed)
    if kind == "F":
        A, a0, a1 = synth.motion_psf(9, 35)
        B = rng.random(A.shape) + 0.05
        return [A, B / B.sum()], (a0, a1)
    H, c0, c1 = synth.disk_psf(5.5)
    E, _, _ = even_mask(rng, c0, c1)
    return [H, E], (c0, c1)


CONFIGS = [(2, "paper", True, "C"), (1, "paper", True, "AR"), (3, "paper+dst3", True, "DST3"),
           (2, "paper", False, "F")]


@pytest.mark.parametrize("degree,family,sym,kind", CONFIGS)
@pytest.mark.parametrize("norm", ["I", "D2"])
@pytest.mark.parametrize("shape", [(70, 133), (131, 64), (20, 17)])
def test_eigs2d_matches_oracle(ht, degree, family, sym, kind, norm, shape):
    n0, n1 = shape
    print("case", kind, norm, shape, flush=True)
    Hs, (c0, c1) = masks(kind, n0 + n1)
    if 2 * max(synth.mask_halfwidths(Hs[0], c0, c1)) + 1 > min(n0, n1) - 2:
        pytest.skip("mask too wide for this shape")
    plan = ht.Plan((n0, n1), degree, psf_symmetric=sym, family=family, max_batch=2)
    assert plan.kinds == [kind, kind]
    d, s = ht.ht_eigs2d(plan, to_dev(np.stack(Hs)), (c0, c1), norm)
    d = d.cpu().numpy()
    s = s.cpu().numpy()
    s_ref = twod.smooth2d(kind, kind, n0, n1, norm)
    for b, H in enumerate(Hs):
        D = twod.eigs2d_general(kind, kind, n0, n1, H, c0, c1)
        err = np.abs(d[b] - D).max() / np.abs(H).sum()
        print("  mask %d: max |d - oracle| / sum|H| = %.2e" % (b, err))
        assert err < 1e-13
        assert np.abs(s[b] - s_ref).max() < 1e-14


def test_separable_mask_full_layout_equals_factors(ht):
    """A separable mask through ht_eigs2d (full layout) and through ht_eigs (factors): same
    spectrum, same GCV values and choice, same restoration."""
    n0, n1 = 96, 75
    h0, c0 = synth.gaussian_psf(5, 1.6)
    h1, c1 = synth.gaussian_psf(4, 1.1)
    plan = ht.Plan((n0, n1), 2, psf_symmetric=True, max_batch=2)
    dF, sF = ht.ht_eigs(plan, to_dev(np.concatenate([h0, h1])), [len(h0), len(h1)], [c0, c1], "D2")
    d2, s2 = ht.ht_eigs2d(plan, to_dev(np.outer(h0, h1)), (c0, c1), "D2")
    dFn = dF.cpu().numpy()[0]
    sFn = sF.cpu().numpy()[0]
    assert np.abs(np.multiply.outer(dFn[:n0], dFn[n0:]) - d2.cpu().numpy()[0]).max() < 1e-14
    assert np.abs(np.add.outer(sFn[:n0], sFn[n0:]) - s2.cpu().numpy()[0]).max() < 1e-14
    rng = np.random.default_rng(5)
    F = synth.piecewise_poly_image(rng, (n0 + 10, n1 + 8))
    G = synth.add_noise(rng, synth.observe_2d(F, h0, c0, h1, c1, (n0, n1)), 0.01)
    ghat = ht.ht_transform_inv(plan, to_dev(G[None]))
    mus = to_dev(synth.mu_grid(-6.0, 0.0, 64))
    Ga, ka, ma = ht.ht_gcv_scan(plan, ghat, dF, sF, mus)
    Gb, kb, mb = ht.ht_gcv_scan(plan, ghat, d2, s2, mus)
    assert np.abs(Ga.cpu().numpy() - Gb.cpu().numpy()).max() <= 1e-12 * Ga.abs().max().item()
    assert int(ka.cpu()[0]) == int(kb.cpu()[0])
    fa = ht.ht_tikhonov_filter(plan, ghat, dF, sF, ma).cpu().numpy()
    fb = ht.ht_tikhonov_filter(plan, ghat, d2, s2, mb).cpu().numpy()
    assert rel_normwise(fb, fa) < 1e-13


@pytest.mark.parametrize("kind,norm", [("C", "I"), ("AR", "D2"), ("F", "D2")])
def test_mask_restoration_matches_oracle(ht, kind, norm):
    """End to end with general masks, two images with their own masks (eig_batch = 2):
    ghat, G over 128 mu, k*, restoration, against the oracle."""
    n0, n1 = 150, 141
    degree = 1 if kind == "AR" else 2
    sym = kind != "F"
    Hs, (c0, c1) = masks(kind, 77)
    m0, m1 = synth.mask_halfwidths(Hs[0], c0, c1)
    rng = np.random.default_rng(11)
    Gs = []
    for H in Hs:
        F = synth.piecewise_poly_image(rng, (n0 + 2 * m0, n1 + 2 * m1))
        Gs.append(synth.add_noise(rng, synth.observe_2d_mask(F, H, c0, c1, (n0, n1)), 0.002))
    plan = ht.Plan((n0, n1), degree, psf_symmetric=sym, max_batch=2)
    assert plan.kinds == [kind, kind]
    d, s = ht.ht_eigs2d(plan, to_dev(np.stack(Hs)), (c0, c1), norm)
    ghat = ht.ht_transform_inv(plan, to_dev(np.stack(Gs)))
    mus = synth.mu_grid(-6.0, 0.0, 128)
    Gv, kb, mb = ht.ht_gcv_scan(plan, ghat, d, s, to_dev(mus))
    f = ht.ht_transform_fwd(plan, ht.ht_tikhonov_filter(plan, ghat, d, s, mb)).cpu().numpy()
    s_ref = twod.smooth2d(kind, kind, n0, n1, norm)
    for b, H in enumerate(Hs):
        D = twod.eigs2d_general(kind, kind, n0, n1, H, c0, c1)
        gh = twod.inverse2d(kind, kind, Gs[b])
        assert rel_normwise(ghat[b].cpu().numpy(), gh) < TOL
        Gw, kw, muw = tk.gcv_scan(gh.ravel(), D.ravel(), s_ref.ravel(), mus)
        assert_gcv_close(Gv[b].cpu().numpy(), Gw, gh.ravel(), D.ravel(), s_ref.ravel(), mus, "mask %d" % b)
        assert int(kb[b]) == kw and float(mb[b]) == muw
        fw = twod.forward2d(kind, kind, tk.tikhonov_filter(gh, D, s_ref, muw))
        assert rel_normwise(f[b], fw.real) < TOL


def test_eigs2d_contract(ht):
    plan = ht.Plan((40, 40), 2, max_batch=1)
    H, c0, c1 = synth.disk_psf(3.0)
    with pytest.raises(ht.HTError, match="max_batch"):
        ht.ht_eigs2d(plan, to_dev(np.stack([H, H])), (c0, c1), "I")
    Hw, w0, w1 = synth.disk_psf(19.0)    # 39 x 39 > n - 2
    with pytest.raises(ht.HTError, match="PSF_TOO_WIDE|2m\\+1"):
        ht.ht_eigs2d(plan, to_dev(Hw), (w0, w1), "I")
    with pytest.raises(ht.HTError, match="center"):
        ht.ht_eigs2d(plan, to_dev(H), (c0, 7), "I")
    p1 = ht.Plan(64, 2)
    with pytest.raises(ValueError):
        ht.ht_eigs2d(p1, to_dev(H), (c0, c1), "I")
    # a full spectrum whose eig_batch is neither 1 nor batch
    d, s = ht.ht_eigs2d(plan, to_dev(H), (c0, c1), "I")
    coeff = torch.zeros((3, 40, 40), dtype=torch.float64, device=DEV)
    with pytest.raises(ht.HTError, match="eig_batch"):
        ht.ht_tikhonov_filter(plan, coeff, torch.cat([d, d]), torch.cat([s, s]),
                              torch.ones(3, dtype=torch.float64, device=DEV))
