"""GPU parity of the 1D hot path (ht_eigs, ht_transform_inv/fwd, ht_tikhonov_filter,
ht_gcv_scan) against the CPU oracle, through the C ABI.

Tolerances: float64 results within 1e-12 relative (max-abs error over max-abs value of the
oracle result); the chosen mu index must match exactly."""

import numpy as np
import pytest
import torch

from oracle import tikhonov as tk
from oracle import transforms as tr
from paper_0906_2704_amd import synth

from parity import assert_gcv_close, assert_scan_arith, rel_normwise

pytestmark = pytest.mark.gpu

TOL = 1e-12
DEV = "cuda"

# (kind, family, degree, symmetric)
KIND_CFG = {
    "AR": ("paper", 1, True),
    "C": ("paper", 2, True),
    "F": ("paper", 2, False),
    "DST2": ("dst", 2, True),
    "DST3": ("dst", 3, True),
}
# sizes spanning every LDS FFT size (512 .. 8192 points) and the split 16384 case,
# with ragged core lengths
SIZES_SMALL = [5, 6, 9, 37, 130, 256, 257, 300, 513, 1000]
SIZES_LARGE = [2050, 3001, 4097]


@pytest.fixture(scope="module")
def ht():
    from paper_0906_2704_amd import ht as _ht
    _ht.lib()
    return _ht


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def plan_for(ht, kind, n):
    fam, deg, sym = KIND_CFG[kind]
    p = ht.Plan(n, deg, psf_symmetric=sym, family=fam)
    assert p.kinds[0] == kind
    return p


def psf_for(kind, n, rng):
    m = max(0, min(6, (n - 3) // 2))
    if kind == "F":
        h = rng.random(2 * m + 1) + 0.05
        h /= h.sum()
        return h, m
    half = rng.random(m + 1) + 0.1
    h = np.concatenate([half[:0:-1], half])
    return h / h.sum(), m


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("kind", list(KIND_CFG))
@pytest.mark.parametrize("n", SIZES_SMALL)
def test_transform_inv_fwd_parity(ht, kind, n):
    print("case", kind, n, flush=True)
    rng = np.random.default_rng(1000 + n)
    p = plan_for(ht, kind, n)
    B = 3
    Y = rng.standard_normal((B, n))
    ghat = ht.ht_transform_inv(p, to_dev(Y)).cpu().numpy()
    want = tr.inverse(kind, Y)
    assert relerr(ghat, want) < TOL
    # forward of the oracle's coefficients (real signal for every kind)
    X = want
    y = ht.ht_transform_fwd(p, to_dev(X)).cpu().numpy()
    assert relerr(y, tr.forward(kind, X).real) < TOL


@pytest.mark.parametrize("kind", list(KIND_CFG))
@pytest.mark.parametrize("n", SIZES_LARGE)
def test_transform_parity_large(ht, kind, n):
    print("case", kind, n, flush=True)
    if tr.is_complex(kind) and n > 3000:
        pytest.skip("complex dense oracle at this size is covered by the sampled test")
    rng = np.random.default_rng(2000 + n)
    p = plan_for(ht, kind, n)
    y = rng.standard_normal(n)
    ghat = ht.ht_transform_inv(p, to_dev(y[None])).cpu().numpy()[0]
    assert relerr(ghat, tr.inverse(kind, y)) < TOL
    back = ht.ht_transform_fwd(p, to_dev(ghat[None])).cpu().numpy()[0]
    assert relerr(back, y) < TOL


@pytest.mark.parametrize("kind", list(KIND_CFG))
@pytest.mark.parametrize("n", [5000, 8192])
def test_transform_sampled_rows_max_size(ht, kind, n):
    """At the largest sizes: rows of T computed one by one by the oracle check
    T (T^{-1} y) = y and T x on sampled rows."""
    print("case", kind, n, flush=True)
    rng = np.random.default_rng(3000 + n)
    p = plan_for(ht, kind, n)
    y = rng.standard_normal(n)
    ghat = ht.ht_transform_inv(p, to_dev(y[None])).cpu().numpy()[0]
    x = rng.standard_normal(n)
    if tr.is_complex(kind):
        x = tr_hermitian(x, n)
    yf = ht.ht_transform_fwd(p, to_dev(x[None])).cpu().numpy()[0]
    rows = sorted(set([0, 1, 2, n // 3, n // 2, n - 3, n - 2, n - 1] + list(rng.integers(0, n, 8))))
    for i in rows:
        row = tr.row_of_T(kind, n, int(i))
        res = complex(np.sum(row * ghat.astype(np.clongdouble))) - y[i]
        assert abs(res) < TOL * np.max(np.abs(y)) * 10
        want = complex(np.sum(row * x.astype(np.clongdouble)))
        assert abs(want.real - yf[i]) < TOL * max(np.max(np.abs(yf)), 1.0) * 10


def tr_hermitian(x, n):
    """A Hermitian coefficient vector for T_F (the image of a real signal)."""
    N = n - 2
    c = np.zeros(n, dtype=np.complex128)
    c[0], c[-1] = x[0], x[-1]
    core = x[1:n - 1] + 1j * np.roll(x, 7)[1:n - 1]
    core[0] = core[0].real
    k = np.arange(1, N)
    core[k] = 0.5 * (core[k] + np.conj(core[N - k]))
    if N % 2 == 0:
        core[N // 2] = core[N // 2].real
    c[1:n - 1] = core
    return c


@pytest.mark.parametrize("kind", list(KIND_CFG))
@pytest.mark.parametrize("norm", ["I", "D2"])
@pytest.mark.parametrize("n", [7, 64, 256, 1031])
def test_eigs_parity(ht, kind, norm, n):
    rng = np.random.default_rng(n)
    p = plan_for(ht, kind, n)
    B = 2
    hs = [psf_for(kind, n, rng) for _ in range(B)]
    L = len(hs[0][0])
    psf = np.stack([h for h, _ in hs])
    d, s = ht.ht_eigs(p, to_dev(psf), [L], [hs[0][1]], norm, batch=B)
    d, s = d.cpu().numpy(), s.cpu().numpy()
    for b in range(B):
        dw = tr.blur_eigs(kind, n, hs[b][0], hs[b][1])
        sw = tr.smooth_eigs(kind, n, norm)
        assert relerr(d[b], dw) < TOL
        assert np.max(np.abs(s[b] - sw)) < TOL * 4


@pytest.mark.parametrize("kind", list(KIND_CFG))
def test_filter_and_gcv_parity(ht, kind):
    n = 256
    B = 4
    rng = np.random.default_rng(5)
    p = plan_for(ht, kind, n)
    h, c = psf_for(kind, n, rng)
    if kind == "F":
        h, c = synth.gaussian_psf(8, 2.0, shift=0.7)
    else:
        h, c = synth.gaussian_psf(8, 2.0)
    G = np.stack([synth.signal_1d(0, b, n, h, c, 0.01, None).g for b in range(B)])
    mus = synth.mu_grid(-6.0, 0.0, 64)
    for norm in ("I", "D2"):
        d, s = ht.ht_eigs(p, to_dev(h), [len(h)], [c], norm)
        ghat = ht.ht_transform_inv(p, to_dev(G))
        Gv, kb, mb = ht.ht_gcv_scan(p, ghat, d, s, to_dev(mus))
        Gv, kb, mb = Gv.cpu().numpy(), kb.cpu().numpy(), mb.cpu().numpy()
        gh = ghat.cpu().numpy()
        dw = tr.blur_eigs(kind, n, h, c)
        sw = tr.smooth_eigs(kind, n, norm)
        for b in range(B):
            gw = tr.inverse(kind, G[b])
            Gw, kw, muw = tk.gcv_scan(gw, dw, sw, mus)
            assert_scan_arith(Gv[b], tk.gcv_values(gh[b], dw, sw, mus), (kind, norm, b))
            assert_gcv_close(Gv[b], Gw, gw, dw, sw, mus, (kind, norm, b), delta=rel_normwise(gh[b], gw))
            assert kb[b] == kw and mb[b] == muw
        mu_t = to_dev(mb)
        fhat = ht.ht_tikhonov_filter(p, ghat, d, s, mu_t)
        f = ht.ht_transform_fwd(p, fhat).cpu().numpy()
        for b in range(B):
            fw = tk.restore_spectral(kind, G[b], h, c, norm, mb[b])
            assert relerr(f[b], fw) < TOL


def test_gcv_per_item_grids_and_eigs(ht):
    """Each item with its own PSF spectrum and its own mu grid (uneven grids)."""
    kind, n, B, K = "DST3", 300, 5, 128
    rng = np.random.default_rng(8)
    p = plan_for(ht, kind, n)
    hs = [synth.gaussian_psf(5, 1.0 + b * 0.5) for b in range(B)]
    psf = np.stack([h for h, _ in hs])
    d, s = ht.ht_eigs(p, to_dev(psf), [11], [5], "D2", batch=B)
    Y = rng.standard_normal((B, n)).cumsum(axis=1)
    ghat = ht.ht_transform_inv(p, to_dev(Y))
    grids = np.stack([synth.mu_grid(lo, lo + 7, K) for lo in rng.uniform(-8, -6, B)])
    Gv, kb, mb = ht.ht_gcv_scan(p, ghat, d, s, to_dev(grids))
    Gv, kb = Gv.cpu().numpy(), kb.cpu().numpy()
    gh = ghat.cpu().numpy()
    for b in range(B):
        gw = tr.inverse(kind, Y[b])
        dw, sw = tr.blur_eigs(kind, n, *hs[b]), tr.smooth_eigs(kind, n, "D2")
        Gw, kw, _ = tk.gcv_scan(gw, dw, sw, grids[b])
        assert_scan_arith(Gv[b], tk.gcv_values(gh[b], dw, sw, grids[b]), b)
        assert_gcv_close(Gv[b], Gw, gw, dw, sw, grids[b], b, delta=rel_normwise(gh[b], gw))
        assert kb[b] == kw


def test_gcv_bitwise_deterministic(ht):
    kind, n, B = "C", 2000, 8
    rng = np.random.default_rng(3)
    p = plan_for(ht, kind, n)
    h, c = synth.gaussian_psf(8, 2.0)
    d, s = ht.ht_eigs(p, to_dev(h), [len(h)], [c], "D2")
    ghat = ht.ht_transform_inv(p, to_dev(rng.standard_normal((B, n))))
    mus = to_dev(synth.mu_grid(-8, 0, 128))
    ref = ht.ht_gcv_scan(p, ghat, d, s, mus)
    for _ in range(5):
        out = ht.ht_gcv_scan(p, ghat, d, s, mus)
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])


def test_polynomials_pass_through_restoration(ht):
    """Noise-free sampled polynomials of the preserved degree are restored exactly with
    the second-difference norm, for every mu (eigenvalue z(0) = 1, s = 0)."""
    n = 700
    x = np.linspace(-1, 2, n)
    for kind in KIND_CFG:
        p = plan_for(ht, kind, n)
        h, c = synth.gaussian_psf(6, 2.0, shift=0.6 if kind == "F" else 0.0)
        if kind != "F":
            h, c = synth.gaussian_psf(6, 2.0)
        deg = tr.degree_of(kind)
        P = np.polyval(np.arange(1, deg + 2, dtype=float), x)
        d, s = ht.ht_eigs(p, to_dev(h), [len(h)], [c], "D2")
        ghat = ht.ht_transform_inv(p, to_dev(P[None]))
        for mu in (1e-6, 1.0):
            f = ht.ht_transform_fwd(p, ht.ht_tikhonov_filter(p, ghat, d, s, to_dev(np.array([mu]))))
            assert relerr(f.cpu().numpy()[0], P) < 1e-12


def test_errors_and_empty_batches(ht):
    with pytest.raises(ht.HTError, match="UNSUPPORTED"):
        ht.Plan(64, 1, psf_symmetric=False, family="paper")
    with pytest.raises(ht.HTError, match="UNSUPPORTED"):
        ht.Plan(64, 3, psf_symmetric=True, family="paper")
    with pytest.raises(ht.HTError, match="INVALID_ARG"):
        ht.Plan(8193, 1)
    with pytest.raises(ht.HTError, match="INVALID_ARG"):
        ht.Plan(4, 1)
    p = ht.Plan(20, 2)
    h = np.ones(19) / 19
    with pytest.raises(ht.HTError, match="PSF_TOO_WIDE"):
        ht.ht_eigs(p, to_dev(h), [19], [9], "D2")
    empty = torch.empty((0, 20), dtype=torch.float64, device=DEV)
    out = ht.ht_transform_inv(p, empty)
    assert out.shape == (0, 20)
    with pytest.raises(ht.HTError):
        ht.ht_transform_inv(p, torch.zeros((1, 20), dtype=torch.float32, device=DEV))
