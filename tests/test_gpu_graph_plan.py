"""The plan-based restore captured in a HIP graph.

Every entry point of a plan launches kernels only (the plan owns its tables and work
buffers), so a whole restore -- eigenvalues, inverse transform, GCV scan, filter, forward
transform -- can be captured once and replayed.  Each replay, with unrelated eager work
and synchronisations in between, must reproduce the eager result bitwise (all reductions
run in a fixed order).  The 2D exact GCV works in the plan's own workspace as well."""

import numpy as np
import pytest
import torch

from paper_0906_2704_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def ht():
    from paper_0906_2704_amd import ht as _ht
    _ht.lib()
    return _ht


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def check_replays(ht, step, outs, noise):
    """Run `step` eagerly, capture it, replay four times and compare every output."""
    step()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(4):
        for o in outs:
            o.zero_()
        graph.replay()
        torch.cuda.synchronize()
        for i, (o, e) in enumerate(zip(outs, eager)):
            assert torch.equal(o, e), (rep, i)
        _ = (noise * 3.0).sum().item()  # unrelated eager work between replays
    del graph


def signals_1d(n, batch, seed, degree=2, shift=0.0):
    rng = np.random.default_rng(seed)
    h, c = synth.gaussian_psf(5, 1.6, shift=shift)
    ext = n + len(h) - 1
    g = np.stack([synth.add_noise(rng, synth.observe_1d(synth.piecewise_poly(rng, ext), h, c, n), 0.01)
                  for _ in range(batch)])
    return g, h, c


@pytest.mark.parametrize("family,degree,sym,exact", [
    ("paper", 2, True, False),     # T_C cores, eq. mugcv
    ("paper", 2, True, True),      # T_C cores, eq. gcv
    ("paper", 1, True, True),      # antireflective, eq. gcv
    ("paper", 2, False, False),    # complex T_F cores
    ("paper+dst3", 3, False, False),  # F3 (rank-2 corrected T_F)
    ("periodic", 0, False, True),  # comparator P
])
def test_1d_plan_pipeline_graph(ht, family, degree, sym, exact):
    n, batch, K = 777, 24, 40
    g_np, h, c = signals_1d(n, batch, seed=5 + degree, shift=0.0 if sym else 0.7)
    plan = ht.Plan(n, degree, psf_symmetric=sym, family=family, max_batch=batch)
    psf = to_dev(h)
    g = to_dev(g_np)
    mus = to_dev(synth.mu_grid(-7.0, 0.0, K))
    d = torch.empty((1, n), dtype=plan.coeff_dtype, device=DEV)
    s = torch.empty((1, n), dtype=torch.float64, device=DEV)
    ghat = torch.empty((batch, n), dtype=plan.coeff_dtype, device=DEV)
    fhat = torch.empty_like(ghat)
    f = torch.empty((batch, n), dtype=torch.float64, device=DEV)
    G = torch.empty((batch, K), dtype=torch.float64, device=DEV)
    kb = torch.empty(batch, dtype=torch.int32, device=DEV)
    mb = torch.empty(batch, dtype=torch.float64, device=DEV)
    scan = ht.ht_gcv_scan_exact if exact else ht.ht_gcv_scan

    def step():
        ht.ht_eigs(plan, psf, [len(h)], [c], "D2", d=d, s=s)
        ht.ht_transform_inv(plan, g, out=ghat)
        scan(plan, ghat, d, s, mus, G=G, kb=kb, mb=mb)
        ht.ht_tikhonov_filter(plan, ghat, d, s, mb, out=fhat)
        ht.ht_transform_fwd(plan, fhat, out=f)

    check_replays(ht, step, [d, s, ghat, G, kb, mb, fhat, f], g)
    plan.close()


@pytest.mark.parametrize("precision,exact", [("f64", False), ("bf16x3", False), ("f32", False), ("f64", True)])
def test_2d_mask_pipeline_graph(ht, precision, exact):
    """General 2D mask (ht_eigs2d, full spectrum layout) on T_C (x) T_C, in each core
    arithmetic the plan offers for real kinds, and with the exact GCV of eq. gcv (the
    plan's workspace)."""
    n0, n1, batch, K = 96, 80, 3, 24
    rng = np.random.default_rng(17)
    H, c0, c1 = synth.disk_psf(3.0)
    w0, w1 = synth.mask_halfwidths(H, c0, c1)
    imgs = []
    for _ in range(batch):
        F = synth.piecewise_poly_image(rng, (n0 + 2 * w0, n1 + 2 * w1))
        imgs.append(synth.add_noise(rng, synth.observe_2d_mask(F, H, c0, c1, (n0, n1)), 0.005))
    plan = ht.Plan((n0, n1), 2, psf_symmetric=True, max_batch=batch)
    plan.set_precision(precision)
    psf = to_dev(H)
    g = to_dev(np.stack(imgs))
    mus = to_dev(synth.mu_grid(-6.0, 0.0, K))
    d = torch.empty((1, n0, n1), dtype=plan.coeff_dtype, device=DEV)
    s = torch.empty((1, n0, n1), dtype=torch.float64, device=DEV)
    ghat = torch.empty((batch, n0, n1), dtype=plan.coeff_dtype, device=DEV)
    fhat = torch.empty_like(ghat)
    f = torch.empty((batch, n0, n1), dtype=torch.float64, device=DEV)
    G = torch.empty((batch, K), dtype=torch.float64, device=DEV)
    kb = torch.empty(batch, dtype=torch.int32, device=DEV)
    mb = torch.empty(batch, dtype=torch.float64, device=DEV)

    scan = ht.ht_gcv_scan_exact if exact else ht.ht_gcv_scan

    def step():
        ht.ht_eigs2d(plan, psf, (c0, c1), "D2", d=d, s=s)
        ht.ht_transform_inv(plan, g, out=ghat)
        scan(plan, ghat, d, s, mus, G=G, kb=kb, mb=mb)
        ht.ht_tikhonov_filter(plan, ghat, d, s, mb, out=fhat)
        ht.ht_transform_fwd(plan, fhat, out=f)

    check_replays(ht, step, [d, s, ghat, G, kb, mb, fhat, f], g)
    plan.close()
