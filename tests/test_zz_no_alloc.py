"""The allocation-free entry point ht_gcv_scan_exact_static through the C ABI: the same
results as ht_gcv_scan_exact (the plan's workspace) on two calls in a row, the second
with a smaller input (fewer images, a shorter grid, G left to the library), and the size
limit of its static workspace enforced before any launch."""

import ctypes

import numpy as np
import pytest
import torch

from paper_0906_2704_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
VP = ctypes.c_void_p


@pytest.fixture(scope="module")
def ht():
    from paper_0906_2704_amd import ht as _ht
    _ht.lib()
    return _ht


def ptr(t):
    return VP(t.data_ptr()) if t is not None else None


def call(L, fn, plan, ghat, d, s, mus, G, kb, mb, batch):
    st = getattr(L, fn)(plan.handle, ptr(ghat), ptr(d), ptr(s), 1, 1, ptr(mus), mus.shape[-1], 0, ptr(G), ptr(kb),
                        ptr(mb), batch, VP(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("kind,sym", [("C", True), ("F", False)])
def test_static_matches_plan_workspace(ht, kind, sym):
    L = ht.lib()
    n0, n1, B = 150, 131, 3
    plan = ht.Plan((n0, n1), 2, psf_symmetric=sym, max_batch=B)
    assert plan.kinds == [kind, kind]
    H, c0, c1 = synth.disk_psf(3.0) if sym else synth.motion_psf(5.0, 30.0)
    rng = np.random.default_rng(7)
    imgs = np.stack([rng.standard_normal((n0, n1)).cumsum(axis=0).cumsum(axis=1) for _ in range(B)])
    d, s = ht.ht_eigs2d(plan, torch.tensor(H, device=DEV), (c0, c1), "D2")
    ghat = ht.ht_transform_inv(plan, torch.tensor(imgs, device=DEV))
    for b, K in ((B, 64), (1, 24)):  # second call: smaller input
        mus = torch.tensor(synth.mu_grid(-6.0 - b, 0.0, K), device=DEV)
        outs = []
        for fn, G in (("ht_gcv_scan_exact", torch.empty((b, K), dtype=torch.float64, device=DEV)),
                      ("ht_gcv_scan_exact_static", torch.empty((b, K), dtype=torch.float64, device=DEV)),
                      ("ht_gcv_scan_exact_static", None)):
            kb = torch.full((b,), -7, dtype=torch.int32, device=DEV)
            mb = torch.empty(b, dtype=torch.float64, device=DEV)
            assert call(L, fn, plan, ghat[:b].contiguous(), d, s, mus, G, kb, mb, b) == 0, L.ht_last_error()
            torch.cuda.synchronize()
            outs.append((G, kb.cpu(), mb.cpu()))
        (G0, k0, m0), (G1, k1, m1), (_, k2, m2) = outs
        assert torch.equal(G0, G1)  # same kernels, same order: bitwise equal
        assert torch.equal(k0, k1) and torch.equal(k0, k2) and (k0 >= 0).all()
        assert torch.equal(m0, m1) and torch.equal(m0, m2)


def test_static_workspace_limit(ht):
    """One 512-row image at K = 1024 needs 11.5 M doubles of row-pass outputs: more than
    the 2^23 of the static workspace, refused on the host."""
    L = ht.lib()
    plan = ht.Plan((512, 40), 2, psf_symmetric=True, max_batch=1)
    d, s = ht.ht_eigs(plan, torch.tensor(np.array([0.25, 0.5, 0.25, 0.2, 0.6, 0.2]), device=DEV), [3, 3], [1, 1],
                      "D2")
    ghat = ht.ht_transform_inv(plan, torch.ones((1, 512, 40), dtype=torch.float64, device=DEV))
    mus = torch.tensor(synth.mu_grid(-6.0, 0.0, 1024), device=DEV)
    kb = torch.empty(1, dtype=torch.int32, device=DEV)
    mb = torch.empty(1, dtype=torch.float64, device=DEV)
    st = L.ht_gcv_scan_exact_static(plan.handle, ptr(ghat), ptr(d), ptr(s), 1, 0, ptr(mus), 1024, 0, None, ptr(kb),
                                    ptr(mb), 1, VP(torch.cuda.current_stream().cuda_stream))
    assert st == 1 and b"static" in L.ht_last_error()
