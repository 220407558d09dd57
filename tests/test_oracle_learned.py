"""Pins of the learned-mu oracle: finite differences of the float64 backward pass,
bfloat16 rounding against exact cases, the feature bands and the certificate rule on
hand-made curves."""

import numpy as np

from oracle import learned, mlp


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    dims = (5, 7, 6, 4, 1)
    params = []
    for l in range(4):
        params.append(rng.standard_normal((dims[l], dims[l + 1])) * 0.7)
        params.append(rng.standard_normal(dims[l + 1]) * 0.1)
    X = rng.standard_normal((9, 5))
    t = rng.standard_normal(9)

    def loss(ps):
        y, _ = mlp.forward(ps, X)
        return np.mean((y - t) ** 2)

    y, cache = mlp.forward(params, X)
    grads = mlp.backward(cache, y, t)
    h = 1e-6
    for pi, p in enumerate(params):
        num = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            plus = [q.copy() for q in params]
            minus = [q.copy() for q in params]
            plus[pi][idx] += h
            minus[pi][idx] -= h
            num[idx] = (loss(plus) - loss(minus)) / (2 * h)
        g = np.asarray(grads[pi]).reshape(p.shape)
        assert np.max(np.abs(g - num)) < 1e-7 * max(1.0, np.max(np.abs(num))), pi


def test_bf16_rounding_exact_cases():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0], dtype=np.float32)
    got = mlp.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even (1); 1 + 3 * 2^-8 rounds up to 1 + 2^-6
    want = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0])
    assert np.array_equal(got, want)


def test_gelu_closed_forms():
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15  # 1 * Phi(1)
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15


def test_feature_bands_and_certificate():
    n = 130  # N = 128: 2 per band of 64, 16 per band of 8
    ghat = np.zeros(n)
    ghat[1:n - 1] = 10.0 ** np.arange(128)[::-1].clip(0, 100) / 1e50
    d = np.ones(n)
    f = learned.features(ghat, d)
    assert f.shape == (72,)
    core = np.log10(ghat[1:n - 1] ** 2 + 1e-20)
    assert abs(f[3] - core[6:8].mean()) < 1e-12
    assert np.allclose(f[64:], np.log10(1.0 + 1e-20))
    G = np.array([5.0, 4.0, 3.0, 2.0, 1.5, 1.4, 1.45, 1.6, 2.0, 3.0, 4.0, 5.0])
    assert learned.certify(G, 5, half=4) == (5, False)
    assert learned.certify(G, 6, half=4) == (5, False)          # within 5% of the bracket minimum
    assert learned.certify(G, 8, half=4) == (5, True)           # G(8) = 2.0 > 1.05 * 1.4: full scan
    assert learned.certify(G, 10, half=4)[1] is True            # minimum on an interior bracket edge
    G2 = G.copy()
    G2[0] = 0.5
    assert learned.certify(G2, 0, half=4) == (0, False)         # minimum at the grid end is allowed
    assert learned.nearest_index([1e-3, 1e-2, 1e-1], -1.6) == 1


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g from zero moments, the bias-corrected moments are exactly
    g and g^2 at every step, so each step moves a parameter by lr g / (|g| + eps)."""
    g = [np.array([[0.5, -2.0], [1e-3, 3.0]]), np.array([-0.25])]
    p = [np.zeros((2, 2)), np.ones(1)]
    m = [np.zeros_like(x) for x in p]
    v = [np.zeros_like(x) for x in p]
    lr, eps = 1e-2, 1e-8
    for step in range(1, 6):
        p, m, v = mlp.adam_step(p, g, m, v, step, lr, eps=eps)
        for pi, gi, p0 in zip(p, g, ([np.zeros((2, 2)), np.ones(1)])):
            want = p0 - step * lr * gi / (np.abs(gi) + eps)
            assert np.allclose(pi, want, rtol=0, atol=1e-15), step


def test_adam_first_step_is_sign_step():
    """From zero moments the first step is lr sign(g) |g| / (|g| + eps), whatever beta."""
    g = [np.array([2.0, -1e-4, 0.0])]
    p, _, _ = mlp.adam_step([np.zeros(3)], g, [np.zeros(3)], [np.zeros(3)], 1, 0.1, beta1=0.5, beta2=0.7)
    assert np.allclose(p[0], -0.1 * g[0] / (np.abs(g[0]) + 1e-8), rtol=0, atol=1e-15)
