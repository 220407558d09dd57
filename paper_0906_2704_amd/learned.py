"""Learned choice of mu for ragged batches: sequencing of libht's calls.

The network (72 -> 256 -> 256 -> 256 -> 1, exact GELU) predicts log10 mu from the 72 band
statistics of ht_batch_features; it is trained on problems the method generates, labelled
by the GCV scan (ht_batch_restore), with mean squared error and Adam.  The network lives in
the library (ht_mlp_*: float32 masters, bfloat16 copies for the matrix-core GEMMs, Adam
moments, standardisation); every step of training and inference - minibatch gathers,
forward, backward, Adam, labels, standardisation, prediction - runs in the library's
kernels.  This module only allocates buffers, draws the epoch permutations and orders the
calls.  Inference: features -> network -> ht_batch_restore_learned (GCV certificate around
the prediction, full-scan fallback), or all of it in one fused pass per signal
(ht_batch_restore_fused, the network evaluated inside the restore kernel with the same
rounding points).
"""

import numpy as np
import torch

from . import ht

DIMS = (72, 256, 256, 256, 1)
GRID_LOG10 = (-8.0, 1.0)  # fixed grid of the learned workload: 128 values on [1e-8, 10]
GRID_K = 128
SHAPES = [(DIMS[l], DIMS[l + 1]) if i == 0 else (DIMS[l + 1],) for l in range(4) for i in range(2)]


class Net:
    """The library's network (ht.Mlp) with He-normal initial weights drawn from `seed`."""

    def __init__(self, device="cuda", seed=0, max_rows=65536):
        self.device = device
        self.mlp = ht.Mlp(max_rows)
        rng = np.random.default_rng(seed)
        params = []
        for l in range(4):
            fan_in, fan_out = DIMS[l], DIMS[l + 1]
            params.append((rng.standard_normal((fan_in, fan_out)) * np.sqrt(2.0 / fan_in)).astype(np.float32))
            params.append(np.zeros(fan_out, dtype=np.float32))
        self.set_params(params)
        self.y = torch.empty(max_rows, dtype=torch.float32, device=device)

    # ------------------------------------------------------------------ parameters
    def _split(self, flat):
        out, off = [], 0
        for shp in SHAPES:
            k = int(np.prod(shp))
            out.append(flat[off:off + k].reshape(shp))
            off += k
        return out

    def set_params(self, params):
        flat = np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in params])
        ht.ht_mlp_set_params(self.mlp, torch.tensor(flat, device=self.device))

    def params_numpy(self):
        return self._split(self.mlp.get(ht.MLP_PARAMS_VEC).cpu().numpy())

    def grads_numpy(self):
        return self._split(self.mlp.get(ht.MLP_GRADS_VEC).cpu().numpy())

    @property
    def mean(self):
        return self.mlp.get(ht.MLP_MEAN_VEC)

    @property
    def std(self):
        return self.mlp.get(ht.MLP_STD_VEC)

    @property
    def step_count(self):
        return self.mlp.steps

    # ------------------------------------------------------------------ passes
    def forward(self, X):
        """X: float32 [B][72] raw features -> predictions (log10 mu), B <= max_rows."""
        B = X.shape[0]
        ht.ht_mlp_forward(self.mlp, X, self.y[:B])
        return self.y[:B]

    def predict(self, X, out=None):
        """Inference only (ht_mlp_predict): predictions for any number of rows, no
        activations kept for a backward pass."""
        return ht.ht_mlp_predict(self.mlp, X, out)

    def backward(self, t, loss=None):
        """Gradients of mean((y - t)^2) for the last forward pass (kept in the library)."""
        ht.ht_mlp_backward(self.mlp, t, loss)

    def adam_step(self, lr):
        ht.ht_mlp_adam_step(self.mlp, lr)

    def weights(self):
        """The network as ht.MlpWeights (device pointers into the library's network)."""
        return ht.ht_mlp_weights_of(self.mlp)

    # ------------------------------------------------------------------ persistence
    def save(self, path):
        g = self.mlp.get
        np.savez(path, params=g(ht.MLP_PARAMS_VEC).cpu().numpy(), m=g(ht.MLP_ADAM_M_VEC).cpu().numpy(),
                 v=g(ht.MLP_ADAM_V_VEC).cpu().numpy(), mean=g(ht.MLP_MEAN_VEC).cpu().numpy(),
                 std=g(ht.MLP_STD_VEC).cpu().numpy(), step=self.mlp.steps)

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            dev = lambda k: torch.tensor(z[k], device=self.device)
            ht.ht_mlp_set_params(self.mlp, dev("params"))
            ht.ht_mlp_set_state(self.mlp, dev("m"), dev("v"), int(z["step"]), dev("mean"), dev("std"))


def fit_standardisation(net, feats):
    """Feature mean / standard deviation of the training set (kept with the weights)."""
    ht.ht_mlp_fit_standardisation(net.mlp, feats)


def train(net, feats, labels, epochs=20, batch=1024, lr=1e-3, seed=0, log=None):
    """Minibatch Adam on (features, log10 mu labels), both device tensors: every epoch a
    fresh permutation of the rows (drawn on the host from `seed`), one library training
    step (device gather, forward, backward, Adam) per minibatch.  Returns the mean training
    loss per epoch."""
    rng = np.random.default_rng(seed)
    n = feats.shape[0]
    steps = n // batch
    losses = torch.zeros((epochs, max(steps, 1)), dtype=torch.float32, device=feats.device)
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device=feats.device)
        for i in range(steps):
            ht.ht_mlp_train_step(net.mlp, feats, labels, perm[i * batch:(i + 1) * batch], lr, loss=losses[ep, i:i + 1])
        if log:
            log("epoch %d  train mse %.4f" % (ep, float(losses[ep, :steps].mean())))
    return [float(v) for v in losses[:, :steps].mean(dim=1).cpu().numpy()]


def fixed_grid(count, device):
    lo, hi = GRID_LOG10
    k = np.arange(GRID_K, dtype=np.float64)
    mus = 10.0 ** (lo + (hi - lo) * k / (GRID_K - 1))
    return torch.tensor(np.tile(mus, (count, 1)), device=device)


def labels_by_scan(batch, g, psf, mus, norm="D2"):
    """log10 of the GCV-optimal mu of every signal (the full scan)."""
    f, _, kb, mb = ht.ht_batch_restore(batch, g, psf, norm, mus, want_G=False)
    return ht.ht_log10_labels(mb), f, kb


CERT_HALF = 8  # certificate bracket: predicted grid index +- 8 (0.57 decades)


def restore_fused(net, batch, g, psf, mus, norm="D2", cert_half=CERT_HALF, restored=None, weights=None, **out):
    """The learned-mu restoration in one fused pass per signal (features, network,
    certificate, filter, forward).  Returns (restored, k_best, mu_best, fallback, pred)."""
    weights = net.weights() if weights is None else weights
    return ht.ht_batch_restore_fused(batch, g, psf, norm, mus, weights, cert_half, restored=restored, **out)


def restore_learned(net, batch, g, psf, mus, norm="D2", coeff=None, feats=None, cert_half=CERT_HALF, spectrum=None):
    """Features and prediction (ht_lambda_predict) -> certified restore.  Returns (restored,
    k_best, mu_best, fallback, pred).  `spectrum` (float64 [total_length]) carries the
    eigenvalues from the feature pass to the restore pass; allocated when not given."""
    if spectrum is None:
        spectrum = torch.empty_like(g)
    pred, coeff, feats = ht.ht_lambda_predict(batch, net.mlp, g, psf, coeff, feats, spectrum)
    coeff, kb, mb, fb = ht.ht_batch_restore_learned(batch, coeff, psf, norm, mus, pred, cert_half,
                                                    spectrum=spectrum)
    return coeff, kb, mb, fb, pred
