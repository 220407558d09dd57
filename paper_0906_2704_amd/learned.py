"""Learned choice of mu for ragged batches: orchestration of libht's kernels.

The network (72 -> 256 -> 256 -> 256 -> 1, exact GELU) predicts log10 mu from the 72 band
statistics of ht_batch_features; it is trained on problems the method generates, labelled
by the GCV scan (ht_batch_restore), with mean squared error and Adam.  Weights are float32
masters with bfloat16 copies; every product runs in ht_gemm_bf16 (matrix cores, float32
accumulation) and every other step in the library's kernels; this module only allocates
buffers, orders the calls and moves minibatches.  Inference: features -> network ->
ht_batch_restore_learned (GCV certificate around the prediction, full-scan fallback), or
all of it in one fused pass per signal (ht_batch_restore_fused, the network evaluated inside
the restore kernel with the same rounding points).
"""

import numpy as np
import torch

from . import ht

DIMS = (72, 256, 256, 256, 1)
GRID_LOG10 = (-8.0, 1.0)  # fixed grid of the learned workload: 128 values on [1e-8, 10]
GRID_K = 128
BF16 = torch.bfloat16


class Net:
    def __init__(self, device="cuda", seed=0):
        self.device = device
        rng = np.random.default_rng(seed)
        self.P, self.Pb = [], []
        for l in range(4):
            fan_in, fan_out = DIMS[l], DIMS[l + 1]
            W = (rng.standard_normal((fan_in, fan_out)) * np.sqrt(2.0 / fan_in)).astype(np.float32)
            self.P.append(torch.tensor(W, device=device))
            self.P.append(torch.zeros(fan_out, dtype=torch.float32, device=device))
        for l in range(4):
            self.Pb.append(torch.empty(self.P[2 * l].shape, dtype=BF16, device=device))
        self.m = [torch.zeros_like(p) for p in self.P]
        self.v = [torch.zeros_like(p) for p in self.P]
        self.G = [torch.zeros_like(p) for p in self.P]
        self.step_count = 0
        self.mean = torch.zeros(DIMS[0], dtype=torch.float32, device=device)
        self.std = torch.ones(DIMS[0], dtype=torch.float32, device=device)
        self.W4r = torch.empty(DIMS[3], dtype=torch.float32, device=device)
        self._B = 0
        self.refresh_bf16()

    def refresh_bf16(self):
        for l in range(4):
            W = self.P[2 * l]
            ht.ht_to_bf16(W, self.Pb[l], W.shape[0], W.shape[1])

    def params_numpy(self):
        return [p.cpu().numpy() for p in self.P]

    def set_params(self, params):
        for p, q in zip(self.P, params):
            p.copy_(torch.as_tensor(np.asarray(q, dtype=np.float32)).reshape(p.shape))
        self.refresh_bf16()

    def _ensure(self, B):
        if B <= self._B:
            return
        dev = self.device
        H = DIMS[1]
        self.Xb = torch.empty((B, DIMS[0]), dtype=BF16, device=dev)
        self.Z = [torch.empty((B, H), dtype=torch.float32, device=dev) for _ in range(3)]
        self.Hb = [torch.empty((B, H), dtype=BF16, device=dev) for _ in range(3)]
        self.H3 = torch.empty((B, H), dtype=torch.float32, device=dev)
        self.y = torch.empty(B, dtype=torch.float32, device=dev)
        self.dy = torch.empty(B, dtype=torch.float32, device=dev)
        self.sq = torch.empty(B, dtype=torch.float32, device=dev)
        self.dH = torch.empty((B, H), dtype=torch.float32, device=dev)
        self.dZ = torch.empty((B, H), dtype=torch.float32, device=dev)
        self.dZb = torch.empty((B, H), dtype=BF16, device=dev)
        self._B = B

    def forward(self, X):
        """X: float32 [B][72] raw features -> predictions y[:B] (log10 mu)."""
        B = X.shape[0]
        self._ensure(B)
        H = DIMS[1]
        Xb, Z, Hb = self.Xb[:B], [z[:B] for z in self.Z], [h[:B] for h in self.Hb]
        ht.ht_to_bf16(X, Xb, B, DIMS[0], self.mean, self.std)
        ht.ht_gemm_bf16(B, H, DIMS[0], Xb, (DIMS[0], 1), self.Pb[0], (H, 1), bias=self.P[1], act=1, Z=Z[0], Cb=Hb[0])
        ht.ht_gemm_bf16(B, H, H, Hb[0], (H, 1), self.Pb[1], (H, 1), bias=self.P[3], act=1, Z=Z[1], Cb=Hb[1])
        ht.ht_gemm_bf16(B, H, H, Hb[1], (H, 1), self.Pb[2], (H, 1), bias=self.P[5], act=1, Z=Z[2], C=self.H3[:B],
                        Cb=Hb[2])
        ht.ht_gemm_bf16(B, 1, H, Hb[2], (H, 1), self.Pb[3], (1, 1), bias=self.P[7], act=0, C=self.y[:B], ldc=1)
        return self.y[:B]

    def backward(self, t):
        """Gradients of mean((y - t)^2) for the last forward pass into self.G."""
        B = t.shape[0]
        H = DIMS[1]
        y, dy, sq = self.y[:B], self.dy[:B], self.sq[:B]
        dH, dZ, dZb = self.dH[:B], self.dZ[:B], self.dZb[:B]
        ht.ht_mse_grad(y, t, dy, sq)
        ht.ht_colsum(self.H3[:B], B, H, self.G[6], weight=dy)
        ht.ht_colsum(dy, B, 1, self.G[7])
        ht.ht_from_bf16(self.Pb[3], self.W4r)
        ht.ht_outer(dy, self.W4r, dH, B, H)
        ins = [self.Xb[:B], self.Hb[0][:B], self.Hb[1][:B]]
        for l in (2, 1, 0):
            ht.ht_gelu_backward(self.Z[l][:B], dH, dZ, dZb)
            fan_in = DIMS[l]
            # dW = H_in^T dZ: (fan_in x H), contraction over the batch
            ht.ht_gemm_bf16(fan_in, H, B, ins[l], (1, fan_in), dZb, (H, 1), C=self.G[2 * l])
            ht.ht_colsum(dZ, B, H, self.G[2 * l + 1])
            if l > 0:
                # dH_in = dZ W^T
                ht.ht_gemm_bf16(B, H, H, dZb, (H, 1), self.Pb[l], (1, H), C=dH)
        return sq

    def weights(self):
        """The network as ht.MlpWeights (device pointers into this object's tensors)."""
        return ht.mlp_weights(self.Pb, [self.P[1], self.P[3], self.P[5], self.P[7]], self.mean, self.std)

    def adam_step(self, lr):
        self.step_count += 1
        for i, p in enumerate(self.P):
            pb = self.Pb[i // 2] if i % 2 == 0 else None
            ht.ht_adam(p, self.G[i], self.m[i], self.v[i], lr, self.step_count, pb=pb)

    def save(self, path):
        np.savez(path, *[p.cpu().numpy() for p in self.P], mean=self.mean.cpu().numpy(), std=self.std.cpu().numpy(),
                 m=np.concatenate([m.cpu().numpy().ravel() for m in self.m]),
                 v=np.concatenate([v.cpu().numpy().ravel() for v in self.v]), step=self.step_count)

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.set_params([z["arr_%d" % i] for i in range(8)])
            self.mean.copy_(torch.as_tensor(z["mean"]))
            self.std.copy_(torch.as_tensor(z["std"]))
            off = 0
            for m, v in zip(self.m, self.v):
                k = m.numel()
                m.copy_(torch.as_tensor(z["m"][off:off + k]).reshape(m.shape))
                v.copy_(torch.as_tensor(z["v"][off:off + k]).reshape(v.shape))
                off += k
            self.step_count = int(z["step"])


def fit_standardisation(net, feats):
    """Feature mean / standard deviation of the training set (stored with the weights)."""
    f = feats.cpu().numpy().astype(np.float64)
    net.mean.copy_(torch.tensor(f.mean(axis=0), dtype=torch.float32))
    net.std.copy_(torch.tensor(np.maximum(f.std(axis=0), 1e-6), dtype=torch.float32))


def train(net, feats, labels, epochs=20, batch=1024, lr=1e-3, seed=0, log=None):
    """Minibatch Adam on (features, log10 mu labels), both device tensors."""
    rng = np.random.default_rng(seed)
    n = feats.shape[0]
    history = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=feats.device)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            X = feats.index_select(0, idx).contiguous()
            t = labels.index_select(0, idx).contiguous()
            net.forward(X)
            sq = net.backward(t)
            net.adam_step(lr)
            tot += float(sq.sum())
            cnt += batch
        history.append(tot / max(cnt, 1))
        if log:
            log("epoch %d  train mse %.4f" % (ep, history[-1]))
    return history


def fixed_grid(count, device):
    lo, hi = GRID_LOG10
    k = np.arange(GRID_K, dtype=np.float64)
    mus = 10.0 ** (lo + (hi - lo) * k / (GRID_K - 1))
    return torch.tensor(np.tile(mus, (count, 1)), device=device)


def labels_by_scan(batch, g, psf, mus, norm="D2"):
    """log10 of the GCV-optimal mu of every signal (the full scan)."""
    f, _, kb, mb = ht.ht_batch_restore(batch, g, psf, norm, mus, want_G=False)
    return torch.log10(mb).to(torch.float32), f, kb


CERT_HALF = 8  # certificate bracket: predicted grid index +- 8 (0.57 decades)


def restore_fused(net, batch, g, psf, mus, norm="D2", cert_half=CERT_HALF, restored=None, weights=None, **out):
    """The learned-mu restoration in one fused pass per signal (features, network,
    certificate, filter, forward).  Returns (restored, k_best, mu_best, fallback, pred)."""
    weights = net.weights() if weights is None else weights
    return ht.ht_batch_restore_fused(batch, g, psf, norm, mus, weights, cert_half, restored=restored, **out)


def restore_learned(net, batch, g, psf, mus, norm="D2", coeff=None, feats=None, cert_half=CERT_HALF, spectrum=None):
    """Features -> prediction -> certified restore.  Returns (restored, k_best, mu_best,
    fallback, pred).  `spectrum` (float64 [total_length]) carries the eigenvalues from the
    feature pass to the restore pass; allocated when not given."""
    if spectrum is None:
        spectrum = torch.empty_like(g)
    coeff, feats = ht.ht_batch_features(batch, g, psf, coeff, feats, spectrum)
    pred = net.forward(feats)
    coeff, kb, mb, fb = ht.ht_batch_restore_learned(batch, coeff, psf, norm, mus, pred, cert_half,
                                                    spectrum=spectrum)
    return coeff, kb, mb, fb, pred
