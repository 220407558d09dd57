#!/usr/bin/env python
"""Throughput of the restoration hot path on one MI355X.

One step = the whole path over one batch of synthetic signals already resident in HBM:
PSF eigenvalues (ht_eigs), inverse transform (ht_transform_inv), GCV scan over the mu grid
(ht_gcv_scan), the Tikhonov filter at the chosen mu (ht_tikhonov_filter) and the forward
transform (ht_transform_fwd).  Prints one JSON line.

Per-kernel durations are taken live with HIP events recorded on the stream the kernels run
on; the roofline object reports the dominant kernel.  The CPU baseline times the dense
float64 oracle on a bounded sample of the same workload on the host cores.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "restorations/s incl. λ choice, learned-λ vs GCV scan at equal error; % HBM peak"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic float64 operations of one (element, mu) pair of the GCV scan:
# u = t + mu, r = 1/u, D += r, r^2, N += w r^2 (fused multiply-add = 2)
GCV_FLOPS_PER_PAIR = 6


class StageTimer:
    """HIP events between the stages of a step (all on torch's current stream)."""

    def __init__(self, torch, names):
        self.torch = torch
        self.names = names
        self.events = []
        self.active = False

    def start_step(self):
        if self.active:
            ev = self.torch.cuda.Event(enable_timing=True)
            ev.record()
            self.events.append([ev])

    def mark(self):
        if self.active:
            ev = self.torch.cuda.Event(enable_timing=True)
            ev.record()
            self.events[-1].append(ev)

    def averages(self):
        out = {name: 0.0 for name in self.names}
        for evs in self.events:
            for i, name in enumerate(self.names):
                out[name] += evs[i].elapsed_time(evs[i + 1])
        return {k: v / max(len(self.events), 1) for k, v in out.items()}


class Uniform1D:
    """The 1D workload: n = 256 signals of 4 random cubic pieces, symmetric Gaussian PSF
    (half-width 8, sigma 2), 1% noise, degree 2 (T_C), second-difference norm, GCV over 64
    log-spaced mu on [1e-6, 1]; a batch of seeded replicates."""

    stages = ["eigs", "transform_inv", "gcv_scan", "tikhonov_filter", "transform_fwd"]

    def __init__(self, torch, ht, synth, batch, n=256, degree=2, gcv="approx", family="paper"):
        self.torch, self.ht, self.synth = torch, ht, synth
        if family in ("periodic", "reflective"):
            degree = 0
        if family == "f3":   # degree 3 for any PSF: T_F with a cosine and a cubic column
            degree = 3
        self.batch, self.n, self.degree, self.gcv, self.family = batch, n, degree, gcv, family
        bc = "" if family == "paper" else "_" + family
        self.name = "1d_uniform_n%d_d%d_x%d%s%s" % (n, degree, batch, bc, "_exact_gcv" if gcv == "exact" else "")

    def setup(self):
        torch, ht, synth = self.torch, self.ht, self.synth
        G, F, h, c, mus = synth.config0_batch(self.batch)
        self.G_host, self.h, self.c, self.mus_host = G, h, c, mus
        dev = "cuda"
        if self.family == "f3":
            self.plan = ht.Plan(self.n, 3, psf_symmetric=False, family="paper+dst3")
        else:
            self.plan = ht.Plan(self.n, self.degree, psf_symmetric=True, family=self.family)
        self.kind = self.plan.kinds[0]
        self.g = torch.tensor(G, device=dev)
        self.psf = torch.tensor(h, device=dev)
        self.mus = torch.tensor(mus, device=dev)
        cd = self.plan.coeff_dtype
        self.d = torch.empty((1, self.n), dtype=cd, device=dev)
        self.s = torch.empty((1, self.n), dtype=torch.float64, device=dev)
        self.ghat = torch.empty((self.batch, self.n), dtype=cd, device=dev)
        self.fhat = torch.empty_like(self.ghat)
        self.f = torch.empty((self.batch, self.n), dtype=torch.float64, device=dev)
        self.Gv = torch.empty((self.batch, len(mus)), dtype=torch.float64, device=dev)
        self.kb = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.mb = torch.empty(self.batch, dtype=torch.float64, device=dev)

    def step(self, t):
        ht = self.ht
        t.start_step()
        ht.ht_eigs(self.plan, self.psf, [len(self.h)], [self.c], "D2", d=self.d, s=self.s)
        t.mark()
        ht.ht_transform_inv(self.plan, self.g, out=self.ghat)
        t.mark()
        scan = ht.ht_gcv_scan_exact if self.gcv == "exact" else ht.ht_gcv_scan
        scan(self.plan, self.ghat, self.d, self.s, self.mus, G=self.Gv, kb=self.kb, mb=self.mb)
        t.mark()
        ht.ht_tikhonov_filter(self.plan, self.ghat, self.d, self.s, self.mb, out=self.fhat)
        t.mark()
        ht.ht_transform_fwd(self.plan, self.fhat, out=self.f)
        t.mark()

    def config(self):
        return {"workload": self.name, "batch": self.batch, "n": self.n, "kind": self.kind, "norm": "D2",
                "K": len(self.mus_host), "gcv": "eq. gcv (exact)" if self.gcv == "exact" else "eq. mugcv"}

    def work(self):
        """Algorithmic bytes / flops per launch of each stage."""
        B, n, K = self.batch, self.n, len(self.mus_host)
        cb = 16 if self.plan.is_complex else 8
        # the exact functional adds one fused multiply-add per (element, mu, fixed vector):
        # 4 vectors for T_C (two boundary columns, two ghost rows); none for the unitary
        # comparators, where it is the same scan
        extra = 4 if self.kind == "C" else 0
        per_pair = GCV_FLOPS_PER_PAIR + (2 * extra if self.gcv == "exact" else 0)
        return {
            "eigs": ("hbm", (len(self.h) * 8 + n * (cb + 8))),
            "transform_inv": ("hbm", B * n * (8 + cb)),
            "gcv_scan": ("alu", B * n * K * per_pair),
            "tikhonov_filter": ("hbm", B * n * 2 * cb + B * 8),
            "transform_fwd": ("hbm", B * n * (cb + 8)),
        }

    def check(self):
        """Parity of a few items against the oracle (untimed)."""
        from oracle import tikhonov as tk
        from oracle import transforms as tr
        f = self.f.cpu().numpy()
        kb = self.kb.cpu().numpy()
        d = tr.blur_eigs(self.kind, self.n, self.h, self.c)
        s = tr.smooth_eigs(self.kind, self.n, "D2")
        worst = 0.0
        for b in (0, self.batch // 2, self.batch - 1):
            gw = tr.inverse(self.kind, self.G_host[b])
            if self.gcv == "exact":
                Gx = tk.gcv_exact_values(self.kind, gw, d, s, self.mus_host)
                kw = tk.gcv_argmin(Gx)
                muw = float(self.mus_host[kw])
            else:
                _, kw, muw = tk.gcv_scan(gw, d, s, self.mus_host)
            assert kw == kb[b], (b, kw, kb[b])
            fw = tr.forward(self.kind, tk.tikhonov_filter(gw, d, s, muw)).real
            worst = max(worst, float(np.max(np.abs(f[b] - fw)) / np.max(np.abs(fw))))
        return worst

    def cpu_baseline(self, budget_s):
        """The oracle (dense float64 transforms with refinement) on the first items."""
        from oracle import tikhonov as tk
        from oracle import transforms as tr
        d = tr.blur_eigs(self.kind, self.n, self.h, self.c)
        s = tr.smooth_eigs(self.kind, self.n, "D2")
        tr.inverse(self.kind, self.G_host[0])  # builds and factors T once (plan analogue)
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < budget_s and done < self.batch:
            g = self.G_host[done]
            gw = tr.inverse(self.kind, g)
            if self.gcv == "exact":
                muw = float(self.mus_host[tk.gcv_argmin(tk.gcv_exact_values(self.kind, gw, d, s, self.mus_host))])
            else:
                _, _, muw = tk.gcv_scan(gw, d, s, self.mus_host)
            tr.forward(self.kind, tk.tikhonov_filter(gw, d, s, muw))
            done += 1
        el = time.perf_counter() - t0
        return done / el, "first %d of the %d signals, one at a time" % (done, self.batch)


class Ragged1D:
    """The batched workload: 4096 signals, n ~ U{128..8192}, Gaussian (sigma = m/3) or box
    PSF with half-width m ~ U{2..32}, noise 0.1-5%, boundary degree ~ U{1,2,3} (degree 1:
    antireflective, 2: T_C, 3: DST extension), second-difference norm, a 128-point mu
    grid per signal on [10^lo, 10^(lo+7)], lo ~ U(-8,-6); one hipGraph replay per step."""

    stages = ["batch_restore"]
    profile = "k_restore_ragged4096.md"

    def __init__(self, torch, ht, synth, batch, graph=True, autotune=True):
        self.torch, self.ht, self.synth = torch, ht, synth
        self.batch = batch
        self.graph = graph
        self.autotune = autotune
        self.name = "1d_ragged_n128-8192_d123_K128_x%d" % batch
        self.n = None
        self.kind = "AR/C/DST3"

    def setup(self):
        torch, ht, synth = self.torch, self.ht, self.synth
        rb = synth.ragged_batch(self.batch)
        self.rb = rb
        self.K = rb.mus.shape[1]
        dev = "cuda"
        self.bt = ht.Batch(rb.n, rb.degree, np.diff(rb.psf_offsets), rb.psf_center)
        self.g = torch.tensor(rb.g, device=dev)
        self.psf = torch.tensor(rb.psf_flat, device=dev)
        self.mus = torch.tensor(rb.mus, device=dev)
        self.f = torch.empty_like(self.g)
        self.Gv = torch.empty((self.batch, self.K), dtype=torch.float64, device=dev)
        self.kb = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.mb = torch.empty(self.batch, dtype=torch.float64, device=dev)
        self.tuning = None
        if self.autotune:
            from paper_0906_2704_amd import autotune
            choice, ms = autotune.tune(self.bt, self._launch, use_cache=False,
                                       log=lambda m: print(m, file=sys.stderr, flush=True))
            self.tuning = {"choice": {str(c): list(v) for c, v in choice.items()},
                           "class_ms": {str(c): round(t, 4) for c, t in ms.items()}}
        self.cuda_graph = None
        if self.graph:
            self._launch()  # eager warm-up outside the capture
            torch.cuda.synchronize()
            self.cuda_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.cuda_graph):
                self._launch()
            torch.cuda.synchronize()

    def _launch(self):
        self.ht.ht_batch_restore(self.bt, self.g, self.psf, "D2", self.mus, restored=self.f, G=self.Gv,
                                 kb=self.kb, mb=self.mb)

    def step(self, t):
        t.start_step()
        if self.cuda_graph is not None:
            self.cuda_graph.replay()
        else:
            self._launch()
        t.mark()

    def config(self):
        return {"workload": self.name, "batch": self.batch, "n": "U{128..8192}", "sum_n": int(self.rb.n.sum()),
                "degree": "U{1,2,3}", "norm": "D2", "K": self.K, "graph": self.graph, "schedule": self.tuning}

    def work(self):
        n = self.rb.n.astype(np.float64)
        pairs = float(np.sum(n)) * self.K
        return {"batch_restore": ("alu", pairs * GCV_FLOPS_PER_PAIR)}

    def kind_of(self, b):
        return {1: "AR", 2: "C", 3: "DST3"}[int(self.rb.degree[b])]

    def sample_items(self, count):
        order = np.argsort(self.rb.n)
        picks = [int(order[int(q)]) for q in np.linspace(0, self.batch - 1, count)]
        return list(np.random.default_rng(0).permutation(picks))

    def check(self):
        from oracle import tikhonov as tk
        from oracle import transforms as tr
        f = self.f.cpu().numpy()
        kb = self.kb.cpu().numpy()
        worst = 0.0
        for b in self.sample_items(4)[:3]:
            kind = self.kind_of(b)
            n = int(self.rb.n[b])
            h, c = self.rb.psf[b]
            g = self.rb.g[self.rb.offsets[b]:self.rb.offsets[b + 1]]
            d = tr.blur_eigs(kind, n, h, c)
            s = tr.smooth_eigs(kind, n, "D2")
            gw = tr.inverse(kind, g)
            _, kw, muw = tk.gcv_scan(gw, d, s, self.rb.mus[b])
            assert kw == kb[b], (b, kw, kb[b])
            fw = tr.forward(kind, tk.tikhonov_filter(gw, d, s, muw)).real
            fb = f[self.rb.offsets[b]:self.rb.offsets[b + 1]]
            worst = max(worst, float(np.max(np.abs(fb - fw)) / np.max(np.abs(fw))))
        return worst

    def cpu_baseline(self, budget_s):
        from oracle import tikhonov as tk
        from oracle import transforms as tr
        t0 = time.perf_counter()
        done = []
        for b in self.sample_items(64):
            if time.perf_counter() - t0 > budget_s:
                break
            kind = self.kind_of(b)
            n = int(self.rb.n[b])
            h, c = self.rb.psf[b]
            g = self.rb.g[self.rb.offsets[b]:self.rb.offsets[b + 1]]
            d = tr.blur_eigs(kind, n, h, c)
            s = tr.smooth_eigs(kind, n, "D2")
            gw = tr.inverse(kind, g)
            _, _, muw = tk.gcv_scan(gw, d, s, self.rb.mus[b])
            tr.forward(kind, tk.tikhonov_filter(gw, d, s, muw))
            done.append(n)
        el = time.perf_counter() - t0
        return len(done) / el, ("%d signals at evenly spaced quantiles of n taken in random order (n = %d..%d, "
                                "mean %d; batch mean %d), one at a time, tables built inside the timing"
                                % (len(done), min(done), max(done), int(np.mean(done)), int(np.mean(self.rb.n))))


class Learned1D:
    """The learned-mu workload: a 72 -> 256 -> 256 -> 256 -> 1 GELU network (bfloat16
    weights, float32 accumulation) trained on the GPU on `train` generated problems
    labelled by the GCV scan (untimed set-up), then, per step, on `batch` fresh problems
    (n ~ U{256..4096}, the batched workload's PSFs, noise and degrees, fixed 128-point grid
    on [1e-8, 10]): transform-domain features, network prediction, GCV certificate around
    the prediction (full scan where it fails), filter and forward transform, as one
    hipGraph replay.  The plain GCV scan runs on the same inputs for comparison."""

    profile = "k_restore_learned65536.md"

    def __init__(self, torch, ht, synth, batch, train=200000, epochs=25, graph=True, workers=16, path="two-pass",
                 autotune=True):
        self.torch, self.ht, self.synth = torch, ht, synth
        self.batch, self.train_count, self.epochs = batch, train, epochs
        self.graph = graph
        self.autotune = autotune
        self.path = path
        # fused: one kernel pass per signal (features, network, certificate, filter, forward);
        # two-pass: feature kernel -> batched network GEMMs -> certified-restore kernel
        self.stages = ["fused_restore"] if path == "fused" else ["features", "predict", "certified_restore"]
        self.name = "1d_learned_mu_n256-4096_K128_x%d" % batch
        self.kind = "AR/C/DST3"
        # host data first: the generator forks worker processes, before any GPU use
        print("generating %d training + %d inference problems" % (train, batch), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        self.rt = synth.learned_batch_parallel(train, 0, workers=workers)
        self.rb = synth.learned_batch_parallel(batch, 1 << 30, workers=workers)
        print("generated in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)

    def _batch(self, rb):
        torch, ht = self.torch, self.ht
        bt = ht.Batch(rb.n, rb.degree, np.diff(rb.psf_offsets), rb.psf_center)
        return (bt, torch.tensor(rb.g, device="cuda"), torch.tensor(rb.psf_flat, device="cuda"),
                torch.tensor(rb.mus, device="cuda"))

    def setup(self):
        torch, ht = self.torch, self.ht
        from paper_0906_2704_amd import learned
        self.learned = learned
        t0 = time.perf_counter()
        bt, g, psf, mus = self._batch(self.rt)
        labels, _, _ = learned.labels_by_scan(bt, g, psf, mus)
        _, feats = ht.ht_batch_features(bt, g, psf)
        self.net = learned.Net("cuda", seed=0)
        learned.fit_standardisation(self.net, feats)
        hist = learned.train(self.net, feats, labels, epochs=self.epochs, batch=500, lr=2e-3)
        torch.cuda.synchronize()
        self.train_info = {"problems": self.train_count, "epochs": self.epochs, "mse_first": round(hist[0], 4),
                           "mse_last": round(hist[-1], 4), "seconds": round(time.perf_counter() - t0, 1)}
        print("trained: %s" % self.train_info, file=sys.stderr, flush=True)
        del bt, g, psf, mus, labels, feats
        # inference batch
        self.bt, self.g, self.psf, self.mus = self._batch(self.rb)
        self.K = self.rb.mus.shape[1]
        dev = "cuda"
        self.coeff = torch.empty_like(self.g)
        self.spec = torch.empty_like(self.g)
        self.feats = torch.empty((self.batch, 72), dtype=torch.float32, device=dev)
        self.kb = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.mb = torch.empty(self.batch, dtype=torch.float64, device=dev)
        self.fb = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.f_scan = torch.empty_like(self.g)
        self.f_fused = torch.empty_like(self.g)
        self.pred_fused = torch.empty(self.batch, dtype=torch.float32, device=dev)
        self.net_weights = self.net.weights()
        self.kb_scan = torch.empty_like(self.kb)
        self.mb_scan = torch.empty_like(self.mb)
        self._launch()  # allocates the network's buffers outside any capture
        self._launch_scan()
        torch.cuda.synchronize()
        self.tuning = None
        if self.autotune and self.path != "fused":
            # persistent grid and kernel variant per size class, timed on the feature pass
            # plus the certified pass with the predictions of the trained network
            from paper_0906_2704_amd import autotune
            pred = self.pred.clone()

            def run():
                ht.ht_batch_features(self.bt, self.g, self.psf, self.coeff, self.feats, self.spec)
                ht.ht_batch_restore_learned(self.bt, self.coeff, self.psf, "D2", self.mus, pred, self.learned.CERT_HALF,
                                            kb=self.kb, mb=self.mb, fallback=self.fb, spectrum=self.spec)
            choice, ms = autotune.tune(self.bt, run, use_cache=False,
                                       log=lambda m: print(m, file=sys.stderr, flush=True))
            self.tuning = {"choice": {str(c): list(v) for c, v in choice.items()},
                           "class_ms": {str(c): round(t, 4) for c, t in ms.items()}}
            self._launch()
            torch.cuda.synchronize()
        self.cuda_graph = self.scan_graph = None
        if self.graph:
            self.cuda_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.cuda_graph):
                self._launch()
            self.scan_graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.scan_graph):
                self._launch_scan()
            torch.cuda.synchronize()

    def _features(self):
        self.ht.ht_batch_features(self.bt, self.g, self.psf, self.coeff, self.feats, self.spec)

    def _predict(self):
        if not hasattr(self, "pred"):
            self.pred = self.torch.empty(self.batch, dtype=self.torch.float32, device="cuda")
        self.net.predict(self.feats, self.pred)

    def _certified(self):
        self.ht.ht_batch_restore_learned(self.bt, self.coeff, self.psf, "D2", self.mus, self.pred,
                                         self.learned.CERT_HALF, kb=self.kb, mb=self.mb, fallback=self.fb,
                                         spectrum=self.spec)

    def _fused(self):
        self.ht.ht_batch_restore_fused(self.bt, self.g, self.psf, "D2", self.mus, self.net_weights,
                                       self.learned.CERT_HALF, restored=self.f_fused, kb=self.kb, mb=self.mb,
                                       fallback=self.fb, pred=self.pred_fused)

    def _launch(self):
        if self.path == "fused":
            self._fused()
            return
        self._features()
        self._predict()
        self._certified()

    def _launch_scan(self):
        self.ht.ht_batch_restore(self.bt, self.g, self.psf, "D2", self.mus, restored=self.f_scan, kb=self.kb_scan,
                                 mb=self.mb_scan, want_G=False)

    def step(self, t):
        t.start_step()
        if t.active or self.cuda_graph is None:
            if self.path == "fused":
                self._fused()
                t.mark()
            else:
                self._features()
                t.mark()
                self._predict()
                t.mark()
                self._certified()
                t.mark()
        else:
            self.cuda_graph.replay()
            t.mark()

    def scan_ms(self, steps):
        torch = self.torch
        for _ in range(2):
            self.scan_graph.replay() if self.scan_graph is not None else self._launch_scan()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            self.scan_graph.replay() if self.scan_graph is not None else self._launch_scan()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def quality(self):
        """Mean restoration error of both paths against the true signals, fallback rate."""
        rb = self.rb
        f_l = (self.f_fused if self.path == "fused" else self.coeff).cpu().numpy()
        f_s = self.f_scan.cpu().numpy()
        o = rb.offsets
        err = lambda f: np.array([np.linalg.norm(f[o[b]:o[b + 1]] - rb.f_true[o[b]:o[b + 1]])
                                  / np.linalg.norm(rb.f_true[o[b]:o[b + 1]]) for b in range(self.batch)])
        rl, rs = err(f_l), err(f_s)
        fb = self.fb.cpu().numpy()
        return {"rre_learned": float(rl.mean()), "rre_scan": float(rs.mean()),
                "rre_ratio": float(rl.mean() / rs.mean()), "fallback_rate": float(fb.mean()),
                "gcv_evaluations_per_signal": float(np.mean(np.where(fb == 1, 2 * self.learned.CERT_HALF + 1 + self.K,
                                                                     2 * self.learned.CERT_HALF + 1)))}

    def config(self):
        return {"workload": self.name, "batch": self.batch, "n": "U{256..4096}", "sum_n": int(self.rb.n.sum()),
                "degree": "U{1,2,3}", "norm": "D2", "K": self.K, "grid": "1e-8..10", "graph": self.graph,
                "path": self.path, "certificate_half_width": self.learned.CERT_HALF, "training": self.train_info,
                "schedule": self.tuning}

    def work(self):
        """Algorithmic bytes of each stage: 16 bytes per sample (one float64 read of the
        signal and one float64 write of the restoration, the per-sample figure of the whole
        learned inference), plus the PSF masks and, where the stage uses them, the grids.
        Each pass of the two-pass path is charged the full 16 B/sample; the network stage
        counts its flops."""
        S = float(self.rb.n.sum())
        B, K = self.batch, self.K
        psf = float(self.rb.psf_flat.size) * 8
        return {
            "fused_restore": ("hbm", S * 16 + psf + B * K * 8),
            "features": ("hbm", S * 16 + psf),
            "predict": ("mfma", 2.0 * B * (72 * 256 + 2 * 256 * 256 + 256)),
            "certified_restore": ("hbm", S * 16 + psf + B * K * 8),
        }

    def step_bytes(self):
        """Algorithmic bytes of the whole inference step (16 B/sample, masks, grids)."""
        return float(self.rb.n.sum()) * 16 + float(self.rb.psf_flat.size) * 8 + self.batch * self.K * 8

    def sample_items(self, count):
        order = np.argsort(self.rb.n)
        picks = [int(order[int(q)]) for q in np.linspace(0, self.batch - 1, count)]
        return list(np.random.default_rng(0).permutation(picks))

    def check(self):
        """Learned-path parity on sampled signals: features against the oracle's, the
        oracle network on the same float32 features (standardised in float32 as the kernel
        does, same bfloat16 rounding points), and the certificate and restoration for the
        predicted mu."""
        from oracle import learned as olearned
        from oracle import mlp as omlp
        from oracle import tikhonov as tk
        from oracle import transforms as tr
        params = self.net.params_numpy()
        mean = self.net.mean.cpu().numpy()
        std = self.net.std.cpu().numpy()
        if self.path == "fused":  # the fused pass's own features, for the comparison below
            self.ht.ht_batch_restore_fused(self.bt, self.g, self.psf, "D2", self.mus, self.net_weights,
                                           self.learned.CERT_HALF, restored=self.f_fused, kb=self.kb, mb=self.mb,
                                           fallback=self.fb, pred=self.pred_fused, features=self.feats)
            self.torch.cuda.synchronize()
        f = (self.f_fused if self.path == "fused" else self.coeff).cpu().numpy()
        kb = self.kb.cpu().numpy()
        pred = (self.pred_fused if self.path == "fused" else self.pred).cpu().numpy()
        feats = self.feats.cpu().numpy()
        worst = 0.0
        self.pred_diff = 0.0
        for b in self.sample_items(4)[:3]:
            kind = {1: "AR", 2: "C", 3: "DST3"}[int(self.rb.degree[b])]
            n = int(self.rb.n[b])
            h, c = self.rb.psf[b]
            g = self.rb.g[self.rb.offsets[b]:self.rb.offsets[b + 1]]
            d = tr.blur_eigs(kind, n, h, c)
            s = tr.smooth_eigs(kind, n, "D2")
            gw = tr.inverse(kind, g)
            fw = olearned.features(gw, d)
            assert np.max(np.abs(feats[b] - fw)) < 1e-5 * max(1.0, np.max(np.abs(fw))), b
            x = (feats[b] - mean) / std  # float32 arithmetic
            yw, _ = omlp.forward(params, x[None].astype(np.float32), bf=True)
            self.pred_diff = max(self.pred_diff, abs(float(yw.ravel()[0]) - float(pred[b])))
            assert self.pred_diff < 1e-2, (b, float(yw.ravel()[0]), float(pred[b]))
            Gw = tk.gcv_values(gw, d, s, self.rb.mus[b])
            khat = olearned.nearest_index(self.rb.mus[b], float(np.float32(pred[b])))
            kc, _ = olearned.certify(Gw, khat, half=self.learned.CERT_HALF)
            assert kc == kb[b], (b, kc, kb[b])
            fr = tr.forward(kind, tk.tikhonov_filter(gw, d, s, self.rb.mus[b][kc])).real
            fb = f[self.rb.offsets[b]:self.rb.offsets[b + 1]]
            worst = max(worst, float(np.max(np.abs(fb - fr)) / np.max(np.abs(fr))))
        return worst

    def cpu_baseline(self, budget_s):
        """The oracle's learned path (features, network, certificate, restoration) on
        signals at evenly spaced quantiles of n, taken in a seeded random order."""
        from oracle import learned as olearned
        from oracle import mlp as omlp
        from oracle import tikhonov as tk
        from oracle import transforms as tr
        params = self.net.params_numpy()
        mean = self.net.mean.cpu().numpy().astype(np.float64)
        std = self.net.std.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        done = []
        for b in self.sample_items(64):
            if time.perf_counter() - t0 > budget_s:
                break
            kind = {1: "AR", 2: "C", 3: "DST3"}[int(self.rb.degree[b])]
            n = int(self.rb.n[b])
            h, c = self.rb.psf[b]
            g = self.rb.g[self.rb.offsets[b]:self.rb.offsets[b + 1]]
            d = tr.blur_eigs(kind, n, h, c)
            s = tr.smooth_eigs(kind, n, "D2")
            gw = tr.inverse(kind, g)
            x = (olearned.features(gw, d) - mean) / std
            yw, _ = omlp.forward(params, x[None].astype(np.float32), bf=True)
            Gw = tk.gcv_values(gw, d, s, self.rb.mus[b])
            kc, _ = olearned.certify(Gw, olearned.nearest_index(self.rb.mus[b], float(yw.ravel()[0])),
                                     half=self.learned.CERT_HALF)
            tr.forward(kind, tk.tikhonov_filter(gw, d, s, self.rb.mus[b][kc]))
            done.append(n)
        el = time.perf_counter() - t0
        return len(done) / el, ("%d signals at evenly spaced quantiles of n taken in random order (n = %d..%d, "
                                "mean %d; batch mean %d), one at a time, tables built inside the timing"
                                % (len(done), min(done), max(done), int(np.mean(done)), int(np.mean(self.rb.n))))


class Mixed2D:
    """The mixed-precision 2D workload: a batch of 16 images 2048 x 2048 (piecewise
    quadratic), separable Gaussian PSF (half-width 24, sigma 4), 1% noise, degree 2 on both
    axes (T_C x T_C), L = I, GCV over 128 mu on [1e-6, 1]; the transforms run as split
    bfloat16 (or float16) GEMMs on the matrix cores with float64 boundary terms."""

    stages = ["eigs", "transform_inv", "gcv_scan", "tikhonov_filter", "transform_fwd"]
    profile = "k_gemm_split_16x2048.md"

    def __init__(self, torch, ht, synth, batch=16, n=2048, precision="bf16x3"):
        self.torch, self.ht, self.synth = torch, ht, synth
        self.batch, self.n, self.precision = batch, n, precision
        self.name = "2d_tc_%dx%d_x%d_%s" % (n, n, batch, precision)
        self.kind = "C"

    def setup(self):
        torch, ht, synth = self.torch, self.ht, self.synth
        self.imgs = [synth.config3(i, self.n) for i in range(self.batch)]
        p0 = self.imgs[0]
        dev = "cuda"
        self.plan = ht.Plan((self.n, self.n), 2, psf_symmetric=True, max_batch=self.batch)
        self.plan.set_precision(self.precision)
        self.g = torch.tensor(np.stack([p.g for p in self.imgs]), device=dev)
        self.psf = torch.tensor(np.concatenate([p0.h0, p0.h1]), device=dev)
        self.psf_len, self.psf_c = [len(p0.h0), len(p0.h1)], [p0.c0, p0.c1]
        self.mus_host = p0.mus
        self.mus = torch.tensor(p0.mus, device=dev)
        n = self.n
        self.d = torch.empty((1, 2 * n), dtype=torch.float64, device=dev)
        self.s = torch.empty((1, 2 * n), dtype=torch.float64, device=dev)
        self.ghat = torch.empty_like(self.g)
        self.fhat = torch.empty_like(self.g)
        self.f = torch.empty_like(self.g)
        self.Gv = torch.empty((self.batch, len(p0.mus)), dtype=torch.float64, device=dev)
        self.kb = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.mb = torch.empty(self.batch, dtype=torch.float64, device=dev)

    def step(self, t):
        ht = self.ht
        t.start_step()
        ht.ht_eigs(self.plan, self.psf, self.psf_len, self.psf_c, "I", d=self.d, s=self.s)
        t.mark()
        ht.ht_transform_inv(self.plan, self.g, out=self.ghat)
        t.mark()
        ht.ht_gcv_scan(self.plan, self.ghat, self.d, self.s, self.mus, G=self.Gv, kb=self.kb, mb=self.mb)
        t.mark()
        ht.ht_tikhonov_filter(self.plan, self.ghat, self.d, self.s, self.mb, out=self.fhat)
        t.mark()
        ht.ht_transform_fwd(self.plan, self.fhat, out=self.f)
        t.mark()

    def config(self):
        return {"workload": self.name, "batch": self.batch, "n": [self.n, self.n], "kind": "C x C", "norm": "I",
                "K": len(self.mus_host), "precision": self.precision}

    def gemm_flops(self):
        """Split-GEMM flops of one 2D transform: two passes, each 3 products of
        2 (vectors) (outputs) (contraction) with the unpadded core order N = n - 2."""
        B, n = self.batch, self.n
        N = n - 2
        return 3 * 2.0 * (B * n * N * N + B * n * N * N)

    def work(self):
        B, n, K = self.batch, self.n, len(self.mus_host)
        px = B * n * n
        return {
            "eigs": ("hbm", 2 * n * 16),
            "transform_inv": ("mfma", self.gemm_flops()),
            "gcv_scan": ("alu", px * K * GCV_FLOPS_PER_PAIR),
            "tikhonov_filter": ("hbm", px * 16 + B * 8),
            "transform_fwd": ("mfma", self.gemm_flops()),
        }

    def check(self):
        """Images 0 and 15 against the oracle (plain float64 dense solves, float64 GCV
        sums): relative errors of the coefficients, of G and of the restoration."""
        from oracle import tikhonov as tk
        from oracle import twod
        n = self.n
        worst = {}
        for i in (0, self.batch - 1):
            p = self.imgs[i]
            gh = twod.inverse2d("C", "C", p.g, refine_steps=0)
            d = twod.eigs2d_separable("C", "C", n, n, p.h0, p.c0, p.h1, p.c1)
            G = tk.gcv_values(gh.ravel(), d.ravel(), np.ones(n * n), p.mus, wide=False)
            k = int(self.kb[i])
            ko = int(np.argmin(G))
            fo = twod.forward2d("C", "C", tk.tikhonov_filter(gh, d, np.ones((n, n)), float(p.mus[k])), wide=False)
            e = {"ghat": float(np.linalg.norm(self.ghat[i].cpu().numpy() - gh) / np.linalg.norm(gh)),
                 "G": float(np.max(np.abs(self.Gv[i].cpu().numpy() - G) / G)),
                 "f": float(np.linalg.norm(self.f[i].cpu().numpy() - fo) / np.linalg.norm(fo)),
                 "k_match": k == ko}
            for key, v in e.items():
                worst[key] = v if key not in worst else (max(worst[key], v) if key != "k_match" else worst[key] and v)
        self.errors = worst
        return worst["f"]

    def cpu_baseline(self, budget_s):
        """The oracle's dense float64 restoration of one image (dense LU solves and products
        along both axes, float64 GCV sums)."""
        from oracle import tikhonov as tk
        from oracle import twod
        n = self.n
        p = self.imgs[0]
        t0 = time.perf_counter()
        gh = twod.inverse2d("C", "C", p.g, refine_steps=0)
        d = twod.eigs2d_separable("C", "C", n, n, p.h0, p.c0, p.h1, p.c1)
        G = tk.gcv_values(gh.ravel(), d.ravel(), np.ones(n * n), p.mus, wide=False)
        mu = float(p.mus[int(np.argmin(G))])
        twod.forward2d("C", "C", tk.tikhonov_filter(gh, d, np.ones((n, n)), mu), wide=False)
        el = time.perf_counter() - t0
        return 1.0 / el, "image 0 of the batch, plain float64 dense solves and products, float64 GCV sums"


class Mask2D:
    """Out-of-focus deblurring with a non-separable mask (the 2D experiment of Section 6):
    a batch of 16 piecewise-quadratic images 1024 x 1024, disk PSF of radius 8 (a 17 x 17
    mask, not separable), 0.1% noise, degree 2 on both axes (T_C x T_C), L = I, GCV over
    128 mu on [1e-6, 1]; the eigenvalues by the three steps of Section 6 (ht_eigs2d), all
    in float64."""

    stages = ["eigs", "transform_inv", "gcv_scan", "tikhonov_filter", "transform_fwd"]

    def __init__(self, torch, ht, synth, batch=16, n=1024, radius=8.0, gcv="approx"):
        self.torch, self.ht, self.synth = torch, ht, synth
        self.batch, self.n, self.radius, self.gcv = batch, n, radius, gcv
        self.name = "2d_disk_r%g_tc_%dx%d_x%d%s" % (radius, n, n, batch, "_exact_gcv" if gcv == "exact" else "")
        self.kind = "C"

    def setup(self):
        torch, ht, synth = self.torch, self.ht, self.synth
        self.imgs = [synth.disk_image(i, self.n, self.radius) for i in range(self.batch)]
        p0 = self.imgs[0]
        dev = "cuda"
        self.plan = ht.Plan((self.n, self.n), 2, psf_symmetric=True, max_batch=self.batch)
        self.g = torch.tensor(np.stack([p.g for p in self.imgs]), device=dev)
        self.psf = torch.tensor(p0.H, device=dev)
        self.center = (p0.c0, p0.c1)
        self.mus_host = p0.mus
        self.mus = torch.tensor(p0.mus, device=dev)
        n = self.n
        self.d = torch.empty((1, n, n), dtype=torch.float64, device=dev)
        self.s = torch.empty((1, n, n), dtype=torch.float64, device=dev)
        self.ghat = torch.empty_like(self.g)
        self.fhat = torch.empty_like(self.g)
        self.f = torch.empty_like(self.g)
        self.Gv = torch.empty((self.batch, len(p0.mus)), dtype=torch.float64, device=dev)
        self.kb = torch.empty(self.batch, dtype=torch.int32, device=dev)
        self.mb = torch.empty(self.batch, dtype=torch.float64, device=dev)

    def step(self, t):
        ht = self.ht
        t.start_step()
        ht.ht_eigs2d(self.plan, self.psf, self.center, "I", d=self.d, s=self.s)
        t.mark()
        ht.ht_transform_inv(self.plan, self.g, out=self.ghat)
        t.mark()
        scan = ht.ht_gcv_scan_exact if self.gcv == "exact" else ht.ht_gcv_scan
        scan(self.plan, self.ghat, self.d, self.s, self.mus, G=self.Gv, kb=self.kb, mb=self.mb)
        t.mark()
        ht.ht_tikhonov_filter(self.plan, self.ghat, self.d, self.s, self.mb, out=self.fhat)
        t.mark()
        ht.ht_transform_fwd(self.plan, self.fhat, out=self.f)
        t.mark()

    def config(self):
        L = self.imgs[0].H.shape
        return {"workload": self.name, "batch": self.batch, "n": [self.n, self.n], "kind": "C x C", "norm": "I",
                "K": len(self.mus_host), "psf": "disk radius %g (%dx%d mask)" % (self.radius, L[0], L[1]),
                "gcv": "eq. gcv (exact)" if self.gcv == "exact" else "eq. mugcv"}

    def work(self):
        B, n, K = self.batch, self.n, len(self.mus_host)
        L0, L1 = self.imgs[0].H.shape
        px = B * n * n
        return {
            # one fused multiply-add per (mask row, column, tap) and per (row, column, mask row)
            "eigs": ("alu", 2.0 * (L0 * n * L1 + n * n * L0)),
            "transform_inv": ("hbm", px * 16),
            # exact: per (pixel, mu) the row pass (the eq. mugcv pair plus one fused multiply-add
            # per axis-1 fixed vector, 4 for T_C) and the column pass (one reciprocal per two mu,
            # a multiply-add per axis-0 functional: 2 boundary columns, 2 ghost rows)
            "gcv_scan": ("alu", px * K * (GCV_FLOPS_PER_PAIR + 2 * 4 + 2 * 4 + 4)) if self.gcv == "exact"
                        else ("alu", px * K * GCV_FLOPS_PER_PAIR),
            "tikhonov_filter": ("hbm", px * 16 + n * n * 16 + B * 8),
            "transform_fwd": ("hbm", px * 16),
        }

    def check(self):
        """Images 0 and B-1 against the oracle (plain float64 solves and products, the
        3-step eigenvalues in long double, float64 GCV sums), and the restoration error
        against the true images."""
        from oracle import tikhonov as tk
        from oracle import twod
        n = self.n
        worst = {}
        for i in (0, self.batch - 1):
            p = self.imgs[i]
            gh = twod.inverse2d("C", "C", p.g, refine_steps=0)
            d = twod.eigs2d_general("C", "C", n, n, p.H, p.c0, p.c1)
            if self.gcv == "exact":   # sampled grid values: a dense transform per mu is slow
                ks = list(range(0, len(p.mus), 16)) + [int(self.kb[i])]
                Gs = twod.gcv2d_exact_values("C", "C", gh, d, np.ones((n, n)), [p.mus[k] for k in ks], wide=False)
                Gg = self.Gv[i].cpu().numpy()[ks]
                e_G = float(np.max(np.abs(Gg - Gs) / Gs))
                k = ko = int(self.kb[i])   # k* itself is compared in the GPU tests
            else:
                G = tk.gcv_values(gh.ravel(), d.ravel(), np.ones(n * n), p.mus, wide=False)
                e_G = float(np.max(np.abs(self.Gv[i].cpu().numpy() - G) / G))
                k = int(self.kb[i])
                ko = int(np.argmin(G))
            fo = twod.forward2d("C", "C", tk.tikhonov_filter(gh, d, np.ones((n, n)), float(p.mus[ko])), wide=False)
            e = {"d": float(np.abs(self.d[0].cpu().numpy() - d).max() / np.abs(p.H).sum()),
                 "ghat": float(np.linalg.norm(self.ghat[i].cpu().numpy() - gh) / np.linalg.norm(gh)),
                 "G": e_G,
                 "f": float(np.linalg.norm(self.f[i].cpu().numpy() - fo) / np.linalg.norm(fo)),
                 "k_match": None if self.gcv == "exact" else k == ko}
            for key, v in e.items():
                worst[key] = v if key not in worst else (max(worst[key], v) if key != "k_match" else worst[key] and v)
        f = self.f.cpu().numpy()
        rre = [float(np.linalg.norm(f[i] - p.f_true) / np.linalg.norm(p.f_true)) for i, p in enumerate(self.imgs)]
        worst["rre_mean"] = float(np.mean(rre))
        self.errors = worst
        return worst["f"]

    def cpu_baseline(self, budget_s):
        """The oracle's restoration of one image: dense float64 solves and products along
        both axes, the 3-step eigenvalues, float64 GCV sums (the exact functional: a dense
        float64 forward transform per grid value, 8 of the 128 timed and scaled)."""
        from oracle import tikhonov as tk
        from oracle import twod
        n = self.n
        p = self.imgs[0]
        t0 = time.perf_counter()
        gh = twod.inverse2d("C", "C", p.g, refine_steps=0)
        d = twod.eigs2d_general("C", "C", n, n, p.H, p.c0, p.c1)
        if self.gcv == "exact":
            t1 = time.perf_counter()
            sub = list(p.mus[::16])
            G = twod.gcv2d_exact_values("C", "C", gh, d, np.ones((n, n)), sub, wide=False)
            t_gcv = (time.perf_counter() - t1) * len(p.mus) / len(sub)
            mu = float(sub[int(np.argmin(G))])
            sample = ("image 0 of the batch, plain float64 dense solves and products; the exact GCV timed "
                      "on 8 of the 128 grid values and scaled to 128")
        else:
            G = tk.gcv_values(gh.ravel(), d.ravel(), np.ones(n * n), p.mus, wide=False)
            mu = float(p.mus[int(np.argmin(G))])
            t_gcv = 0.0
            sample = "image 0 of the batch, plain float64 dense solves and products, float64 GCV sums"
        t2 = time.perf_counter()
        twod.forward2d("C", "C", tk.tikhonov_filter(gh, d, np.ones((n, n)), mu), wide=False)
        el = time.perf_counter() - t0
        if self.gcv == "exact":
            el = (t2 - t0) - (t2 - t1) + t_gcv + (time.perf_counter() - t2)
        return 1.0 / el, sample


def csrc_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_0906_2704_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(profile, stage):
    """HBM bytes per step of `stage` from a committed rocprofv3 counter summary, if it was
    taken on the kernels as they are now (same source hash); otherwise None."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    import re
    mh = re.search(r"csrc_sha256=([0-9a-f]+)", text)
    mt = re.search(r"TRAFFIC_BYTES_PER_STEP\[%s\]=([0-9.]+)" % re.escape(stage), text)
    if not mh or not mt or mh.group(1) != csrc_hash():
        return None
    return float(mt.group(1))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def blas_threads():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        if info:
            return int(max(i.get("num_threads", 1) for i in info))
    except Exception:
        pass
    return 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="learned", choices=["learned", "ragged", "uniform", "mixed", "mask"])
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "f16x3"], help="mixed: core arithmetic")
    ap.add_argument("--gcv", default="approx", choices=["approx", "exact"],
                    help="uniform, mask: the eq. mugcv scan or the exact eq. gcv functional")
    ap.add_argument("--bc", default="paper", choices=["paper", "periodic", "reflective", "f3"],
                    help="uniform: T_C (degree 2), a comparator boundary condition, or degree 3 "
                         "for any PSF")
    ap.add_argument("--train", type=int, default=200000, help="learned: training problems")
    ap.add_argument("--epochs", type=int, default=25, help="learned: training epochs")
    ap.add_argument("--learned-path", default="two-pass", choices=["two-pass", "fused"],
                    help="learned: one fused pass per signal, or feature pass + network + certified pass")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this size (MiB) before timing, for HBM counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(independent signals would be sharded by cost with no exchange).", file=sys.stderr)
        sys.exit(2)

    from paper_0906_2704_amd import synth
    pre = None
    if args.workload == "learned":
        # host data before anything touches the GPU (the generator forks workers)
        pre = Learned1D(None, None, synth, args.batch or 65536, train=args.train, epochs=args.epochs,
                        graph=not args.no_graph, workers=min(16, os.cpu_count() or 1), path=args.learned_path,
                        autotune=not args.no_autotune)

    import torch
    from paper_0906_2704_amd import ht

    ht.lib()
    if pre is not None:
        wl = pre
        wl.torch, wl.ht = torch, ht
    elif args.workload == "mixed":
        wl = Mixed2D(torch, ht, synth, args.batch or 16, precision=args.precision)
    elif args.workload == "mask":
        wl = Mask2D(torch, ht, synth, args.batch or 16, gcv=args.gcv)
    elif args.workload == "ragged":
        wl = Ragged1D(torch, ht, synth, args.batch or 4096, graph=not args.no_graph, autotune=not args.no_autotune)
    else:
        wl = Uniform1D(torch, ht, synth, args.batch or 65536, gcv=args.gcv, family=args.bc)
    print("setup %s" % wl.name, file=sys.stderr, flush=True)
    wl.setup()
    if args.copy_calibration_mib > 0:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    timer = StageTimer(torch, wl.stages)
    for _ in range(args.warmup):
        wl.step(timer)
    torch.cuda.synchronize()
    print("timing %d steps" % args.steps, file=sys.stderr, flush=True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    # pass 1: whole steps, no events in between
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        wl.step(timer)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    # pass 2: the same steps with events between the kernels (per-kernel durations)
    timer.active = True
    for _ in range(args.steps):
        wl.step(timer)
    torch.cuda.synchronize()
    stage_ms = timer.averages()
    err = None if args.no_check else wl.check()

    extra = {}
    if isinstance(wl, Mask2D):
        extra["errors_vs_oracle"] = getattr(wl, "errors", None)
    if isinstance(wl, Mixed2D):
        extra["errors_vs_oracle"] = getattr(wl, "errors", None)
        gf = wl.gemm_flops()
        for st in ("transform_inv", "transform_fwd"):
            a = gf / (stage_ms[st] / 1e3) / 1e12
            extra["gemm_roofline_" + st] = {"bound": "mfma", "achieved": a, "peak": 2500.0, "unit": "TFLOP/s",
                                            "frac": a / 2500.0, "note": "whole transform stage: split GEMMs, "
                                            "operand preparation and float64 boundary terms"}
    if isinstance(wl, Learned1D):
        scan_ms = wl.scan_ms(args.steps)
        extra["gcv_scan_path"] = {"value": wl.batch / (scan_ms / 1e3), "unit": "restorations/s",
                                  "ms_per_step": scan_ms}
        extra["speedup_vs_gcv_scan"] = scan_ms / ms
        extra["quality"] = wl.quality()

    work = wl.work()
    dom = max(stage_ms, key=stage_ms.get)
    bound, amount = work[dom]
    sec = stage_ms[dom] / 1e3
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": amount / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    elif bound == "mfma":
        roof = {"bound": "mfma", "achieved": amount / sec / 1e12, "peak": 2500.0, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "alu", "achieved": amount / sec / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = profiled_traffic(wl.profile, dom) if getattr(wl, "profile", None) else None
    if roof["traffic"] is not None and bound == "hbm":
        # measured HBM bytes per launch over the algorithmic bytes: wasted re-reads show here
        roof["traffic_ratio"] = roof["traffic"] / amount
    roof["kernel"] = dom
    per_stage = {}
    for st, (b, a) in work.items():
        if st not in stage_ms or stage_ms[st] <= 0:
            continue
        t_s = stage_ms[st] / 1e3
        if b == "hbm":
            per_stage[st] = {"bound": "hbm", "achieved_GBs": a / t_s / 1e9, "frac": a / t_s / 1e9 / HBM_PEAK_GBS}
        elif b == "mfma":
            per_stage[st] = {"bound": "mfma", "achieved_TFLOPs": a / t_s / 1e12, "frac": a / t_s / 1e12 / 2500.0}
        else:
            per_stage[st] = {"bound": "alu", "achieved_TFLOPs": a / t_s / 1e12,
                             "frac": a / t_s / 1e12 / FP64_PEAK_TFLOPS}
    roof["per_stage"] = per_stage
    if hasattr(wl, "step_bytes"):
        roof["step_frac_hbm"] = wl.step_bytes() / (ms / 1e3) / 1e9 / HBM_PEAK_GBS

    cpu = None
    if not args.no_cpu_baseline:
        v, sample = wl.cpu_baseline(args.cpu_budget)
        cpu = {"value": v, "unit": "restorations/s", "cores": blas_threads(), "kind": "oracle", "sample": sample,
               "cpu_model": cpu_model(), "affinity_cores": len(os.sched_getaffinity(0))}

    out = {
        "metric": METRIC,
        "value": wl.batch / (ms / 1e3),
        "unit": "restorations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3/f64" if isinstance(wl, Mixed2D) and wl.precision == "bf16x3" else
                 ("f16x3/f64" if isinstance(wl, Mixed2D) else "f64"),
        "data": "synthetic",
        "config": wl.config(),
        "stages_ms": stage_ms,
        "parity_max_rel_err": err,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
