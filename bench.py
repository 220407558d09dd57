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

    def __init__(self, torch, ht, synth, batch, n=256, degree=2):
        self.torch, self.ht, self.synth = torch, ht, synth
        self.batch, self.n, self.degree = batch, n, degree
        self.name = "1d_uniform_n%d_d%d_x%d" % (n, degree, batch)

    def setup(self):
        torch, ht, synth = self.torch, self.ht, self.synth
        G, F, h, c, mus = synth.config0_batch(self.batch)
        self.G_host, self.h, self.c, self.mus_host = G, h, c, mus
        dev = "cuda"
        self.plan = ht.Plan(self.n, self.degree, psf_symmetric=True)
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
        ht.ht_gcv_scan(self.plan, self.ghat, self.d, self.s, self.mus, G=self.Gv, kb=self.kb, mb=self.mb)
        t.mark()
        ht.ht_tikhonov_filter(self.plan, self.ghat, self.d, self.s, self.mb, out=self.fhat)
        t.mark()
        ht.ht_transform_fwd(self.plan, self.fhat, out=self.f)
        t.mark()

    def work(self):
        """Algorithmic bytes / flops per launch of each stage."""
        B, n, K = self.batch, self.n, len(self.mus_host)
        cb = 16 if self.plan.is_complex else 8
        return {
            "eigs": ("hbm", (len(self.h) * 8 + n * (cb + 8))),
            "transform_inv": ("hbm", B * n * (8 + cb)),
            "gcv_scan": ("alu", B * n * K * GCV_FLOPS_PER_PAIR),
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
            _, _, muw = tk.gcv_scan(gw, d, s, self.mus_host)
            tr.forward(self.kind, tk.tikhonov_filter(gw, d, s, muw))
            done += 1
        el = time.perf_counter() - t0
        return done / el, "first %d of the %d signals, one at a time" % (done, self.batch)


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
    ap.add_argument("--workload", default="uniform", choices=["uniform"])
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(independent signals would be sharded by cost with no exchange).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0906_2704_amd import ht, synth

    ht.lib()
    wl = Uniform1D(torch, ht, synth, args.batch)
    print("setup %s" % wl.name, file=sys.stderr, flush=True)
    wl.setup()
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

    work = wl.work()
    dom = max(stage_ms, key=stage_ms.get)
    bound, amount = work[dom]
    sec = stage_ms[dom] / 1e3
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": amount / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": amount / sec / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom

    cpu = None
    if not args.no_cpu_baseline:
        v, sample = wl.cpu_baseline(args.cpu_budget)
        cpu = {"value": v, "unit": "restorations/s", "cores": blas_threads(), "kind": "oracle", "sample": sample}

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "batch": wl.batch, "n": wl.n, "kind": wl.kind,
                   "norm": "D2", "K": len(wl.mus_host)},
        "stages_ms": stage_ms,
        "parity_max_rel_err": err,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
