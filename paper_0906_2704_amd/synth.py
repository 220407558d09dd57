"""Seeded synthetic workloads: piecewise-polynomial signals and images, PSF masks,
blurring of the true signal over the field of view, noise and mu grids.

This module holds no arithmetic of the restoration method; it produces the inputs both
the HIP path and the CPU checker consume.  The true signal is generated on an extended
support so that the observed samples are the plain discretised convolution of the
integral model (eq. mod_cont) over the field of view, without any boundary condition
(the boundary condition is the model's guess about what lies outside, Section 2).

PSF masks are returned as (h, center): h[idx] is the tap h_{idx-center}.
"""

from dataclasses import dataclass

import numpy as np
from scipy.ndimage import convolve1d
from scipy.signal import fftconvolve

SEED_BASE = 0x0906_2704


def rng_for(config, item):
    return np.random.default_rng([SEED_BASE, int(config), int(item)])


# ------------------------------------------------------------------------------- PSFs

def gaussian_psf(m, sigma, shift=0.0):
    j = np.arange(-m, m + 1, dtype=np.float64)
    h = np.exp(-((j - shift) ** 2) / (2.0 * sigma * sigma))
    return h / h.sum(), m


def box_psf(m):
    return np.full(2 * m + 1, 1.0 / (2 * m + 1)), m


def disk_psf(radius):
    """Out-of-focus blur: equal weights on the pixels whose centre lies within ``radius``
    of the origin, unit sum.  Even in each axis.  Returns (H, c0, c1) with H[a, b] the tap
    at offset (a - c0, b - c1)."""
    r = int(np.floor(radius))
    j = np.arange(-r, r + 1)
    H = ((j[:, None] ** 2 + j[None, :] ** 2) <= radius * radius).astype(np.float64)
    return H / H.sum(), r, r


def motion_psf(length, angle_deg):
    """Linear motion blur: a segment of ``length`` pixels that starts at the origin and
    points at ``angle_deg`` (0 = along axis 1, 90 = along axis 0), rasterised from 8
    samples per pixel rounded to the nearest pixel, unit sum.  One-sided, so not even in
    any axis unless the segment is degenerate.  Returns (H, c0, c1)."""
    t = np.linspace(0.0, float(length), 8 * int(np.ceil(length)) + 1)
    a = np.deg2rad(angle_deg)
    p0 = np.rint(t * np.sin(a)).astype(np.int64)
    p1 = np.rint(t * np.cos(a)).astype(np.int64)
    lo0, lo1 = int(p0.min()), int(p1.min())
    H = np.zeros((int(p0.max()) - lo0 + 1, int(p1.max()) - lo1 + 1))
    np.add.at(H, (p0 - lo0, p1 - lo1), 1.0)
    return H / H.sum(), -lo0, -lo1


def mask_halfwidths(H, c0, c1):
    return max(c0, H.shape[0] - 1 - c0), max(c1, H.shape[1] - 1 - c1)


def delta_psf():
    return np.array([1.0]), 0


# ---------------------------------------------------------------------------- signals

def piecewise_poly(rng, length, pieces=4, degree=3):
    """`pieces` equal contiguous pieces, each sum_p c_p t^p with local t in [-1, 1] and
    c_p ~ N(0, 1)."""
    out = np.empty(length, dtype=np.float64)
    edges = np.linspace(0, length, pieces + 1).round().astype(int)
    for a, b in zip(edges[:-1], edges[1:]):
        t = np.linspace(-1.0, 1.0, b - a)
        c = rng.standard_normal(degree + 1)
        out[a:b] = np.polyval(c[::-1], t)
    return out


def piecewise_poly_image(rng, shape, blocks=4, degree=2):
    """blocks x blocks tiles, each sum_{a+b<=degree} c_ab u^a v^b, u, v in [-1, 1]."""
    n0, n1 = shape
    img = np.empty(shape, dtype=np.float64)
    e0 = np.linspace(0, n0, blocks + 1).round().astype(int)
    e1 = np.linspace(0, n1, blocks + 1).round().astype(int)
    for a0, b0 in zip(e0[:-1], e0[1:]):
        u = np.linspace(-1.0, 1.0, b0 - a0)[:, None]
        for a1, b1 in zip(e1[:-1], e1[1:]):
            v = np.linspace(-1.0, 1.0, b1 - a1)[None, :]
            tile = np.zeros((b0 - a0, b1 - a1))
            for pa in range(degree + 1):
                for pb in range(degree + 1 - pa):
                    tile = tile + rng.standard_normal() * u ** pa * v ** pb
            img[a0:b0, a1:b1] = tile
    return img


def observe_1d(f_ext, h, center, n):
    """Observed samples g_i = sum_j h_j f_{i-j}, i = 1..n, from a true signal given on
    the extended support i = 1-mr .. n+ml (mr = len(h)-1-center, ml = center)."""
    h = np.asarray(h, dtype=np.float64)
    ml, mr = int(center), h.size - 1 - int(center)
    assert f_ext.shape[-1] == n + ml + mr
    if f_ext.ndim == 1:
        # 'valid' convolution: output i sums h[idx] f_ext[i + mr - (idx - center)]
        return np.convolve(f_ext, h, mode="valid")
    g = np.zeros(f_ext.shape[:-1] + (n,))
    for idx in range(h.size):
        j = idx - center
        # f_{i-j} for i = 1..n sits at extended position (i - j) - (1 - mr)
        start = mr - j
        g += h[idx] * f_ext[..., start:start + n]
    return g


def _observe_axis(F_ext, h, center, n, axis):
    """observe_1d along one axis of a 2D array.  For odd mask lengths L = 2m+1 the valid
    samples are entries m .. m+n-1 of the zero-padded 'same' convolution, whatever the
    centre: g_i = sum_idx h[idx] f[i + L-1 - idx]."""
    h = np.asarray(h, dtype=np.float64)
    if h.size % 2 == 0:
        if axis == 1:
            return observe_1d(F_ext, h, center, n)
        return observe_1d(F_ext.T, h, center, n).T
    m = (h.size - 1) // 2
    full = convolve1d(F_ext, h, axis=axis, mode="constant")
    return full[:, m:m + n] if axis == 1 else full[m:m + n, :]


def observe_2d(F_ext, h0, c0, h1, c1, shape):
    n0, n1 = shape
    tmp = _observe_axis(F_ext, h1, c1, n1, 1)       # along axis 1
    return _observe_axis(tmp, h0, c0, n0, 0)        # along axis 0


def observe_2d_mask(F_ext, H, c0, c1, shape):
    """Blur by a general 2D mask over the field of view: g[p, q] = sum_{a,b} H[a, b]
    f[p - (a - c0), q - (b - c1)], with F_ext the true image extended by the half-widths
    (m0, m1) of ``mask_halfwidths`` on each side.  Full linear convolution by FFT, then the
    field-of-view window."""
    n0, n1 = shape
    m0, m1 = mask_halfwidths(H, c0, c1)
    assert F_ext.shape == (n0 + 2 * m0, n1 + 2 * m1)
    full = fftconvolve(F_ext, np.asarray(H, dtype=np.float64), mode="full")
    # full[i, j] = sum H[a, b] F_ext[i - a, j - b]; p sits at i = p + m0 + c0
    return full[m0 + c0:m0 + c0 + n0, m1 + c1:m1 + c1 + n1].copy()


def add_noise(rng, g, eta):
    """e = eta ||g|| w / ||w||, w ~ N(0, I) (relative noise level eta)."""
    w = rng.standard_normal(g.shape)
    return g + eta * np.linalg.norm(g) * w / np.linalg.norm(w)


def mu_grid(lo, hi, K):
    """K log-spaced values 10^(lo + (hi-lo) k/(K-1))."""
    k = np.arange(K, dtype=np.float64)
    return 10.0 ** (lo + (hi - lo) * k / (K - 1))


# ------------------------------------------------------------------------ workloads

@dataclass
class Problem1D:
    f_true: np.ndarray      # true signal on the field of view (n)
    g: np.ndarray           # observed signal (n)
    h: np.ndarray
    center: int
    degree: int
    eta: float
    mus: np.ndarray


def signal_1d(config, item, n, h, center, eta, mus, degree=1, pieces=4, poly_degree=3):
    rng = rng_for(config, item)
    ml, mr = int(center), len(h) - 1 - int(center)
    f_ext = piecewise_poly(rng, n + ml + mr, pieces, poly_degree)
    g = add_noise(rng, observe_1d(f_ext, h, center, n), eta)
    return Problem1D(f_ext[mr:mr + n].copy(), g, np.asarray(h), int(center), degree, eta, mus)


def config0(item, degree=1):
    """1D plain method: n = 256, 4 cubic pieces, Gaussian PSF half-width 8 sigma 2,
    1% noise, 64 log-spaced mu on [1e-6, 1]."""
    h, c = gaussian_psf(8, 2.0)
    return signal_1d(0, item, 256, h, c, 0.01, mu_grid(-6.0, 0.0, 64), degree)


def config0_batch(count, first_item=0):
    """`count` seeded replicates of the n = 256 problem stacked as a (count, 256) batch."""
    h, c = gaussian_psf(8, 2.0)
    G = np.empty((count, 256))
    F = np.empty((count, 256))
    for b in range(count):
        p = signal_1d(0, first_item + b, 256, h, c, 0.01, None)
        G[b], F[b] = p.g, p.f_true
    return G, F, h, c, mu_grid(-6.0, 0.0, 64)


@dataclass
class Problem2D:
    f_true: np.ndarray
    g: np.ndarray
    h0: np.ndarray
    c0: int
    h1: np.ndarray
    c1: int
    eta: float
    mus: np.ndarray


def config1(item=0, n=512):
    """2D plain method: piecewise-quadratic image, separable nonsymmetric PSF (half-width
    12, sigmas 2.5 / 1.5, both masks centred one pixel off), 0.5% noise, 128 mu."""
    rng = rng_for(1, item)
    m = 12
    h0, c0 = gaussian_psf(m, 2.5, shift=1.0)
    h1, c1 = gaussian_psf(m, 1.5, shift=1.0)
    F_ext = piecewise_poly_image(rng, (n + 2 * m, n + 2 * m))
    g = add_noise(rng, observe_2d(F_ext, h0, c0, h1, c1, (n, n)), 0.005)
    return Problem2D(F_ext[m:m + n, m:m + n].copy(), g, h0, c0, h1, c1, 0.005,
                     mu_grid(-6.0, 0.0, 128))


def config3(item, n=2048):
    """Mixed precision: 2048 x 2048 image, separable Gaussian PSF half-width 24 sigma 4,
    1% noise, L = I, 128 mu on [1e-6, 1]."""
    rng = rng_for(3, item)
    m = 24
    h, c = gaussian_psf(m, 4.0)
    F_ext = piecewise_poly_image(rng, (n + 2 * m, n + 2 * m))
    g = add_noise(rng, observe_2d(F_ext, h, c, h, c, (n, n)), 0.01)
    return Problem2D(F_ext[m:m + n, m:m + n].copy(), g, h, c, h, c, 0.01, mu_grid(-6.0, 0.0, 128))


@dataclass
class ProblemMask2D:
    f_true: np.ndarray
    g: np.ndarray
    H: np.ndarray
    c0: int
    c1: int
    eta: float
    mus: np.ndarray


def disk_image(item, n=512, radius=6.0, eta=0.001, config=4):
    """Out-of-focus deblurring (the 2D experiment of Section 6): piecewise-quadratic
    n x n image, disk PSF of the given radius, 0.1% noise, 128 mu on [1e-6, 1]."""
    rng = rng_for(config, item)
    H, c0, c1 = disk_psf(radius)
    m0, m1 = mask_halfwidths(H, c0, c1)
    F_ext = piecewise_poly_image(rng, (n + 2 * m0, n + 2 * m1))
    g = add_noise(rng, observe_2d_mask(F_ext, H, c0, c1, (n, n)), eta)
    return ProblemMask2D(F_ext[m0:m0 + n, m1:m1 + n].copy(), g, H, c0, c1, eta, mu_grid(-6.0, 0.0, 128))


@dataclass
class RaggedBatch:
    """Concatenated signals of uneven length with per-signal PSF, degree and mu grid."""
    n: np.ndarray           # int64 [B]
    offsets: np.ndarray     # int64 [B+1] into the concatenated signal arrays
    g: np.ndarray           # float64 [sum n]
    f_true: np.ndarray      # float64 [sum n]
    degree: np.ndarray      # int32 [B]
    psf: list               # list of (h, center)
    psf_flat: np.ndarray    # float64, all masks concatenated
    psf_offsets: np.ndarray  # int64 [B+1]
    psf_center: np.ndarray  # int64 [B]
    eta: np.ndarray         # float64 [B]
    mus: np.ndarray         # float64 [B, K]


def ragged_batch(count=4096, n_lo=128, n_hi=8192, K=128, degrees=(1, 2, 3), config=2,
                 first_item=0, sort_desc=True, n_values=None, grid=None):
    """Batched workload: n ~ U{n_lo..n_hi}; Gaussian (sigma = m/3) or box PSF with equal
    probability, half-width m ~ U{2..32}; noise level log-uniform in [0.1%, 5%]; degree
    uniform over `degrees`; per-signal grid of K log-spaced mu on [10^lo, 10^(lo+7)],
    lo ~ U(-8, -6) (or the fixed grid 10^grid[0] .. 10^grid[1]).  Signals are 4 random cubic
    pieces.  Sorted by n, longest first (unless sort_desc is False)."""
    items = []
    for b in range(count):
        rng = rng_for(config, first_item + b)
        n = int(rng.integers(n_lo, n_hi + 1)) if n_values is None else int(n_values[b])
        m = int(rng.integers(2, 33))
        m = min(m, (n - 3) // 2)
        if rng.random() < 0.5:
            h, c = gaussian_psf(m, m / 3.0)
        else:
            h, c = box_psf(m)
        eta = float(10.0 ** rng.uniform(-3.0, np.log10(0.05)))
        deg = int(degrees[int(rng.integers(0, len(degrees)))])
        lo = float(rng.uniform(-8.0, -6.0))
        mus = mu_grid(lo, lo + 7.0, K) if grid is None else mu_grid(grid[0], grid[1], K)
        f_ext = piecewise_poly(rng, n + 2 * m, 4, 3)
        g = add_noise(rng, observe_1d(f_ext, h, c, n), eta)
        items.append((n, g, f_ext[m:m + n], deg, (h, c), eta, mus))
    if sort_desc:
        items.sort(key=lambda t: -t[0])
    ns = np.array([t[0] for t in items], dtype=np.int64)
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum(ns)
    psf_lens = np.array([len(t[4][0]) for t in items], dtype=np.int64)
    poffs = np.zeros(count + 1, dtype=np.int64)
    poffs[1:] = np.cumsum(psf_lens)
    return RaggedBatch(
        n=ns, offsets=offs,
        g=np.concatenate([t[1] for t in items]),
        f_true=np.concatenate([t[2] for t in items]),
        degree=np.array([t[3] for t in items], dtype=np.int32),
        psf=[t[4] for t in items],
        psf_flat=np.concatenate([t[4][0] for t in items]),
        psf_offsets=poffs,
        psf_center=np.array([t[4][1] for t in items], dtype=np.int64),
        eta=np.array([t[5] for t in items]),
        mus=np.stack([t[6] for t in items]),
    )


def concat_batches(parts):
    """One RaggedBatch from several, in order."""
    ns = np.concatenate([p.n for p in parts])
    offs = np.zeros(ns.size + 1, dtype=np.int64)
    offs[1:] = np.cumsum(ns)
    psf_lens = np.concatenate([np.diff(p.psf_offsets) for p in parts])
    poffs = np.zeros(ns.size + 1, dtype=np.int64)
    poffs[1:] = np.cumsum(psf_lens)
    return RaggedBatch(
        n=ns, offsets=offs,
        g=np.concatenate([p.g for p in parts]),
        f_true=np.concatenate([p.f_true for p in parts]),
        degree=np.concatenate([p.degree for p in parts]),
        psf=[x for p in parts for x in p.psf],
        psf_flat=np.concatenate([p.psf_flat for p in parts]),
        psf_offsets=poffs,
        psf_center=np.concatenate([p.psf_center for p in parts]),
        eta=np.concatenate([p.eta for p in parts]),
        mus=np.concatenate([p.mus for p in parts]),
    )


def _learned_chunk(args):
    return learned_batch(*args)


def learned_batch_parallel(count, first_item=0, workers=8, chunk=4096):
    """learned_batch(count, first_item) generated in worker processes (same items, same
    order).  Must run before the calling process touches the GPU (the workers are forked)."""
    import multiprocessing as mp
    jobs = [(min(chunk, count - s), first_item + s) for s in range(0, count, chunk)]
    if workers <= 1 or len(jobs) == 1:
        return concat_batches([learned_batch(c, f) for c, f in jobs])
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_learned_chunk, jobs)
    return concat_batches(parts)


def learned_batch(count, first_item=0, K=128, grid=(-8.0, 1.0)):
    """Learned-mu workload: signals as the batched workload with n ~ U{256..4096} and the
    fixed grid of K log-spaced mu on [1e-8, 10]; item order kept."""
    return ragged_batch(count, n_lo=256, n_hi=4096, K=K, config=4, first_item=first_item, sort_desc=False,
                        grid=grid)
