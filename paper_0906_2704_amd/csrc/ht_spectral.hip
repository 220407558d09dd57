// Spectra (eqs. jcf, Ac, Af and the smoothing spectra of Section 4), the reblurred
// Tikhonov filter (eq. freg) and the GCV scan (eqs. gcv2, mugcv).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fft_lds.h"
#include "ht_internal.h"

namespace ht {

// ------------------------------------------------------------------------ eigenvalues

// Eigenvalue of column i of the plan's transform: the preserved-polynomial columns carry
// z(0) = sum_j h_j; core column i carries z at frequency pi * num / den with
//   AR / DST:  num = i        (y = j pi / (n-1), core index j = i)          eq. jcf
//   C:         num = i - 1    (x = (i-1) pi / (n-2))                         eq. Ac
//   F:         num = -2(i-1)  (conj z(2 pi (i-1) / (n-2)) for the convolution model)
//   P:         num = -2i      (conj z(2 pi i / n); no polynomial columns)            eq. permat
//   R:         num = i        (x = i pi / n; no polynomial columns)                   eq. refm
//   F3:        as F, with the cubic column n-2 polynomial and Re z on the cosine column 2
// evaluated by direct summation over the taps with every angle reduced exactly.
__global__ void k_eigs(Axis ax, const double* __restrict__ psf, int64_t plen, int64_t pcenter,
                       int64_t psf_stride, int norm, double s_ident, void* d, double* s,
                       int64_t out_stride, int cplx_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (i >= ax.n) return;
    const double* h = psf + b * psf_stride;
    const int n = ax.n;
    const bool cmp = ax.kind == HT_KIND_P || ax.kind == HT_KIND_R;
    const bool f3 = ax.kind == HT_KIND_F3;
    const bool poly = !cmp && ((i == 0) || (i == n - 1) || (i >= 1 && i <= ax.rank) || (f3 && i == n - 2));
    int64_t num;
    if (ax.kind == HT_KIND_C)
        num = i - 1;
    else if (ax.kind == HT_KIND_F || f3)
        num = -2 * static_cast<int64_t>(i - 1);
    else if (ax.kind == HT_KIND_P)
        num = -2 * static_cast<int64_t>(i);
    else
        num = i;
    const int64_t period = 2 * static_cast<int64_t>(ax.den);
    double dr = 0.0, di = 0.0, sv;
    if (poly) {
        for (int64_t k = 0; k < plen; ++k) dr += h[k];
        sv = norm == HT_NORM_IDENTITY ? s_ident : 0.0;
    } else {
        for (int64_t k = 0; k < plen; ++k) {
            int64_t r = ((k - pcenter) * num) % period;
            if (r < 0) r += period;
            dr = fma(h[k], ax.tcos[r], dr);
            di = fma(h[k], ax.tsin[r], di);
        }
        if (f3 && i == 2) di = 0.0;  // the cosine column: Re z(x_1)
        int64_t r = num % period;
        if (r < 0) r += period;
        sv = norm == HT_NORM_IDENTITY ? s_ident : 2.0 - 2.0 * ax.tcos[r];
    }
    const int64_t o = b * out_stride + i;
    if (cplx_out)
        static_cast<double2*>(d)[o] = make_double2(dr, di);
    else
        static_cast<double*>(d)[o] = dr;
    s[o] = sv;
}

// ------------------------------------------------------------- eigenvalues, 2D masks

// Frequency number of column i (angle pi * num / den), 0 on the polynomial columns.
__device__ __forceinline__ int64_t freq_num(const Axis& ax, int i) {
    if (ax.kind == HT_KIND_P) return -2 * static_cast<int64_t>(i);
    if (ax.kind == HT_KIND_R) return i;
    const bool poly = (i == 0) || (i == ax.n - 1) || (i >= 1 && i <= ax.rank);
    if (poly) return 0;
    if (ax.kind == HT_KIND_C) return i - 1;
    if (ax.kind == HT_KIND_F) return -2 * static_cast<int64_t>(i - 1);
    return i;
}

// angle index of offset * num modulo 2 den, in [0, 2 den)
__device__ __forceinline__ int64_t angle_index(int64_t offset, int64_t num, int64_t period) {
    int64_t r = (offset * num) % period;
    return r < 0 ? r + period : r;
}

// Step one of the factorisation: W[b][a][j] = sum_k H[b][a][k] e^{i (k - c1) u_j} over
// the taps of mask row a, at the axis-1 frequency u_j of column j (cos only for the real
// kinds: the part of the row even about c1).  One thread per (j, a, b); the angle index
// advances by num_j per tap, so the loop has no division.
template <bool CPLX>
__global__ void k_eigs2d_rows(Axis ax1, const double* __restrict__ psf, int64_t len0, int64_t len1,
                              int64_t c1, double2* __restrict__ W) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t a = blockIdx.y, b = blockIdx.z;
    if (j >= ax1.n) return;
    const double* h = psf + (b * len0 + a) * len1;
    const int64_t period = 2 * static_cast<int64_t>(ax1.den);
    const int64_t num = freq_num(ax1, j);
    const int64_t step = angle_index(1, num, period);
    int64_t r = angle_index(-c1, num, period);
    double wr = 0.0, wi = 0.0;
    for (int64_t k = 0; k < len1; ++k) {
        wr = fma(h[k], ax1.tcos[r], wr);
        if (CPLX) wi = fma(h[k], ax1.tsin[r], wi);
        r += step;
        if (r >= period) r -= period;
    }
    W[(b * len0 + a) * ax1.n + j] = make_double2(wr, wi);
}

constexpr int E2_TJ = 64;     // columns per tile (one per lane)
constexpr int E2_RG = 4;      // row groups (waves) per tile
constexpr int E2_RPT = 16;    // rows per thread
constexpr int E2_TI = E2_RG * E2_RPT;
constexpr int E2_AC = 32;     // mask rows per LDS chunk

// Step two: d[b][i][j] = sum_a W[b][a][j] e^{i (a - c0) t_i} (real kinds: cos and the
// real part of W, i.e. sum H cos cos), and s[b][i][j].  A 64 x 64 tile per block: lane j
// of wave g owns rows g, g + 4, ... of the tile; the factors e^{i (a - c0) t_i} of a
// chunk of mask rows are staged in LDS, W[a][j] is read once per tile from global memory.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_eigs2d_cols(Axis ax0, Axis ax1, const double2* __restrict__ W,
                                                     int64_t len0, int64_t c0, int norm, void* d, double* s) {
    __shared__ double2 E[E2_AC][E2_TI];
    const int jj = threadIdx.x & (E2_TJ - 1), g = threadIdx.x / E2_TJ;
    const int j = blockIdx.x * E2_TJ + jj;
    const int i0 = blockIdx.y * E2_TI;
    const int64_t b = blockIdx.z;
    const int n0 = ax0.n, n1 = ax1.n;
    const int64_t period0 = 2 * static_cast<int64_t>(ax0.den);
    double2 acc[E2_RPT];
#pragma unroll
    for (int r = 0; r < E2_RPT; ++r) acc[r] = make_double2(0.0, 0.0);
    const double2* Wb = W + b * len0 * n1;
    for (int64_t a0 = 0; a0 < len0; a0 += E2_AC) {
        __syncthreads();
        for (int e = threadIdx.x; e < E2_AC * E2_TI; e += 256) {
            const int aa = e / E2_TI, ii = e - aa * E2_TI;
            const int i = i0 + ii;
            const int64_t num = i < n0 ? freq_num(ax0, i) : 0;
            const int64_t r = angle_index(a0 + aa - c0, num, period0);
            E[aa][ii] = make_double2(ax0.tcos[r], ax0.tsin[r]);
        }
        __syncthreads();
        const int na = static_cast<int>(len0 - a0 < E2_AC ? len0 - a0 : E2_AC);
        if (j < n1) {
            for (int aa = 0; aa < na; ++aa) {
                const double2 w = Wb[(a0 + aa) * n1 + j];
#pragma unroll
                for (int r = 0; r < E2_RPT; ++r) {
                    const double2 e = E[aa][g + E2_RG * r];
                    if (CPLX) {
                        acc[r].x = fma(w.x, e.x, fma(-w.y, e.y, acc[r].x));
                        acc[r].y = fma(w.x, e.y, fma(w.y, e.x, acc[r].y));
                    } else {
                        acc[r].x = fma(w.x, e.x, acc[r].x);
                    }
                }
            }
        }
    }
    if (j >= n1) return;
    const int64_t num1 = freq_num(ax1, j);
    const double s1 = num1 == 0 ? 0.0 : 2.0 - 2.0 * ax1.tcos[angle_index(1, num1, 2 * static_cast<int64_t>(ax1.den))];
#pragma unroll
    for (int r = 0; r < E2_RPT; ++r) {
        const int i = i0 + g + E2_RG * r;
        if (i >= n0) break;
        const int64_t o = (b * n0 + i) * n1 + j;
        if (CPLX)
            static_cast<double2*>(d)[o] = acc[r];
        else
            static_cast<double*>(d)[o] = acc[r].x;
        double sv = 1.0;
        if (norm != HT_NORM_IDENTITY) {
            const int64_t num0 = freq_num(ax0, i);
            sv = (num0 == 0 ? 0.0 : 2.0 - 2.0 * ax0.tcos[angle_index(1, num0, period0)]) + s1;
        }
        s[o] = sv;
    }
}

// ------------------------------------------------------------------- shared accessors

struct Spec {          // how to find d_i and s_i of element e of item b
    const void* d;
    const double* s;
    int factored;      // 2D separable factors [d0 | d1]; else one entry per element
    int n0, n1;        // 2D factor lengths
    int64_t eig_stride;  // 0 (shared) or per_item (one spectrum per item)
    int64_t per_item;    // elements per item (n or n0 * n1)
    int cplx;
};

__device__ __forceinline__ void spec_at(const Spec& sp, int64_t b, int64_t e, double2& dd, double& ss) {
    if (!sp.factored) {
        const int64_t o = b * sp.eig_stride + e;
        dd = sp.cplx ? static_cast<const double2*>(sp.d)[o]
                     : make_double2(static_cast<const double*>(sp.d)[o], 0.0);
        ss = sp.s[o];
    } else {
        const int64_t i0 = e / sp.n1, i1 = e - i0 * sp.n1;
        double2 a, c;
        if (sp.cplx) {
            a = static_cast<const double2*>(sp.d)[i0];
            c = static_cast<const double2*>(sp.d)[sp.n0 + i1];
        } else {
            a = make_double2(static_cast<const double*>(sp.d)[i0], 0.0);
            c = make_double2(static_cast<const double*>(sp.d)[sp.n0 + i1], 0.0);
        }
        dd = cmul(a, c);
        ss = sp.s[i0] + sp.s[sp.n0 + i1];
    }
}

__device__ __forceinline__ double2 cload(const void* p, int64_t o, int cplx) {
    return cplx ? static_cast<const double2*>(p)[o] : make_double2(static_cast<const double*>(p)[o], 0.0);
}

// --------------------------------------------------------------------------- filter

// fhat = conj(d) g / (|d|^2 + mu |s|^2): Phi D^{-1} of eq. freg without the 0/0 of a
// vanishing eigenvalue.
__global__ void k_filter(Spec sp, const void* __restrict__ coeff, const double* __restrict__ mu,
                         void* fhat, int64_t per_item, int64_t total) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t b = idx / per_item, e = idx - b * per_item;
    double2 dd;
    double ss;
    spec_at(sp, b, e, dd, ss);
    const double2 g = cload(coeff, idx, sp.cplx);
    const double den = fma(dd.x, dd.x, dd.y * dd.y) + mu[b] * (ss * ss);
    const double2 num = cmulc(g, dd);
    if (sp.cplx)
        static_cast<double2*>(fhat)[idx] = make_double2(num.x / den, num.y / den);
    else
        static_cast<double*>(fhat)[idx] = num.x / den;
}

// ----------------------------------------------------------------------------- GCV

constexpr int GCV_THREADS = 256;
constexpr int GCV_CHUNK = 2048;  // elements staged in LDS at a time

// 1/u to full float64 accuracy: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_nr(double u) {
    double r = __builtin_amdgcn_rcp(u);
    double e = fma(-u, r, 1.0);
    r = fma(r, e, r);
    e = fma(-u, r, 1.0);
    return fma(r, e, r);
}

// With sigma_i = |s_i|^2 / (|d_i|^2 + mu |s_i|^2) = 1 / (t_i + mu), t_i = |d_i|^2/|s_i|^2,
// the two sums of eq. mugcv are D(mu) = sum_i 1/(t_i + mu), N(mu) = sum_i w_i/(t_i + mu)^2
// with w_i = |ghat_i|^2.  Entries with s_i = 0 have sigma_i = 0; they are staged with
// w = 0 and t = 1e150, so that their 1/(t + mu) ~ 1e-150 rounds away against the other
// terms of D (and products of two staged t stay finite).
// Sums of two grid values (mua, mub) over the staged pairs part, part + nparts, ... < len,
// two elements at a time with one reciprocal per element pair and grid value:
// 1/u0 = u1 / (u0 u1), 1/u1 = u0 / (u0 u1).  The staged t never exceeds 1e150, so the
// products stay finite.
__device__ __forceinline__ void gcv_pair_sums(const double2* stage, int len, int part, int nparts, double mua,
                                              double mub, double& Na, double& Da, double& Nb, double& Db) {
    double na0 = 0.0, na1 = 0.0, da0 = 0.0, da1 = 0.0;
    double nb0 = 0.0, nb1 = 0.0, db0 = 0.0, db1 = 0.0;
    int i = part;
    for (; i + nparts < len; i += 2 * nparts) {
        const double2 p0 = stage[i], p1 = stage[i + nparts];
        const double ua0 = p0.x + mua, ua1 = p1.x + mua;
        const double ub0 = p0.x + mub, ub1 = p1.x + mub;
        const double ra = rcp_nr(ua0 * ua1), rb = rcp_nr(ub0 * ub1);
        const double ra0 = ua1 * ra, ra1 = ua0 * ra, rb0 = ub1 * rb, rb1 = ub0 * rb;
        da0 += ra0;
        da1 += ra1;
        db0 += rb0;
        db1 += rb1;
        na0 = fma(p0.y, ra0 * ra0, na0);
        na1 = fma(p1.y, ra1 * ra1, na1);
        nb0 = fma(p0.y, rb0 * rb0, nb0);
        nb1 = fma(p1.y, rb1 * rb1, nb1);
    }
    if (i < len) {
        const double2 p0 = stage[i];
        const double ra = rcp_nr(p0.x + mua), rb = rcp_nr(p0.x + mub);
        da0 += ra;
        db0 += rb;
        na0 = fma(p0.y, ra * ra, na0);
        nb0 = fma(p0.y, rb * rb, nb0);
    }
    Na = na0 + na1;
    Da = da0 + da1;
    Nb = nb0 + nb1;
    Db = db0 + db1;
}

// Thread (part, kl) accumulates the grid values 2 (k0 + kl) and 2 (k0 + kl) + 1 over the
// staged elements part, part + nparts, ... of each chunk; chunk totals are added in order,
// parts are added in order: the result does not depend on scheduling.
__device__ void gcv_accumulate(const Spec& sp, const void* coeff, int64_t b, int64_t e_begin,
                               int64_t e_end, const double* mus, int K, double2* part_out,
                               double2* stage, double2* red, int chunk_cap = GCV_CHUNK) {
    const int tid = threadIdx.x;
    const int Kh = (K + 1) / 2;
    const int Kb = Kh < GCV_THREADS ? Kh : GCV_THREADS;
    const int nparts = GCV_THREADS / Kb;
    const int part = tid / Kb, kl = tid - part * Kb;
    for (int k0 = 0; k0 < Kh; k0 += Kb) {
        const int kk = k0 + kl;
        const bool active = part < nparts && kk < Kh;
        const int ka = 2 * kk, kb2 = ka + 1 < K ? ka + 1 : ka;
        const double mua = active ? mus[ka] : 1.0, mub = active ? mus[kb2] : 1.0;
        double Nat = 0.0, Dat = 0.0, Nbt = 0.0, Dbt = 0.0;
        for (int64_t c0 = e_begin; c0 < e_end; c0 += chunk_cap) {
            const int len = static_cast<int>((e_end - c0) < chunk_cap ? (e_end - c0) : chunk_cap);
            __syncthreads();
            for (int i = tid; i < len; i += GCV_THREADS) {
                const int64_t e = c0 + i;
                double2 dd;
                double ss;
                spec_at(sp, b, e, dd, ss);
                const double2 g = cload(coeff, b * sp.per_item + e, sp.cplx);
                const double s2 = ss * ss;
                double t = 1e150, w = 0.0;
                if (s2 != 0.0) {
                    t = fma(dd.x, dd.x, dd.y * dd.y) / s2;
                    w = fma(g.x, g.x, g.y * g.y);
                }
                stage[i] = make_double2(t, w);
            }
            __syncthreads();
            if (active) {
                double Na, Da, Nb, Db;
                gcv_pair_sums(stage, len, part, nparts, mua, mub, Na, Da, Nb, Db);
                Nat += Na;
                Dat += Da;
                Nbt += Nb;
                Dbt += Db;
            }
        }
        __syncthreads();
        if (part < nparts) {
            red[2 * (part * Kb + kl)] = make_double2(Nat, Dat);
            red[2 * (part * Kb + kl) + 1] = make_double2(Nbt, Dbt);
        }
        __syncthreads();
        if (part == 0 && kk < Kh) {
            double2 A = red[2 * kl], B = red[2 * kl + 1];
            for (int p = 1; p < nparts; ++p) {
                const double2 va = red[2 * (p * Kb + kl)], vb = red[2 * (p * Kb + kl) + 1];
                A.x += va.x;
                A.y += va.y;
                B.x += vb.x;
                B.y += vb.y;
            }
            part_out[ka] = A;
            if (ka + 1 < K) part_out[ka + 1] = B;
        }
    }
    __syncthreads();
}


// argmin over G[0..K) in LDS by the first wave: first index of the minimum; -1 if any
// value is not finite.
__device__ void gcv_argmin(const double* G, int K, int* kbest_out) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        double best = 0.0;
        int bk = -1;
        int bad = 0;
        for (int k = tid; k < K; k += 64) {
            const double g = G[k];
            if (!isfinite(g)) bad = 1;
            if (bk < 0 || g < best) {
                best = g;
                bk = k;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int ok = __shfl_xor(bk, off, 64);
            const int obad = __shfl_xor(bad, off, 64);
            bad |= obad;
            if (ok >= 0 && (bk < 0 || ob < best || (ob == best && ok < bk))) {
                best = ob;
                bk = ok;
            }
        }
        if (tid == 0) *kbest_out = bad ? -1 : bk;
    }
    __syncthreads();
}

__device__ void gcv_finish(const double2* sums, int K, const double* mus, double* G_out,
                           int32_t* kbest_out, double* mubest_out, double* Gs, int* kshared) {
    for (int k = threadIdx.x; k < K; k += GCV_THREADS) {
        const double2 v = sums[k];
        const double g = v.x / (v.y * v.y);
        Gs[k] = g;
        if (G_out) G_out[k] = g;
    }
    __syncthreads();
    gcv_argmin(Gs, K, kshared);
    if (threadIdx.x == 0) {
        const int kb = *kshared;
        *kbest_out = kb;
        if (mubest_out) mubest_out[0] = kb >= 0 ? mus[kb] : __builtin_nan("");
    }
}

struct GcvOut {
    const double* mus;
    int64_t mu_stride;  // 0: one grid for all items, K: one grid per item
    int K;
    double* G;
    int32_t* kbest;
    double* mubest;
};

// One block per item.  LDS sized to the item (dynamic): the staged elements of one chunk
// (min(per_item, GCV_CHUNK) pairs), the K sums and G values, so that short items at small K
// keep several blocks per CU; the staging chunk equals the static bound whenever an item
// needs more than one, so the summation order does not depend on the sizing.
inline size_t gcv_single_lds(int64_t per_item, int K, int* chunk_cap) {
    const int cap = static_cast<int>(per_item < GCV_CHUNK ? (per_item < 1 ? 1 : per_item) : GCV_CHUNK);
    *chunk_cap = cap;
    return sizeof(double2) * (static_cast<size_t>(cap) + K) + sizeof(double) * K;
}

__global__ __launch_bounds__(GCV_THREADS) void k_gcv_single(Spec sp, const void* __restrict__ coeff, GcvOut o,
                                                            int chunk_cap) {
    extern __shared__ double2 dyn[];
    __shared__ double2 red[2 * GCV_THREADS];
    __shared__ int kshared;
    double2* stage = dyn;
    double2* sums = dyn + chunk_cap;
    double* Gs = reinterpret_cast<double*>(sums + o.K);
    const int64_t b = blockIdx.x;
    const double* mus = o.mus + b * o.mu_stride;
    gcv_accumulate(sp, coeff, b, 0, sp.per_item, mus, o.K, sums, stage, red, chunk_cap);
    gcv_finish(sums, o.K, mus, o.G ? o.G + b * o.K : nullptr, o.kbest + b,
               o.mubest ? o.mubest + b : nullptr, Gs, &kshared);
}

// Partial sums over a span of a large item: staging chunks of GCV_PART_CHUNK pairs keep the
// block at 32 KiB of LDS, five blocks per CU (the register bound) instead of four.
constexpr int GCV_PART_CHUNK = 1536;

__global__ __launch_bounds__(GCV_THREADS) void k_gcv_partial(Spec sp, const void* __restrict__ coeff, GcvOut o,
                                                             int64_t span, double2* part) {
    __shared__ double2 stage[GCV_PART_CHUNK];
    __shared__ double2 red[2 * GCV_THREADS];
    const int64_t w = blockIdx.x, b = blockIdx.y;
    const int64_t e0 = w * span;
    int64_t e1 = e0 + span;
    if (e1 > sp.per_item) e1 = sp.per_item;
    const double* mus = o.mus + b * o.mu_stride;
    gcv_accumulate(sp, coeff, b, e0, e1, mus, o.K, part + (b * gridDim.x + w) * o.K, stage, red, GCV_PART_CHUNK);
}

// Sum of the partial (N, D) of every grid value over the parts: block (group of 8 grid
// values, item); 32 lanes per grid value each add the parts w = lane, lane + 32, ... in
// order, then a fixed butterfly over the 32 lanes; the total replaces part w = 0 (read by
// this block only).
constexpr int GCV_RK = GCV_THREADS / 32;

__global__ __launch_bounds__(GCV_THREADS) void k_gcv_reduce(int K, int64_t nparts, double2* part) {
    const int64_t b = blockIdx.y;
    const int g = threadIdx.x / 32, lane = threadIdx.x & 31;
    const int k = blockIdx.x * GCV_RK + g;
    const int kk = k < K ? k : K - 1;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t w = lane; w < nparts; w += 32) {
        const double2 v = part[(b * nparts + w) * K + kk];
        acc.x += v.x;
        acc.y += v.y;
    }
    for (int off = 16; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, 32);
        acc.y += __shfl_xor(acc.y, off, 32);
    }
    if (lane == 0 && k < K) part[(b * nparts) * K + k] = acc;
}

__global__ __launch_bounds__(GCV_THREADS) void k_gcv_finalize(GcvOut o, int64_t nparts, const double2* __restrict__ part) {
    __shared__ double2 sums[1024];
    __shared__ double Gs[1024];
    __shared__ int kshared;
    const int64_t b = blockIdx.x;
    for (int k = threadIdx.x; k < o.K; k += GCV_THREADS) sums[k] = part[(b * nparts) * o.K + k];
    __syncthreads();
    const double* mus = o.mus + b * o.mu_stride;
    gcv_finish(sums, o.K, mus, o.G ? o.G + b * o.K : nullptr, o.kbest + b,
               o.mubest ? o.mubest + b : nullptr, Gs, &kshared);
}

// ----------------------------------------------------------------------- exact GCV

// Eq. gcv for a 1D batch: G(mu) = ||T (sigma ghat)||^2 / (sum sigma)^2 (the residual norm
// of eq. gcnum without its approximation), ||T v||^2 from the structure of T (XgcvParams).
// One block per signal.  Per chunk of the core range j = 1..N the block stages t_j,
// w_j = |ghat_j|^2 and u_kj = vec[k][j-1] ghat_j; thread (part, kl) takes the grid values
// a = 2 (k0 + kl) and b = a + 1 and accumulates, with r = 1/(t + mu) (one reciprocal of
// (t + mu_a)(t + mu_b) per element for both), D += r, W += w r^2, P_k += u_k r over the
// staged elements part, part + nparts, ...; parts are added in order (bitwise
// reproducible).
constexpr int XG_THREADS = 256;
constexpr int XG_CHUNK = 256;
constexpr int XG_NV = 4;                 // fixed vectors: |C| + 2 ghost rows <= 4 for every kind
constexpr int XG_ACC = 2 + 2 * XG_NV;     // D, W, complex P_k

// ROWS: the "signals" are the rows of a chunk of images (block (row i, image b0 + y)); per
// row and grid value the kernel writes the row's functionals ell(v_i) = [P_c, v_c, y_0,
// y_{n-1}] (complex), ||T v_i||^2 and its part of the trace to rows_out[((y n0 + i) K + k)]
// (XG2_RW doubles) instead of G.
constexpr int XG2_RW = 2 * (2 * XG_MAXC + 2) + 2;

template <bool CPLX, bool ROWS>
__global__ __launch_bounds__(XG_THREADS) void k_gcv_exact(Spec sp, const void* __restrict__ coeff, GcvOut o,
                                                          XgcvParams xp, int n, int64_t b0, double* rows_out) {
    constexpr int UW = CPLX ? 2 : 1;  // doubles per staged u
    __shared__ double st_t[XG_CHUNK], st_w[XG_CHUNK];
    __shared__ double st_u[XG_NV * UW][XG_CHUNK];
    __shared__ double red[XG_THREADS][XG_ACC + 1];
    __shared__ double Gs[ROWS ? 1 : 1024];
    __shared__ int kshared;
    const int tid = threadIdx.x;
    const int64_t b = ROWS ? b0 + blockIdx.y : blockIdx.x;
    const int64_t off = ROWS ? static_cast<int64_t>(blockIdx.x) * n : 0;  // first element of the row
    const double* mus = o.mus + b * o.mu_stride;
    const int K = o.K, N = n - 2, nv = xp.nv;
    const int Kh = (K + 1) / 2;
    const int Kb = Kh < XG_THREADS ? Kh : XG_THREADS;
    const int nparts = XG_THREADS / Kb;
    const int part = tid / Kb, kl = tid - part * Kb;
    // t and ghat of element e (t = 1e150 where s = 0, as in the approximate scan)
    auto load = [&](int64_t e, double& t, double2& g) {
        double2 dd;
        double ss;
        spec_at(sp, b, off + e, dd, ss);
        g = cload(coeff, b * sp.per_item + off + e, sp.cplx);
        const double s2 = ss * ss;
        t = 1e150;
        if (s2 != 0.0) t = fma(dd.x, dd.x, dd.y * dd.y) / s2;
    };
    for (int k0 = 0; k0 < Kh; k0 += Kb) {
        const int kk = k0 + kl;
        const bool active = part < nparts && kk < Kh;
        const int ka = 2 * kk, kb2 = ka + 1 < K ? ka + 1 : ka;
        const double mua = active ? mus[ka] : 1.0, mub = active ? mus[kb2] : 1.0;
        double Da = 0.0, Wa = 0.0, Db = 0.0, Wb = 0.0;
        double2 Pa[XG_NV], Pb[XG_NV];
#pragma unroll
        for (int v = 0; v < XG_NV; ++v) Pa[v] = Pb[v] = make_double2(0.0, 0.0);
        for (int c0 = 0; c0 < N; c0 += XG_CHUNK) {
            const int len = N - c0 < XG_CHUNK ? N - c0 : XG_CHUNK;
            __syncthreads();
            for (int i = tid; i < len; i += XG_THREADS) {
                const int j = c0 + i;  // core index; coefficient j + 1
                double t;
                double2 g;
                load(j + 1, t, g);
                const bool zero = t == 1e150;
                st_t[i] = t;
                st_w[i] = zero ? 0.0 : fma(g.x, g.x, g.y * g.y);
                for (int v = 0; v < nv; ++v) {
                    const double2 u = zero ? make_double2(0.0, 0.0) : cmul(xp.vec[static_cast<int64_t>(v) * N + j], g);
                    st_u[v * UW][i] = u.x;
                    if (CPLX) st_u[v * UW + 1][i] = u.y;
                }
            }
            __syncthreads();
            if (active) {
                for (int i = part; i < len; i += nparts) {
                    const double t = st_t[i], w = st_w[i];
                    const double ua = t + mua, ub = t + mub;
                    const double R = rcp_nr(ua * ub);
                    const double ra = ub * R, rb = ua * R;
                    Da += ra;
                    Db += rb;
                    Wa = fma(w, ra * ra, Wa);
                    Wb = fma(w, rb * rb, Wb);
#pragma unroll
                    for (int v = 0; v < XG_NV; ++v) {
                        if (v < nv) {
                            const double ux = st_u[v * UW][i];
                            Pa[v].x = fma(ux, ra, Pa[v].x);
                            Pb[v].x = fma(ux, rb, Pb[v].x);
                            if (CPLX) {
                                const double uy = st_u[v * UW + UW - 1][i];
                                Pa[v].y = fma(uy, ra, Pa[v].y);
                                Pb[v].y = fma(uy, rb, Pb[v].y);
                            }
                        }
                    }
                }
            }
        }
        // two rounds through the reduction buffer: grid value a, then b
        for (int round = 0; round < 2; ++round) {
            __syncthreads();
            if (part < nparts) {
                double* rr = red[tid];
                rr[0] = round ? Db : Da;
                rr[1] = round ? Wb : Wa;
                for (int v = 0; v < XG_NV; ++v) {
                    const double2 P = round ? Pb[v] : Pa[v];
                    rr[2 + 2 * v] = P.x;
                    rr[3 + 2 * v] = P.y;
                }
            }
            __syncthreads();
            const int k = round ? ka + 1 : ka;
            if (part == 0 && kk < Kh && k < K) {
                const double mu = round ? mub : mua;
                double acc[XG_ACC];
                for (int a = 0; a < XG_ACC; ++a) acc[a] = red[kl][a];
                for (int p = 1; p < nparts; ++p)
                    for (int a = 0; a < XG_ACC; ++a) acc[a] += red[p * Kb + kl][a];
                // boundary and replaced coefficients: v_c = ghat_c r_c
                double2 vc[XG_MAXC];
                double Dt = acc[0];
                for (int c = 0; c < xp.nc; ++c) {
                    double t;
                    double2 g;
                    load(xp.cidx[c], t, g);
                    const double r = rcp_nr(t + mu);
                    vc[c] = t == 1e150 ? make_double2(0.0, 0.0) : make_double2(g.x * r, g.y * r);
                    if (c < 2) Dt += r;  // the two polynomial entries of the trace
                }
                double num = acc[1];
                for (int c = 0; c < xp.nc; ++c) {
                    const double2 Pc = make_double2(acc[2 + 2 * c], acc[3 + 2 * c]);
                    num += 2.0 * (Pc.x * vc[c].x + Pc.y * vc[c].y);   // 2 Re(conj(P_c) v_c)
                    for (int c2 = 0; c2 < xp.nc; ++c2)
                        num += xp.gam[c][c2] * (vc[c].x * vc[c2].x + vc[c].y * vc[c2].y);
                }
                // boundary rows: y_0 = t00 v_0 + t0n v_{n-1} (+ a . v_mid), y_{n-1} likewise
                double2 y0 = make_double2(xp.t00 * vc[0].x + xp.t0n * vc[1].x, xp.t00 * vc[0].y + xp.t0n * vc[1].y);
                double2 yn = make_double2(xp.tn0 * vc[0].x + xp.tnn * vc[1].x, xp.tn0 * vc[0].y + xp.tnn * vc[1].y);
                if (xp.rows) {
                    y0.x += acc[2 + 2 * xp.nc];
                    y0.y += acc[3 + 2 * xp.nc];
                    yn.x += acc[4 + 2 * xp.nc];
                    yn.y += acc[5 + 2 * xp.nc];
                }
                num += y0.x * y0.x + y0.y * y0.y + yn.x * yn.x + yn.y * yn.y;
                if (ROWS) {
                    double* out = rows_out + ((static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * K + k) * XG2_RW;
                    const int nc = xp.nc;
                    for (int c = 0; c < nc; ++c) {
                        out[2 * c] = acc[2 + 2 * c];
                        out[2 * c + 1] = acc[3 + 2 * c];
                        out[2 * (nc + c)] = vc[c].x;
                        out[2 * (nc + c) + 1] = vc[c].y;
                    }
                    out[4 * nc] = y0.x;
                    out[4 * nc + 1] = y0.y;
                    out[4 * nc + 2] = yn.x;
                    out[4 * nc + 3] = yn.y;
                    out[XG2_RW - 2] = num;
                    out[XG2_RW - 1] = Dt;
                } else {
                    const double g = num / (Dt * Dt);
                    Gs[k] = g;
                    if (o.G) o.G[b * K + k] = g;
                }
            }
        }
    }
    if (ROWS) return;
    __syncthreads();
    gcv_argmin(Gs, K, &kshared);
    if (tid == 0) {
        const int kb = kshared;
        o.kbest[b] = kb;
        if (o.mubest) o.mubest[b] = kb >= 0 ? mus[kb] : __builtin_nan("");
    }
}

// The column pass of the 2D exact GCV.  With V = sigma ghat and the axis-0 functionals
// lambda_p = [P_c, e_c, y_0, y_{n0-1}], u_p = sum_i lambda_p[i] v_i (a vector over the
// columns); for every interior column j this thread accumulates u_{P_c}[j], u_y[j] and
// the entries v_{c, j} of the boundary / replaced rows for four grid values at a time, then
// the products the axis-0 low-rank form needs, S = [conj(u_{P_c}) v_c (c < nc),
// conj(v_c) v_c' (c, c' < nc), |u_{y0}|^2, |u_{yn}|^2], added over the 64 columns of the
// wave by a fixed butterfly; part[((y nblk + block) K + k) XG2_NE + e].  Block (column
// tile, image, group of XG2_MU grid values).
constexpr int XG2_NE = XG_MAXC + XG_MAXC * XG_MAXC + 2;
constexpr int XG2_MU = 8;   // grid values per block, in pairs sharing one reciprocal

// acc += w v (complex, or the real parts only for the real kinds)
template <bool CPLX>
__device__ __forceinline__ void xg_fma(double2& acc, double2 w, double2 v) {
    if (CPLX) {
        acc.x = fma(w.x, v.x, fma(-w.y, v.y, acc.x));
        acc.y = fma(w.x, v.y, fma(w.y, v.x, acc.y));
    } else {
        acc.x = fma(w.x, v.x, acc.x);
    }
}

template <bool CPLX>
__global__ __launch_bounds__(64) void k_xg2_cols(Spec sp, const void* __restrict__ coeff, const double* __restrict__ mus,
                                                 int64_t mu_stride, int K, XgcvParams x0, int n0, int n1, int64_t b0,
                                                 double2* part) {
    const int lane = threadIdx.x;
    const int64_t b = b0 + blockIdx.y;
    const int jc = blockIdx.x * 64 + lane;           // core column, coefficient jc + 1
    const bool active = jc < n1 - 2;
    const int j = active ? jc + 1 : 1;
    const int nc = x0.nc, N0 = n0 - 2;
    const double* mb = mus + b * mu_stride;
    {
        const int k0 = blockIdx.z * XG2_MU;
        double mu[XG2_MU];
#pragma unroll
        for (int m = 0; m < XG2_MU; ++m) mu[m] = mb[k0 + m < K ? k0 + m : K - 1];
        double2 uP[XG_MAXC][XG2_MU], uE[XG_MAXC][XG2_MU], uY[2][XG2_MU];
#pragma unroll
        for (int m = 0; m < XG2_MU; ++m) {
#pragma unroll
            for (int c = 0; c < XG_MAXC; ++c) uP[c][m] = uE[c][m] = make_double2(0.0, 0.0);
            uY[0][m] = uY[1][m] = make_double2(0.0, 0.0);
        }
        for (int i = 0; i < n0; ++i) {
            const int64_t e = static_cast<int64_t>(i) * n1 + j;
            double2 dd;
            double ss;
            spec_at(sp, b, e, dd, ss);
            const double2 g = cload(coeff, b * sp.per_item + e, sp.cplx);
            const double s2 = ss * ss;
            const bool zero = s2 == 0.0;
            const double t = zero ? 1.0 : fma(dd.x, dd.x, dd.y * dd.y) / s2;
            const bool mid = i >= 1 && i <= N0;
            // weights of row i in the axis-0 functionals
            double2 wP[XG_MAXC];
#pragma unroll
            for (int c = 0; c < XG_MAXC; ++c)
                wP[c] = (mid && c < nc) ? x0.vec[static_cast<int64_t>(c) * N0 + i - 1] : make_double2(0.0, 0.0);
            double2 wy0 = make_double2(i == 0 ? x0.t00 : (i == n0 - 1 ? x0.t0n : 0.0), 0.0);
            double2 wyn = make_double2(i == 0 ? x0.tn0 : (i == n0 - 1 ? x0.tnn : 0.0), 0.0);
            if (mid && x0.rows) {
                wy0 = x0.vec[static_cast<int64_t>(nc) * N0 + i - 1];
                wyn = x0.vec[static_cast<int64_t>(nc + 1) * N0 + i - 1];
            }
            int ce = -1;  // the boundary / replaced row this is, if any
#pragma unroll
            for (int c = 0; c < XG_MAXC; ++c)
                if (c < nc && i == x0.cidx[c]) ce = c;
#pragma unroll
            for (int m = 0; m < XG2_MU; m += 2) {
                const double ua = t + mu[m], ub = t + mu[m + 1];
                const double R = zero ? 0.0 : rcp_nr(ua * ub);
                const double rr[2] = {ub * R, ua * R};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double2 v = make_double2(g.x * rr[h], g.y * rr[h]);
#pragma unroll
                    for (int c = 0; c < XG_MAXC; ++c) xg_fma<CPLX>(uP[c][m + h], wP[c], v);
                    xg_fma<CPLX>(uY[0][m + h], wy0, v);
                    xg_fma<CPLX>(uY[1][m + h], wyn, v);
#pragma unroll
                    for (int c = 0; c < XG_MAXC; ++c)
                        if (c == ce) uE[c][m + h] = v;
                }
            }
        }
        for (int m = 0; m < XG2_MU && k0 + m < K; ++m) {
            double2 S[XG2_NE];
#pragma unroll
            for (int q = 0; q < XG2_NE; ++q) S[q] = make_double2(0.0, 0.0);
            if (active) {
                for (int c = 0; c < nc; ++c) {
                    S[c] = cmulc(uE[c][m], uP[c][m]);  // conj(u_P) v_c
                    for (int c2 = 0; c2 < nc; ++c2) S[XG_MAXC + c * XG_MAXC + c2] = cmulc(uE[c2][m], uE[c][m]);
                }
                S[XG2_NE - 2] = make_double2(uY[0][m].x * uY[0][m].x + uY[0][m].y * uY[0][m].y, 0.0);
                S[XG2_NE - 1] = make_double2(uY[1][m].x * uY[1][m].x + uY[1][m].y * uY[1][m].y, 0.0);
            }
#pragma unroll
            for (int q = 0; q < XG2_NE; ++q) {
                double2 v = S[q];
                for (int w = 32; w > 0; w >>= 1) {
                    v.x += __shfl_xor(v.x, w, 64);
                    v.y += __shfl_xor(v.y, w, 64);
                }
                S[q] = v;
            }
            if (lane == 0) {
                double2* dst = part + ((static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * K + k0 + m) * XG2_NE;
#pragma unroll
                for (int q = 0; q < XG2_NE; ++q) dst[q] = S[q];
            }
        }
    }
}

// B1(x, z) = ell(x)^H M1 ell(z) of axis 1 for functional vectors laid out [P_c, v_c, y0, yn].
__device__ __forceinline__ double2 xg_bilinear(const XgcvParams& x1, const double2* x, const double2* z) {
    const int nc = x1.nc;
    double2 acc = make_double2(0.0, 0.0);
    for (int c = 0; c < nc; ++c) {
        acc = cadd(acc, cmulc(z[nc + c], x[c]));      // conj(x_P) z_e
        acc = cadd(acc, cmulc(z[c], x[nc + c]));      // conj(x_e) z_P
        for (int c2 = 0; c2 < nc; ++c2) {
            const double2 p = cmulc(z[nc + c2], x[nc + c]);
            acc.x += x1.gam[c][c2] * p.x;
            acc.y += x1.gam[c][c2] * p.y;
        }
    }
    acc = cadd(acc, cmulc(z[2 * nc], x[2 * nc]));
    acc = cadd(acc, cmulc(z[2 * nc + 1], x[2 * nc + 1]));
    return acc;
}

// G(mu_k) of one image: the interior rows' ||T1 v_i||^2 plus the axis-0 low-rank form
// sum_{p,q} M0[p,q] (S_pq + B1(ell1(u_p), ell1(u_q))) over (sum sigma)^2, with
// ell1(u_p) = sum_i lambda_p[i] ell1(v_i) from the row pass.  Block (k, image): lane t
// owns the weighted row sum (p, q) = (t / k1, t % k1); sums in a fixed order.
__global__ __launch_bounds__(64) void k_xg2_combine(const double* __restrict__ rows_in, const double2* __restrict__ part,
                                                    int nblk, int K, XgcvParams x0, XgcvParams x1, int n0, int64_t b0,
                                                    double* G) {
    __shared__ double2 rt[2 * XG_MAXC + 2][2 * XG_MAXC + 2];   // ell1(u_p), p over [P_c, e_c, y0, yn]
    __shared__ double2 Ssum[XG2_NE];
    __shared__ double sums[2][64];
    const int lane = threadIdx.x, k = blockIdx.x;
    const int64_t y = blockIdx.y;
    const int nc0 = x0.nc, k1 = 2 * x1.nc + 2, N0 = n0 - 2;
    const double* rows = rows_in + y * static_cast<int64_t>(n0) * K * XG2_RW;
    auto row = [&](int i) { return rows + (static_cast<int64_t>(i) * K + k) * XG2_RW; };
    // interior rows' norms and the whole trace
    double rs = 0.0, ds = 0.0;
    for (int i = lane; i < n0; i += 64) {
        const double* r = row(i);
        if (i >= 1 && i <= N0) rs += r[XG2_RW - 2];
        ds += r[XG2_RW - 1];
    }
    sums[0][lane] = rs;
    sums[1][lane] = ds;
    // weighted row sums of the functionals: P_c (c < nc0), then y0, yn
    const int nw = nc0 + 2;
    if (lane < nw * k1) {
        const int p = lane / k1, q = lane - p * k1;
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < n0; ++i) {
            const bool mid = i >= 1 && i <= N0;
            double2 w = make_double2(0.0, 0.0);
            if (p < nc0) {
                if (mid) w = x0.vec[static_cast<int64_t>(p) * N0 + i - 1];
            } else {
                const int yy = p - nc0;  // 0: y0, 1: yn
                if (i == 0) w.x = yy ? x0.tn0 : x0.t00;
                else if (i == n0 - 1) w.x = yy ? x0.tnn : x0.t0n;
                else if (x0.rows) w = x0.vec[static_cast<int64_t>(nc0 + yy) * N0 + i - 1];
            }
            const double* r = row(i);
            acc = cadd(acc, cmul(w, make_double2(r[2 * q], r[2 * q + 1])));
        }
        const int slot = p < nc0 ? p : 2 * nc0 + (p - nc0);
        rt[slot][q] = acc;
    }
    // ell1 of the e_c functionals: the rows themselves
    if (lane < nc0 * k1) {
        const int c = lane / k1, q = lane - c * k1;
        const double* r = row(x0.cidx[c]);
        rt[nc0 + c][q] = make_double2(r[2 * q], r[2 * q + 1]);
    }
    // S over the column blocks, in order
    if (lane < XG2_NE) {
        double2 acc = make_double2(0.0, 0.0);
        for (int w = 0; w < nblk; ++w) acc = cadd(acc, part[((y * nblk + w) * K + k) * XG2_NE + lane]);
        Ssum[lane] = acc;
    }
    __syncthreads();
    if (lane == 0) {
        double rsum = 0.0, dsum = 0.0;
        for (int t = 0; t < 64; ++t) {
            rsum += sums[0][t];
            dsum += sums[1][t];
        }
        double num = rsum;
        for (int c = 0; c < nc0; ++c) {
            const double2 a = cadd(Ssum[c], xg_bilinear(x1, rt[c], rt[nc0 + c]));
            num += 2.0 * a.x;
            for (int c2 = 0; c2 < nc0; ++c2) {
                const double2 e = cadd(Ssum[XG_MAXC + c * XG_MAXC + c2], xg_bilinear(x1, rt[nc0 + c], rt[nc0 + c2]));
                num += x0.gam[c][c2] * e.x;
            }
        }
        num += Ssum[XG2_NE - 2].x + xg_bilinear(x1, rt[2 * nc0], rt[2 * nc0]).x;
        num += Ssum[XG2_NE - 1].x + xg_bilinear(x1, rt[2 * nc0 + 1], rt[2 * nc0 + 1]).x;
        G[(b0 + y) * K + k] = num / (dsum * dsum);
    }
}

// ------------------------------------------------------------------- exact GCV, 2D

__global__ __launch_bounds__(64) void k_xg2_argmin(const double* __restrict__ G, GcvOut o) {
    const int64_t b = blockIdx.x;
    __shared__ int kshared;
    gcv_argmin(G + b * o.K, o.K, &kshared);
    if (threadIdx.x == 0) {
        const int kb = kshared;
        o.kbest[b] = kb;
        if (o.mubest) o.mubest[b] = kb >= 0 ? o.mus[b * o.mu_stride + kb] : __builtin_nan("");
    }
}

static Spec make_spec(const ht_plan* plan, const void* d, const double* s, int64_t eig_batch, int layout) {
    Spec sp;
    sp.d = d;
    sp.s = s;
    sp.factored = plan->ndim == 2 && layout == HT_SPECTRUM_FACTORS;
    sp.n0 = plan->ax[0].n;
    sp.n1 = plan->ndim == 2 ? plan->ax[1].n : 1;
    sp.per_item = plan->ndim == 2 ? static_cast<int64_t>(sp.n0) * sp.n1 : sp.n0;
    sp.eig_stride = (!sp.factored && eig_batch > 1) ? sp.per_item : 0;
    sp.cplx = plan->cplx;
    return sp;
}

// shared argument checks of the filter and the GCV scan
static ht_status check_spectrum(const ht_plan* plan, int64_t eig_batch, int layout, int64_t batch, const char* who) {
    if (!(eig_batch == 1 || eig_batch == batch))
        return fail(HT_ERR_INVALID_ARG, std::string(who) + ": eig_batch must be 1 or batch");
    if (plan->ndim == 2) {
        if (layout != HT_SPECTRUM_FACTORS && layout != HT_SPECTRUM_FULL)
            return fail(HT_ERR_INVALID_ARG, std::string(who) + ": bad spectrum layout");
        if (layout == HT_SPECTRUM_FACTORS && eig_batch != 1)
            return fail(HT_ERR_INVALID_ARG, std::string(who) + ": separable 2D factors are shared (eig_batch = 1)");
    }
    return HT_OK;
}

}  // namespace ht

using namespace ht;

extern "C" ht_status ht_eigs(const ht_plan* plan, const double* psf, const int64_t* psf_len,
                             const int64_t* psf_center, int norm, void* d, double* s,
                             int64_t batch, hipStream_t stream) {
    if (!plan || !psf_len || !psf_center) return fail(HT_ERR_INVALID_ARG, "ht_eigs: null argument");
    if (batch != 0 && (!psf || !d || !s)) return fail(HT_ERR_INVALID_ARG, "ht_eigs: null argument");
    if (norm != HT_NORM_IDENTITY && norm != HT_NORM_SECOND_DIFF)
        return fail(HT_ERR_INVALID_ARG, "ht_eigs: bad norm");
    if (batch < 0 || batch > 65535) return fail(HT_ERR_INVALID_ARG, "ht_eigs: batch out of range [0, 65535]");
    if (plan->ndim == 2 && batch != 1) return fail(HT_ERR_INVALID_ARG, "ht_eigs: 2D plans take one separable PSF (batch = 1)");
    if (batch == 0) return HT_OK;
    for (int a = 0; a < plan->ndim; ++a) {
        const int64_t len = psf_len[a], c = psf_center[a];
        if (len < 1 || c < 0 || c >= len) return fail(HT_ERR_INVALID_ARG, "ht_eigs: bad PSF length or center");
        const int64_t m = c > len - 1 - c ? c : len - 1 - c;
        if (2 * m + 1 > plan->ax[a].N) return fail(HT_ERR_PSF_TOO_WIDE, "ht_eigs: PSF half-width m needs 2m+1 <= n-2 (n for P, R)");
    }
    int64_t off_d = 0, off_psf = 0;
    for (int a = 0; a < plan->ndim; ++a) {
        const Axis& ax = plan->ax[a];
        const double s_ident = (plan->ndim == 2 && a == 1) ? 0.0 : 1.0;
        const int cp = plan->cplx;
        // 2D with one complex axis stores both factors as complex
        const int cp_out = plan->cplx;
        void* dd = cp_out ? static_cast<void*>(static_cast<double2*>(d) + off_d)
                          : static_cast<void*>(static_cast<double*>(d) + off_d);
        (void)cp;
        dim3 grid((ax.n + 255) / 256, static_cast<unsigned>(batch));
        hipLaunchKernelGGL(k_eigs, grid, dim3(256), 0, stream, ax, psf + off_psf, psf_len[a], psf_center[a],
                           psf_len[a], norm, s_ident, dd, s + off_d, static_cast<int64_t>(ax.n), cp_out);
        ht_status st = check_hip(hipGetLastError(), "ht_eigs launch");
        if (st != HT_OK) return st;
        off_d += ax.n;
        off_psf += psf_len[a];
    }
    return HT_OK;
}

extern "C" ht_status ht_eigs2d(const ht_plan* plan, const double* psf, int64_t len0, int64_t len1,
                               int64_t c0, int64_t c1, int norm, void* d, double* s, int64_t batch,
                               hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_eigs2d: null plan");
    if (plan->ndim != 2) return fail(HT_ERR_INVALID_ARG, "ht_eigs2d: needs a 2D plan");
    if (plan->ax[0].kind == HT_KIND_F3 || plan->ax[1].kind == HT_KIND_F3)
        return fail(HT_ERR_UNSUPPORTED, "ht_eigs2d: not defined for the degree-3 Fourier kind (use separable factors)");
    if (norm != HT_NORM_IDENTITY && norm != HT_NORM_SECOND_DIFF) return fail(HT_ERR_INVALID_ARG, "ht_eigs2d: bad norm");
    if (batch < 0 || batch > plan->max_batch) return fail(HT_ERR_INVALID_ARG, "ht_eigs2d: batch must be in [0, max_batch]");
    if (batch == 0) return HT_OK;
    if (!psf || !d || !s) return fail(HT_ERR_INVALID_ARG, "ht_eigs2d: null argument");
    const int64_t lens[2] = {len0, len1}, cens[2] = {c0, c1};
    for (int a = 0; a < 2; ++a) {
        if (lens[a] < 1 || cens[a] < 0 || cens[a] >= lens[a]) return fail(HT_ERR_INVALID_ARG, "ht_eigs2d: bad mask shape or center");
        const int64_t m = cens[a] > lens[a] - 1 - cens[a] ? cens[a] : lens[a] - 1 - cens[a];
        if (2 * m + 1 > plan->ax[a].N) return fail(HT_ERR_PSF_TOO_WIDE, "ht_eigs2d: PSF half-width m needs 2m+1 <= n-2 (n for P, R) per axis");
    }
    const Axis& ax0 = plan->ax[0];
    const Axis& ax1 = plan->ax[1];
    // W [batch][len0][n1] fits the [max_batch][n0][n1] workspace: len0 <= n0 - 2
    double2* W = plan->work;
    hipLaunchKernelGGL(plan->cplx ? k_eigs2d_rows<true> : k_eigs2d_rows<false>,
                       dim3((ax1.n + 255) / 256, static_cast<unsigned>(len0), static_cast<unsigned>(batch)), dim3(256), 0,
                       stream, ax1, psf, len0, len1, c1, W);
    ht_status st = check_hip(hipGetLastError(), "ht_eigs2d rows launch");
    if (st != HT_OK) return st;
    hipLaunchKernelGGL(plan->cplx ? k_eigs2d_cols<true> : k_eigs2d_cols<false>,
                       dim3((ax1.n + E2_TJ - 1) / E2_TJ, (ax0.n + E2_TI - 1) / E2_TI, static_cast<unsigned>(batch)),
                       dim3(256), 0, stream, ax0, ax1, static_cast<const double2*>(W), len0, c0, norm, d, s);
    return check_hip(hipGetLastError(), "ht_eigs2d launch");
}

extern "C" ht_status ht_tikhonov_filter(const ht_plan* plan, const void* coeff, const void* d,
                                        const double* s, int64_t eig_batch, int layout, const double* mu,
                                        void* fhat, int64_t batch, hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_tikhonov_filter: null plan");
    if (batch < 0) return fail(HT_ERR_INVALID_ARG, "ht_tikhonov_filter: negative batch");
    if (batch == 0) return HT_OK;
    if (!coeff || !d || !s || !mu || !fhat) return fail(HT_ERR_INVALID_ARG, "ht_tikhonov_filter: null argument");
    ht_status st = check_spectrum(plan, eig_batch, layout, batch, "ht_tikhonov_filter");
    if (st != HT_OK) return st;
    const Spec sp = make_spec(plan, d, s, eig_batch, layout);
    const int64_t total = batch * sp.per_item;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffffLL) return fail(HT_ERR_INVALID_ARG, "ht_tikhonov_filter: batch too large");
    hipLaunchKernelGGL(k_filter, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, sp, coeff, mu, fhat,
                       sp.per_item, total);
    return check_hip(hipGetLastError(), "ht_tikhonov_filter launch");
}

extern "C" ht_status ht_gcv_scan(const ht_plan* plan, const void* coeff, const void* d, const double* s,
                                 int64_t eig_batch, int layout, const double* mu_grid, int32_t K, int grid_per_item,
                                 double* G, int32_t* k_best, double* mu_best, int64_t batch,
                                 hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan: null plan");
    if (K < 1 || K > 1024) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan: K must be in [1, 1024]");
    if (batch < 0 || batch > 0x7fffffffLL) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan: batch out of range");
    if (batch == 0) return HT_OK;
    if (!coeff || !d || !s || !mu_grid || !k_best) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan: null argument");
    ht_status st0 = check_spectrum(plan, eig_batch, layout, batch, "ht_gcv_scan");
    if (st0 != HT_OK) return st0;
    const Spec sp = make_spec(plan, d, s, eig_batch, layout);
    GcvOut o{mu_grid, grid_per_item ? static_cast<int64_t>(K) : 0, K, G, k_best, mu_best};
    if (plan->ndim == 1) {
        int cap = 0;
        const size_t lds = gcv_single_lds(sp.per_item, K, &cap);
        hipLaunchKernelGGL(k_gcv_single, dim3(static_cast<unsigned>(batch)), dim3(GCV_THREADS), lds, stream, sp, coeff,
                           o, cap);
        return check_hip(hipGetLastError(), "ht_gcv_scan launch");
    }
    if (batch > plan->max_batch) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan: batch exceeds the plan's max_batch");
    int64_t nw = (sp.per_item + GCV_CHUNK - 1) / GCV_CHUNK;
    if (nw > 512) nw = 512;
    const int64_t span = (sp.per_item + nw - 1) / nw;
    nw = (sp.per_item + span - 1) / span;
    if (nw * K * batch * 2 > plan->gcv_part_elems) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan: workspace too small");
    double2* part = reinterpret_cast<double2*>(plan->gcv_part);
    hipLaunchKernelGGL(k_gcv_partial, dim3(static_cast<unsigned>(nw), static_cast<unsigned>(batch)), dim3(GCV_THREADS), 0,
                       stream, sp, coeff, o, span, part);
    ht_status st = check_hip(hipGetLastError(), "ht_gcv_scan partial launch");
    if (st != HT_OK) return st;
    hipLaunchKernelGGL(k_gcv_reduce, dim3(static_cast<unsigned>((K + GCV_RK - 1) / GCV_RK), static_cast<unsigned>(batch)),
                       dim3(GCV_THREADS), 0, stream, static_cast<int>(K), nw, part);
    st = check_hip(hipGetLastError(), "ht_gcv_scan reduce launch");
    if (st != HT_OK) return st;
    hipLaunchKernelGGL(k_gcv_finalize, dim3(static_cast<unsigned>(batch)), dim3(GCV_THREADS), 0, stream, o, nw, part);
    return check_hip(hipGetLastError(), "ht_gcv_scan finalize launch");
}

// Eq. gcv for images, ||T0 V T1^T||^2 with V = sigma ghat, from the structure of both axes:
// ||T0 W||^2 over the columns of W = V T1^T is the interior rows' ||T1 v_i||^2 plus the
// axis-0 low-rank form of the functionals of W's columns, which are T1 applied to the
// weighted row sums u_p = sum_i lambda_p[i] v_i; so ||.||^2 = sum_{i interior} ||T1 v_i||^2
// + sum_{p,q} M0[p,q] (<u_p, u_q>_interior + ell1(u_p)^H M1 ell1(u_q)).  Row pass (the 1D
// kernel on every row, emitting its functionals), column pass (u_p over the interior
// columns and their products), combination per grid value.  Images in chunks that fit the
// workspace: row-pass outputs n0 K XG2_RW doubles and column-pass partials
// nblk K XG2_NE double2 per image, and K doubles per image for G when the caller passes
// none.
struct Xg2Work {
    double* rows;
    int64_t rows_elems;
    double2* part;
    int64_t part_elems;
    double* G;            // used when the caller's G is null
    int64_t g_elems;
};

static int64_t xg2_rows_per_img(const ht_plan* p, int K) { return static_cast<int64_t>(p->ax[0].n) * K * XG2_RW; }
static int64_t xg2_part_per_img(const ht_plan* p, int K) {
    return static_cast<int64_t>((p->ax[1].n - 2 + 63) / 64) * K * XG2_NE;
}

namespace ht {
// Reserve the plan's 2D exact GCV workspace for grids of up to max_k values: row-pass
// outputs for a chunk of images (at most 256 MiB, at least one image: fewer, larger chunks
// keep the column pass's grid wide), partials for the same chunk, G for max_batch images.
ht_status reserve_exact_gcv_2d(ht_plan* p, int max_k) {
    const int64_t cap = int64_t{1} << 25;  // doubles: 256 MiB
    const int64_t ri = xg2_rows_per_img(p, max_k);
    int64_t chunk = cap / ri;
    chunk = chunk < 1 ? 1 : (chunk > p->max_batch ? p->max_batch : chunk);
    const int64_t rows = chunk * ri, part = chunk * xg2_part_per_img(p, max_k), g = int64_t{max_k} * p->max_batch;
    void* mem = nullptr;
    if (hipMalloc(&mem, sizeof(double) * (rows + g) + sizeof(double2) * part) != hipSuccess) {
        (void)hipGetLastError();
        return fail(HT_ERR_OOM, "exact GCV workspace allocation failed");
    }
    if (p->xg2_mem) (void)hipFree(p->xg2_mem);
    p->xg2_mem = mem;
    p->xg2_max_k = max_k;
    p->xg2_rows_elems = rows;
    p->xg2_part_elems = part;
    p->xg2_g_elems = g;
    return HT_OK;
}
}  // namespace ht

static ht_status gcv_exact_2d(const ht_plan* plan, const void* coeff, const Spec& sp, GcvOut o, int64_t batch,
                              const Xg2Work& ws, hipStream_t stream) {
    const int n0 = plan->ax[0].n, n1 = plan->ax[1].n, K = o.K;
    const int64_t ri = xg2_rows_per_img(plan, K), pi = xg2_part_per_img(plan, K);
    int64_t chunk = ws.rows_elems / ri;
    if (pi * chunk > ws.part_elems) chunk = ws.part_elems / pi;
    chunk = chunk > batch ? batch : chunk;
    if (chunk < 1) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: one image at this K exceeds the workspace");
    double* Gb = o.G;
    if (!Gb) {
        if (int64_t{K} * batch > ws.g_elems)
            return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: the G values exceed the workspace (pass G)");
        Gb = ws.G;
    }
    const int nblk = (n1 - 2 + 63) / 64;
    const bool cp = plan->cplx != 0;
    ht_status st = HT_OK;
    for (int64_t b0 = 0; st == HT_OK && b0 < batch; b0 += chunk) {
        const unsigned nb = static_cast<unsigned>(batch - b0 < chunk ? batch - b0 : chunk);
        hipLaunchKernelGGL((cp ? k_gcv_exact<true, true> : k_gcv_exact<false, true>), dim3(n0, nb), dim3(XG_THREADS), 0,
                           stream, sp, coeff, o, plan->xg[1], n1, b0, ws.rows);
        st = check_hip(hipGetLastError(), "ht_gcv_scan_exact row launch");
        if (st != HT_OK) break;
        hipLaunchKernelGGL(cp ? k_xg2_cols<true> : k_xg2_cols<false>, dim3(nblk, nb, (K + XG2_MU - 1) / XG2_MU), dim3(64),
                           0, stream, sp, coeff,
                           o.mus, o.mu_stride, K, plan->xg[0], n0, n1, b0, ws.part);
        st = check_hip(hipGetLastError(), "ht_gcv_scan_exact column launch");
        if (st != HT_OK) break;
        hipLaunchKernelGGL(k_xg2_combine, dim3(K, nb), dim3(64), 0, stream, static_cast<const double*>(ws.rows),
                           static_cast<const double2*>(ws.part), nblk, K, plan->xg[0], plan->xg[1], n0, b0, Gb);
        st = check_hip(hipGetLastError(), "ht_gcv_scan_exact combine launch");
    }
    if (st == HT_OK) {
        hipLaunchKernelGGL(k_xg2_argmin, dim3(static_cast<unsigned>(batch)), dim3(64), 0, stream,
                           static_cast<const double*>(Gb), o);
        st = check_hip(hipGetLastError(), "ht_gcv_scan_exact argmin launch");
    }
    return st;
}

extern "C" ht_status ht_plan_reserve_exact_gcv(ht_plan* plan, int32_t max_k) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_plan_reserve_exact_gcv: null plan");
    if (max_k < 1 || max_k > 1024) return fail(HT_ERR_INVALID_ARG, "ht_plan_reserve_exact_gcv: max_k must be in [1, 1024]");
    if (plan->ndim != 2 || !plan->xg_mem[0] || max_k <= plan->xg2_max_k) return HT_OK;
    ht_status st = check_hip(hipSetDevice(plan->device), "ht_plan_reserve_exact_gcv: hipSetDevice");
    if (st != HT_OK) return st;
    st = check_hip(hipDeviceSynchronize(), "ht_plan_reserve_exact_gcv: synchronize");
    return st != HT_OK ? st : reserve_exact_gcv_2d(plan, max_k);
}

// ---- the allocation-free variant (ht_gcv_scan_exact_static): the workspace is one
// file-scope device array of fixed size.  Host code never passes the array's name to a
// kernel (in host code it is a stand-in, not a device address): its device address is
// taken once per device with hipGetSymbolAddress, with that device current, and kept.
constexpr int64_t STATIC_SCRATCH_DOUBLES = int64_t{1} << 23;  // 64 MiB per device
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[MAX_DEVICES] = {};

namespace ht {
// Device address of the static scratch on `device` (which must be current).
ht_status static_scratch_init(int device, double** out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(HT_ERR_INVALID_ARG, "static scratch: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return check_hip(e, "static scratch: hipGetSymbolAddress");
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    if (out) *out = g_scratch_ptr[device];
    return HT_OK;
}
}  // namespace ht

static Xg2Work plan_xg2_work(const ht_plan* p) {
    double* base = static_cast<double*>(p->xg2_mem);
    return Xg2Work{base, p->xg2_rows_elems, reinterpret_cast<double2*>(base + p->xg2_rows_elems + p->xg2_g_elems),
                   p->xg2_part_elems, base + p->xg2_rows_elems, p->xg2_g_elems};
}

extern "C" ht_status ht_gcv_scan_exact_static(const ht_plan* plan, const void* coeff, const void* d,
                                              const double* s, int64_t eig_batch, int layout, const double* mu_grid,
                                              int32_t K, int grid_per_item, double* G, int32_t* k_best,
                                              double* mu_best, int64_t batch, hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: null plan");
    if (plan->ndim != 2 || !plan->xg_mem[0])  // 1D plans and the comparators use no workspace
        return ht_gcv_scan_exact(plan, coeff, d, s, eig_batch, layout, mu_grid, K, grid_per_item, G, k_best, mu_best,
                                 batch, stream);
    if (K < 1 || K > 1024) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: K must be in [1, 1024]");
    if (batch < 0 || batch > plan->max_batch)
        return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: batch exceeds the plan's max_batch");
    if (batch == 0) return HT_OK;
    if (!coeff || !d || !s || !mu_grid || !k_best)
        return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: null argument");
    ht_status st = check_spectrum(plan, eig_batch, layout, batch, "ht_gcv_scan_exact_static");
    if (st != HT_OK) return st;
    int dev = -1;
    if ((st = check_hip(hipGetDevice(&dev), "ht_gcv_scan_exact_static: hipGetDevice")) != HT_OK) return st;
    if (dev != plan->device)
        return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: the plan's device is not the current device");
    double* base = nullptr;
    if ((st = static_scratch_init(dev, &base)) != HT_OK) return st;
    // partition for this call: G values (when the caller passes none), then row-pass
    // outputs and column-pass partials for as many images per chunk as fit
    const int64_t ri = xg2_rows_per_img(plan, K), pi = xg2_part_per_img(plan, K);
    const int64_t g_need = G ? 0 : int64_t{K} * batch;
    const int64_t chunk = (STATIC_SCRATCH_DOUBLES - g_need) / (ri + 2 * pi);
    if (chunk < 1)
        return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: one image at this K exceeds the 64 MiB static "
                                        "workspace");
    const int64_t c = chunk > batch ? batch : chunk;
    // 256-byte aligned pieces (the array is 256-byte aligned, ri and 2 pi are whole doubles)
    auto up = [](int64_t e) { return (e + 31) & ~int64_t{31}; };
    if (up(g_need) + up(c * ri) + 2 * c * pi > STATIC_SCRATCH_DOUBLES)
        return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact_static: workspace partition does not fit");
    const Xg2Work ws{base + up(g_need), c * ri, reinterpret_cast<double2*>(base + up(g_need) + up(c * ri)), c * pi,
                     base, g_need};
    const Spec sp = make_spec(plan, d, s, eig_batch, layout);
    GcvOut o{mu_grid, grid_per_item ? static_cast<int64_t>(K) : 0, K, G, k_best, mu_best};
    return gcv_exact_2d(plan, coeff, sp, o, batch, ws, stream);
}

extern "C" ht_status ht_gcv_scan_exact(const ht_plan* plan, const void* coeff, const void* d, const double* s,
                                       int64_t eig_batch, int layout, const double* mu_grid, int32_t K,
                                       int grid_per_item, double* G, int32_t* k_best, double* mu_best, int64_t batch,
                                       hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: null plan");
    for (int a = 0; a < plan->ndim; ++a)
        if (plan->ax[a].kind == HT_KIND_F3)
            return fail(HT_ERR_UNSUPPORTED, "ht_gcv_scan_exact: not for the degree-3 Fourier kind");
    if (plan->ndim == 2 && !plan->xg_mem[0])  // periodic / reflective: eq. gcv2 is eq. gcv
        return ht_gcv_scan(plan, coeff, d, s, eig_batch, layout, mu_grid, K, grid_per_item, G, k_best, mu_best, batch,
                           stream);
    if (plan->ndim == 2) {
        if (K < 1 || K > 1024) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: K must be in [1, 1024]");
        if (batch < 0 || batch > plan->max_batch)
            return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: batch exceeds the plan's max_batch");
        if (batch == 0) return HT_OK;
        if (!coeff || !d || !s || !mu_grid || !k_best) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: null argument");
        ht_status st2 = check_spectrum(plan, eig_batch, layout, batch, "ht_gcv_scan_exact");
        if (st2 != HT_OK) return st2;
        const Spec sp = make_spec(plan, d, s, eig_batch, layout);
        if (K > plan->xg2_max_k)
            return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: K exceeds the grid size reserved for the plan "
                                            "(ht_plan_reserve_exact_gcv)");
        GcvOut o{mu_grid, grid_per_item ? static_cast<int64_t>(K) : 0, K, G, k_best, mu_best};
        return gcv_exact_2d(plan, coeff, sp, o, batch, plan_xg2_work(plan), stream);
    }
    if (!plan->xg_mem[0])  // periodic / reflective: T is unitary and eq. gcv2 is eq. gcv
        return ht_gcv_scan(plan, coeff, d, s, eig_batch, layout, mu_grid, K, grid_per_item, G, k_best, mu_best, batch,
                           stream);
    if (K < 1 || K > 1024) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: K must be in [1, 1024]");
    if (batch < 0 || batch > 0x7fffffffLL) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: batch out of range");
    if (batch == 0) return HT_OK;
    if (!coeff || !d || !s || !mu_grid || !k_best) return fail(HT_ERR_INVALID_ARG, "ht_gcv_scan_exact: null argument");
    ht_status st = check_spectrum(plan, eig_batch, HT_SPECTRUM_FULL, batch, "ht_gcv_scan_exact");
    if (st != HT_OK) return st;
    const Spec sp = make_spec(plan, d, s, eig_batch, HT_SPECTRUM_FULL);
    GcvOut o{mu_grid, grid_per_item ? static_cast<int64_t>(K) : 0, K, G, k_best, mu_best};
    hipLaunchKernelGGL((plan->cplx ? k_gcv_exact<true, false> : k_gcv_exact<false, false>),
                       dim3(static_cast<unsigned>(batch)), dim3(XG_THREADS), 0, stream, sp, coeff, o, plan->xg[0],
                       plan->ax[0].n, static_cast<int64_t>(0), static_cast<double*>(nullptr));
    return check_hip(hipGetLastError(), "ht_gcv_scan_exact launch");
}
