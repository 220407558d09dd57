// The persistent fused restore kernel of ragged batches (device code shared by the
// per-mode source files ht_batch_k_*.hip and the host code in ht_batch.hip).
//
// For every signal a workgroup runs the whole method without leaving the chip between
// steps: inverse transform (Theorem th:inv) -> eigenvalues of the blur and of the
// smoothing operator on the signal's grid (eqs. jcf, Ac) -> GCV over the signal's grid
// (eq. mugcv) -> Tikhonov filter at the chosen mu (eq. freg) -> forward transform.  The
// coefficients, eigenvalues and filter factors live in registers; LDS holds the FFT, then
// the exactly rounded cosine table of the signal's grid, then the (t_i, w_i) pairs the
// GCV sums read.  Workgroups take signals from a per-class queue (an atomic counter),
// longest first.
#pragma once

#include <hip/hip_runtime.h>

#include "chirp_core.h"
#include "ht_internal.h"

namespace ht {

constexpr int NCLASS = 6;          // (LOGP, S): (9,1) (10,1) (11,1) (12,1) (13,1) (13,2)
// Each size class's queue is cut into one contiguous segment per XCD (the GPU hands
// workgroup b to XCD b mod 8): a workgroup drains its own XCD's segment first, so signals of
// equal length and kind, which sit next to each other in the longest-first order, run on
// one XCD and share its L2 copy of their transform tables; then it takes work from the
// other segments in turn.
constexpr int NSEG = 8;
static_assert(NCLASS * NSEG <= 64, "the counter reset kernel has 64 threads");
constexpr int BATCH_MAX_K = 256;

struct RSig {
    int64_t off;        // offset of the signal in the concatenated signal / output arrays
    int64_t psf_off;    // offset of its mask in the concatenated PSF array
    int32_t psf_len, psf_center;
    int32_t axis;       // index of its transform tables
    int32_t item;       // caller's index (row of the mu grid, outputs)
};

struct RaggedArgs {
    const Axis* axes;
    const RSig* sigs;
    int* counters;
    const double* g;
    const double* psf;
    const double* mus;
    int K;
    int norm;
    double* f;
    double* G;
    int32_t* kbest;
    double* mubest;
    double* scratch;    // MAX_N doubles per persistent workgroup of the split class
    const float* pred;  // learned mode: predicted log10(mu) per item
    int32_t* fallback;  // learned mode: 1 where the certificate failed and the full scan ran
    float* feat;        // feature mode: [count][NFEAT]
    int cert_half;      // learned mode: certificate bracket half-width in grid steps
    double* spec;       // feature mode: blur eigenvalues written here; learned mode: read (or null)
    // fused mode: the network 72 -> 256 -> 256 -> 256 -> 1 (bfloat16 weights [in][out],
    // float32 biases, feature standardisation); pred / feat receive the prediction and the
    // features when non-null
    const uint16_t* w[4];
    const float* bias[4];
    const float* fmean;
    const float* fstd;
    float* pred_out;
    // per class, NSEG contiguous segments of its longest-first queue ([NCLASS][NSEG + 1]
    // offsets within the class); counters then hold one queue head per (class, segment)
    const int* seg;
};

// What one pass of the fused kernel does with each signal.
enum BatchMode {
    MODE_SCAN = 0,      // inverse, eigenvalues, full GCV scan, filter, forward
    MODE_FEATURES = 1,  // inverse, eigenvalues, band statistics; the coefficients go to f
    MODE_LEARNED = 2,   // coefficients from f, eigenvalues, GCV certificate around the
                        // predicted mu (full scan if it fails), filter, forward
    MODE_FUSED = 3,     // inverse, eigenvalues, features, the network's prediction, then as
                        // MODE_LEARNED: one pass per signal
    MODE_LEARNED_RC = 4 // MODE_LEARNED without the feature pass's spectrum: the eigenvalues
                        // are recomputed from the PSF
};
constexpr int MLP_H = 256;  // hidden width of the network
constexpr int NFEAT_G = 64, NFEAT_D = 8, NFEAT = NFEAT_G + NFEAT_D;
constexpr int HS_MAX = 64;  // centred masks up to this half-width get their tap pairs staged in LDS
constexpr double CERT_SLACK = 1.05;   // G(predicted) may exceed the bracket minimum by 5%
constexpr float LOG10_2F = 0.30102999566398120f;

inline int class_of(const Axis& a) { return a.S == 2 ? 5 : a.logP - MIN_LOGP; }


// 1/u to full float64 accuracy: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_nr(double u) {
    double r = __builtin_amdgcn_rcp(u);
    double e = fma(-u, r, 1.0);
    r = fma(r, e, r);
    e = fma(-u, r, 1.0);
    return fma(r, e, r);
}

// Partial GCV sums of two grid values mu_a, mu_b over the staged elements
// i = part, part + nparts, ... < n.  Two elements share one reciprocal:
// 1/u0 = u1 / (u0 u1), 1/u1 = u0 / (u0 u1) (u >= mu > 0, the staged t are < 1e150).
__device__ __forceinline__ void gcv_two(const double2* stage, int n, int part, int nparts, double mua, double mub,
                                        double& Na, double& Da, double& Nb, double& Db) {
    double na0 = 0.0, na1 = 0.0, da0 = 0.0, da1 = 0.0;
    double nb0 = 0.0, nb1 = 0.0, db0 = 0.0, db1 = 0.0;
    int i = part;
    for (; i + nparts < n; i += 2 * nparts) {
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
    if (i < n) {
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

// Copy a record that every lane reads at the same address into scalar registers: each
// 32-bit word goes through readfirstlane, so the compiler knows the fields (sizes, table
// pointers) are wave-uniform and addresses tables as scalar base + lane offset.
template <class T>
__device__ __forceinline__ T uniform_load(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "record must be a whole number of words");
    T out;
    const int* src = reinterpret_cast<const int*>(p);
    int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

// float32 -> bfloat16 (round to nearest even) -> float32, and the exact GELU: the rounding
// points and activation of the network kernels of the learned-mu predictor.
__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ float bf16_load(const uint16_t* p, int i) {
    return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
}
__device__ __forceinline__ float gelu_exact(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

// One dense layer of the network for one signal, in LDS: out[j] = act(sum_k in[k] W[k][j]
// + b[j]) for j < 256.  With BLOCK >= 256 the contraction is split into BLOCK / 256 equal
// ranges whose float32 partial sums are added in order; smaller workgroups give each
// thread 256 / BLOCK outputs.  act: 1 = GELU then bfloat16 rounding, 0 = none.
template <int BLOCK>
__device__ __forceinline__ void mlp_layer(const float* in, int K, const uint16_t* __restrict__ W,
                                          const float* __restrict__ b, float* out, float* part, int act) {
    const int tid = threadIdx.x;
    if constexpr (BLOCK >= MLP_H) {
        constexpr int G = BLOCK / MLP_H;
        const int j = tid % MLP_H, gi = tid / MLP_H;
        const int k0 = gi * K / G, k1 = (gi + 1) * K / G;
        float acc = 0.0f;
#pragma unroll 2
        for (int k = k0; k < k1; ++k) acc = fmaf(in[k], bf16_load(W, k * MLP_H + j), acc);
        part[gi * MLP_H + j] = acc;
        __syncthreads();
        if (gi == 0) {
            float z = part[j];
#pragma unroll
            for (int q = 1; q < G; ++q) z += part[q * MLP_H + j];
            z += b[j];
            out[j] = act ? bf16_round(gelu_exact(z)) : z;
        }
    } else {
        for (int j = tid; j < MLP_H; j += BLOCK) {
            float acc = 0.0f;
#pragma unroll 2
            for (int k = 0; k < K; ++k) acc = fmaf(in[k], bf16_load(W, k * MLP_H + j), acc);
            const float z = acc + b[j];
            out[j] = act ? bf16_round(gelu_exact(z)) : z;
        }
    }
    __syncthreads();
}

// ---- Half-length real cores (the algebra is in make_half, ht_plan.hip).  They run on an
// LDS FFT of 2^LOGP points (no split); the input comes through x(j) (core index j < N),
// which may read LDS; the result goes to the caller's slots; LDS is free on return.

// Chirp-z DFT on slot values: v[k] holds the input of j = tid + k BLOCK < nin and receives
// post_j * (b * (pre x))_j for j < nout (the tables fix the length and sign).
template <int LOGP, int SL>
__device__ __forceinline__ void chirp_slots(double2 (&v)[SL], const Chirp& ch, int nin, int nout, double2* lds,
                                            const double2* __restrict__ tw) {
    constexpr int BLOCK = (1 << LOGP) / SL;
    // a fresh thread index per phase: no lane offset is held across the FFTs
    int tid = local_tid();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        v[k] = j < nin ? cmul(v[k], tload(ch.pre, j)) : make_double2(0.0, 0.0);
    }
    __builtin_amdgcn_sched_barrier(0);
    fft_slots<LOGP, -1, SL, true>(v, lds, tw);
    __builtin_amdgcn_sched_barrier(0);
    tid = local_tid();
#pragma unroll
    for (int k = 0; k < SL; ++k) v[k] = cmul(v[k], tload(ch.B, static_cast<unsigned>(tid + k * BLOCK)));
    __builtin_amdgcn_sched_barrier(0);
    fft_slots<LOGP, 1, SL, true>(v, lds, tw);
    __builtin_amdgcn_sched_barrier(0);
    tid = local_tid();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        if (j < nout) v[k] = cmul(v[k], tload(ch.post, j));
    }
}

// Split a complex DFT Z of length H of z_m = y_{2m} + i y_{2m+1} (held in LDS) into the
// two real-input halves at index k: E_k = (Z_k + conj Z_{H-k}) / 2 and
// O_k = (Z_k - conj Z_{H-k}) / (2i) (indices mod H).
__device__ __forceinline__ void split_real(const double2* Z, int H, int k, double2& E, double2& O) {
    const double2 a = Z[k == H ? 0 : k], b = Z[k == 0 ? 0 : H - k];
    E = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    O = make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x));
}

// DCT-II analysis of the cosine core: X_j = w_j sum_i x_i cos(pi j (2i+1) / (2N)).
template <int LOGP, int SL, class X>
__device__ __forceinline__ void half_dct2(double (&out)[SL], const Axis& ax, double2* lds,
                                          const double2* __restrict__ tw, X x) {
    constexpr int BLOCK = (1 << LOGP) / SL;
    int tid = local_tid();
    const int N = ax.N, H = ax.H;
    auto vsrc = [&](int p) { return p < (N + 1) / 2 ? 2 * p : 2 * N - 2 * p - 1; };  // Makhoul order
    double2 v[SL];
    if (ax.half == 2) {  // N odd: V_k (k < H = (N+1)/2) of the real v, by chirp-z of length N
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int p = tid + k * BLOCK;
            v[k] = make_double2(p < N ? x(vsrc(p)) : 0.0, 0.0);
        }
        __syncthreads();
        chirp_slots<LOGP, SL>(v, ax.ana, N, H, lds, tw);
        tid = local_tid();
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int m = tid + k * BLOCK;
            if (m < H) lds[m] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j < N) {
                const int kk = j < H ? j : N - j;                      // V_{N-j} = conj V_j
                const double2 W = cmul(tload(ax.htw, kk), lds[kk]);   // e^{-i pi kk/(2N)} V_kk
                const double w = j == 0 ? ax.hw[0] : ax.hw[1];
                out[k] = j < H ? w * W.x : -w * W.y;
            }
        }
        __syncthreads();
        return;
    }
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int m = tid + k * BLOCK;
        v[k] = m < H ? make_double2(x(vsrc(2 * m)), x(vsrc(2 * m + 1))) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    chirp_slots<LOGP, SL>(v, ax.ana, H, H, lds, tw);
    tid = local_tid();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int m = tid + k * BLOCK;
        if (m < H) lds[m] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        if (j < N) {
            const int kk = j <= H ? j : N - j;
            double2 E, O;
            split_real(lds, H, kk, E, O);
            const double2 V = cadd(E, cmul(tload(ax.htw, kk), O));        // V_kk = E + e^{-2 pi i kk/N} O
            const double2 W = cmul(tload(ax.htw, H + 1 + kk), V);         // e^{-i pi kk/(2N)} V_kk
            const double w = j == 0 ? ax.hw[0] : ax.hw[1];
            out[k] = j <= H ? w * W.x : -w * W.y;
        }
    }
    __syncthreads();
}

// DCT-III synthesis of the cosine core: u_i = sum_j w_j y_j cos(pi j (2i+1) / (2N)).
template <int LOGP, int SL, class Y>
__device__ __forceinline__ void half_dct3(double (&out)[SL], const Axis& ax, double2* lds,
                                          const double2* __restrict__ tw, Y y) {
    constexpr int BLOCK = (1 << LOGP) / SL;
    int tid = local_tid();
    const int N = ax.N, H = ax.H;
    auto wy = [&](int j) { return j < N ? (j == 0 ? ax.hw[0] : ax.hw[1]) * y(j) : 0.0; };
    // V_k = e^{i pi k/(2N)} (Y_k - i Y_{N-k}) for 0 < k <= H, and V_0 = 2 Y_0 (the k = 0
    // term has no mirror partner in v_p = sum_k V_k e^{2 pi i kp/N} / 2)
    auto Vof = [&](int k) {
        return k == 0 ? make_double2(2.0 * wy(0), 0.0)
                      : cmulc(make_double2(wy(k), -wy(N - k)), tload(ax.htw, H + 1 + k));
    };
    double2 v[SL];
    if (ax.half == 2) {
        // N odd: u_p = Re sum_{k < H} U_k e^{2 pi i kp/N} with U_0 = w_0 y_0 and
        // U_k = e^{i pi k/(2N)} (w y_k - i w y_{N-k}), by chirp-z of length N (H inputs)
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int m = tid + k * BLOCK;
            v[k] = m == 0 ? make_double2(wy(0), 0.0)
                 : m < H  ? cmulc(make_double2(wy(m), -wy(N - m)), tload(ax.htw, m))
                          : make_double2(0.0, 0.0);
        }
        __syncthreads();
        chirp_slots<LOGP, SL>(v, ax.syn, H, N, lds, tw);
        tid = local_tid();
        double* ur = reinterpret_cast<double*>(lds);
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int p = tid + k * BLOCK;
            if (p < N) ur[p] = v[k].x;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j < N) out[k] = ur[(j & 1) ? N - 1 - (j >> 1) : (j >> 1)];  // Makhoul position of u_j
        }
        __syncthreads();
        return;
    }
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int m = tid + k * BLOCK;
        if (m < H) {
            const double2 a = Vof(m), b = Vof(H - m);
            // U_m = ((V_m + conj V_{H-m}) + i e^{2 pi i m/N} (V_m - conj V_{H-m})) / 2
            const double2 T = cmulc(make_double2(a.x - b.x, a.y + b.y), tload(ax.htw, m));
            v[k] = make_double2(0.5 * (a.x + b.x - T.y), 0.5 * (a.y - b.y + T.x));
        } else {
            v[k] = make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    chirp_slots<LOGP, SL>(v, ax.syn, H, H, lds, tw);
    tid = local_tid();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int m = tid + k * BLOCK;
        if (m < H) lds[m] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        if (j < N) {
            const int p = (j & 1) ? N - 1 - (j >> 1) : (j >> 1);  // Makhoul position of u_j
            const double2 um = lds[p >> 1];
            out[k] = (p & 1) ? um.y : um.x;
        }
    }
    __syncthreads();
}

// Sine core (L = N + 1 = 2H), both directions: out_j = sqrt(2/L) S_{j+1},
// S_s = sum_t x_t sin(pi s t / L) (1-based, x_t = x(t - 1)).  wsum: 16 doubles of LDS.
template <int LOGP, int SL, class X>
__device__ __forceinline__ void half_dst(double (&out)[SL], const Axis& ax, double2* lds,
                                         const double2* __restrict__ tw, X x, double* wsum) {
    constexpr int BLOCK = (1 << LOGP) / SL;
    int tid = local_tid();
    const int N = ax.N, H = ax.H, L = 2 * H;
    auto xs = [&](int t) { return t >= 1 && t <= N ? x(t - 1) : 0.0; };
    auto ys = [&](int t) {  // y_t = sin(pi t/L) (x_t + x_{L-t}) + (x_t - x_{L-t}) / 2
        const double sn = tload(ax.htw, H + 1 + (t <= H ? t : L - t)).x;
        const double a = xs(t), b = xs(L - t);
        return fma(sn, a + b, 0.5 * (a - b));
    };
    double2 v[SL];
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int m = tid + k * BLOCK;
        v[k] = m < H ? make_double2(ys(2 * m), ys(2 * m + 1)) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    chirp_slots<LOGP, SL>(v, ax.ana, H, H, lds, tw);
    tid = local_tid();
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int m = tid + k * BLOCK;
        if (m < H) lds[m] = v[k];
    }
    __syncthreads();
    // real DFT Y_k = E_k + e^{2 pi i k/L} O_k: R_k = Re Y_k (R_0 halved), I_k = Im Y_k
    double rr[SL], ii[SL];
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int kk = tid + k * BLOCK;
        rr[k] = ii[k] = 0.0;
        if (kk < H) {
            double2 E, O;
            split_real(lds, H, kk, E, O);
            const double2 Y = cadd(E, cmul(tload(ax.htw, kk), O));
            rr[k] = kk == 0 ? 0.5 * Y.x : Y.x;
            ii[k] = Y.y;
        }
    }
    __syncthreads();
    double* Rs = reinterpret_cast<double*>(lds);  // [H]: R, then its inclusive prefix sums
    double* Is = Rs + H;                          // [H]
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int kk = tid + k * BLOCK;
        if (kk < H) {
            Rs[kk] = rr[k];
            Is[kk] = ii[k];
        }
    }
    __syncthreads();
    // inclusive prefix sums of Rs: a contiguous chunk per thread (H <= P/2, so at most SL/2
    // entries), the chunk totals scanned across each wave, then across the waves (fixed order)
    {
        constexpr int CMAX = SL / 2;
        const int C = (H + BLOCK - 1) / BLOCK;
        const int k0 = tid * C;
        double loc[CMAX];
        double run = 0.0;
#pragma unroll
        for (int e = 0; e < CMAX; ++e) {
            if (e < C && k0 + e < H) run += Rs[k0 + e];
            loc[e] = run;
        }
        const int lane = tid & 63, wv = tid >> 6;
        double incl = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        double off = incl - run;
        for (int w = 0; w < wv; ++w) off += wsum[w];
#pragma unroll
        for (int e = 0; e < CMAX; ++e)
            if (e < C && k0 + e < H) Rs[k0 + e] = off + loc[e];
        __syncthreads();
    }
    const double sc = ax.hw[0];
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        if (j < N) {
            const int s = j + 1;
            out[k] = sc * ((s & 1) ? Rs[s >> 1] : Is[s >> 1]);
        }
    }
    __syncthreads();
}

// The 1024-, 2048- and 4096-point classes with 8 points per thread are held to 128
// registers per lane (four waves per SIMD): two to eight workgroups then share a CU and
// cover each other's barrier and memory waits, which pays for the spills this costs
// (measured: 20 % less time in the 2048- and 4096-point classes; the 512-point class of
// single-wave workgroups is slower so, and the 8192-point classes are bound by their LDS
// to one workgroup per CU).
template <int LOGP, int S, int SL>
constexpr int restore_waves_per_eu() { return LOGP >= 10 && LOGP <= 12 && SL == 8 ? 4 : 1; }

template <int LOGP, int S, int SL, int MODE>
__global__ __launch_bounds__((1 << LOGP) / SL)
__attribute__((amdgpu_waves_per_eu(restore_waves_per_eu<LOGP, S, SL>())))
void k_restore(RaggedArgs a, int cls, int start, int count) {
    constexpr int P = 1 << LOGP;
    constexpr int BLOCK = P / SL;
    // cross-part GCV reduction buffer: only 64-thread groups can need more than one pass
    // over the grid (K > 2 * BLOCK); otherwise the reduction reuses the staging buffer
    constexpr int RED = BLOCK < BATCH_MAX_K / 2 ? 2 * BLOCK : 1;
    __shared__ double2 lds[P];
    __shared__ double2 red_small[RED];
    __shared__ double Gs[BATCH_MAX_K];
    __shared__ double2 bc[3];
    __shared__ int s_item, s_kbest;
    __shared__ float s_pred;
    __shared__ double s_wsum[16];  // wave totals of the half sine core's prefix sums
    __shared__ double2 s_spread[2 * (BLOCK / 64)];  // per-wave sums of a spread GCV pair
    __shared__ double s_hs[HS_MAX + 1];              // tap pairs of a centred mask
    const int tid = threadIdx.x;
    double* scratch = a.scratch + static_cast<int64_t>(blockIdx.x) * MAX_N;
    // Classes of 4096 points and more take their next queue entry while the current signal
    // runs (the atomic's latency then hides behind the signal's own loads); their long
    // queues per workgroup make the one reserved entry irrelevant to the load balance,
    // which it does disturb for the short queues of the small classes.
    constexpr bool PREFETCH = LOGP >= 12;
    // queue position of thread 0: the segment it takes from, and how many it has left
    const int* segb = a.seg + cls * (NSEG + 1);
    int* qc = a.counters + cls * NSEG;
    int sq = blockIdx.x % NSEG, left = NSEG;
    auto next_item = [&]() -> int {
        while (left > 0) {
            const int lo = segb[sq], hi = segb[sq + 1];
            if (hi > lo) {
                const int i = lo + atomicAdd(&qc[sq], 1);
                if (i < hi) return i;
            }
            sq = sq + 1 == NSEG ? 0 : sq + 1;
            --left;
        }
        return count;
    };
    // the certified pass: coefficients from f (left there by the feature pass); the lean
    // form also takes d from the feature pass's spectrum and keeps neither the coefficients
    // nor d, s in registers across the GCV phase (it re-reads them), which is what bounds
    // its register use
    constexpr bool FROM_F = MODE == MODE_LEARNED || MODE == MODE_LEARNED_RC;
    constexpr bool LEAN = MODE == MODE_LEARNED;
    constexpr bool CERT = FROM_F || MODE == MODE_FUSED;
    int nxt = 0;
    if (PREFETCH && tid == 0) nxt = next_item();
    for (;;) {
        if (tid == 0) s_item = PREFETCH ? nxt : next_item();
        __syncthreads();
        // uniform across the workgroup: keeps the signal's descriptor and table pointers in
        // scalar registers
        const int qi = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (qi >= count) break;
        if (PREFETCH && tid == 0) nxt = next_item();
        // per signal: nothing derived from the thread index is held across signals
        const int tid = local_tid();
        const RSig sg = uniform_load(a.sigs + start + qi);
        const Axis ax = uniform_load(a.axes + sg.axis);
        // read per signal so that no twiddle address is hoisted out of the queue loop
        const double2* __restrict__ tw = ax.tw;
        const int n = ax.n, N = ax.N, rank = ax.rank, kind = ax.kind, den = ax.den;
        const double* g = a.g + sg.off;
        double* f = a.f + sg.off;
        const double* h = a.psf + sg.psf_off;
        const double q1 = ax.q1;

        // ---- inverse transform: boundary coefficients, interior correction, core analysis
        double x1, xn;
        double c[SL];
        float lcf[SL];  // feature pass: log10(c^2 + 1e-20)
        if constexpr (FROM_F) {  // coefficients left in f by the feature pass
            x1 = f[0];
            xn = f[n - 1];
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                // the lean pass re-reads them where it needs them (no registers held
                // across the GCV phase)
                c[k] = (!LEAN && j < N) ? f[j + 1] : 0.0;
            }
        } else {
        {
            const double y0 = g[0], y1 = g[1], yN = g[n - 2], yL = g[n - 1];
            if (kind == HT_KIND_C) {
                const double r1 = y0 - y1, r2 = yL - yN;
                x1 = ax.minv[0] * r1 + ax.minv[1] * r2;
                xn = ax.minv[2] * r1 + ax.minv[3] * r2;
            } else {
                x1 = y0 / q1;
                xn = yL / q1;
            }
        }
        {
            auto in_inv = [&](int, int j) {
                return make_double2(g[j + 1] - dtab(ax.q, j + 1) * x1 - dtab(ax.q, N - j) * xn, 0.0);
            };
            auto park = [&](int j, double y) { f[j + 1] = y; };
            auto unpark = [&](int j) { return f[j + 1]; };
            bool done = false;
            if constexpr (S == 1) {
                if (ax.half) {  // uniform per signal
                    auto xg = [&](int j) { return g[j + 1] - dtab(ax.q, j + 1) * x1 - dtab(ax.q, N - j) * xn; };
                    if constexpr (MODE == MODE_FEATURES || MODE == MODE_FUSED) {
                        // the corrected interior goes through LDS: coalesced reads of g and q
                        // here, the cores' reordered reads from LDS (measured faster in
                        // these modes, slower in the scan mode, which reads g directly)
                        double* rs = reinterpret_cast<double*>(lds);
#pragma unroll
                        for (int k = 0; k < SL; ++k) {
                            const int j = tid + k * BLOCK;
                            if (j < N) rs[j] = xg(j);
                        }
                        __syncthreads();
                        auto xr = [&](int j) { return rs[j]; };
                        if (kind == HT_KIND_C)
                            half_dct2<LOGP, SL>(c, ax, lds, tw, xr);
                        else
                            half_dst<LOGP, SL>(c, ax, lds, tw, xr, s_wsum);
                    } else {
                        if (kind == HT_KIND_C)
                            half_dct2<LOGP, SL>(c, ax, lds, tw, xg);
                        else
                            half_dst<LOGP, SL>(c, ax, lds, tw, xg, s_wsum);
                    }
                    done = true;
                }
            }
            if (!done) chirp_core<LOGP, S, SL, true>(c, ax.ana, ax.ana.mode, N, lds, tw, in_inv, park, unpark);
        }
        if (rank > 0) {  // DST family correction x_mid -= U (E^T K)^{-1} E^T x_mid
            if (tid < rank) bc[tid].x = c[0];
            __syncthreads();
            const double s0 = bc[0].x, s1 = rank > 1 ? bc[1].x : 0.0;
            const double a0 = ax.Gm[0] * s0 + ax.Gm[1] * s1;
            const double a1 = ax.Gm[2] * s0 + ax.Gm[3] * s1;
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N) {
                    c[k] -= dtab(ax.U, j) * a0;
                    if (rank > 1) c[k] -= dtab(ax.U, N + j) * a1;
                }
            }
        }
        if constexpr (MODE == MODE_FEATURES) {  // the coefficient vector for the learned pass
            __syncthreads();
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N) f[j + 1] = c[k];
                // only the logarithm is needed from here on (the features): one float
                // register per slot instead of a double across the eigenvalue sums
                lcf[k] = __builtin_amdgcn_logf(static_cast<float>(c[k] * c[k] + 1e-20)) * LOG10_2F;
            }
            if (tid == 0) {
                f[0] = x1;
                f[n - 1] = xn;
            }
        }
        }

        __builtin_amdgcn_sched_barrier(0);
        // ---- eigenvalues on the signal's grid: cos(pi r / den), r <= den, staged in LDS
        // (the learned pass reads d from the feature pass and needs only cos(pi num / den)
        // at its own frequency for s: it reads those straight from the table, coalesced,
        // and skips the staging)
        const bool staged = !LEAN;
        double* ctab = reinterpret_cast<double*>(lds);
        // centred masks up to HS_MAX taps per side: the tap pairs h_t + h_{-t} staged in LDS
        // (the same sums as in the loop below: results do not change)
        const bool hstage = staged && 2 * sg.psf_center + 1 == sg.psf_len && sg.psf_center <= HS_MAX;
        if (staged) {
            __syncthreads();
            for (int r = tid; r <= den; r += BLOCK) ctab[r] = dtab(ax.tcos, r);
            if (hstage) {
                const int pc0 = sg.psf_center;
                for (int t = tid; t <= pc0; t += BLOCK) s_hs[t] = t == 0 ? h[pc0] : h[pc0 + t] + h[pc0 - t];
            }
            __syncthreads();
        }
        double z0 = 0.0;
        for (int t = 0; t < sg.psf_len; ++t) z0 += h[t];
        const bool ident = a.norm == HT_NORM_IDENTITY;
        const double s_poly = ident ? 1.0 : 0.0;
        const int per = 2 * den;
        const int pc = sg.psf_center, pl = sg.psf_len;
        const bool centred = 2 * pc + 1 == pl;
        // Mirror pairs (centred masks): the frequency of index mj = (C: N - j, sine: N - 1 - j)
        // is pi - theta_j, where cos(t (pi - theta)) = (-1)^t cos(t theta); summing the even
        // and the odd taps apart gives d_j = E + O and d_mj = E - O in one pass over the
        // taps.  The lower index of a pair computes both and leaves d_mj in LDS behind the
        // staged table (den + 1 + N <= 2P doubles) for the owner of mj.
        const bool pair = staged && centred;
        double* dmir = ctab + den + 1;
        auto mirror = [&](int j) { return kind == HT_KIND_C ? N - j : N - 1 - j; };
        double dj[SL], sj[SL];
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            dj[k] = z0;
            sj[k] = s_poly;
            if (!LEAN && j < N && j >= rank) {
                const int num = kind == HT_KIND_C ? j : j + 1;  // frequency pi * num / den
                const int mj = mirror(j);
                const bool lead = pair && mj > j && mj < N && mj >= rank;
                const bool follow = pair && mj < j && mj >= rank;
                double acc = 0.0;
                if (LEAN) {
                    // d and s are read where they are used (lean_ds)
                } else if (follow) {
                    // d_j arrives from the owner of mj below
                } else if (centred && hstage) {
                    double ev = s_hs[0], od = 0.0;
                    int r = 0, t = 1;
                    for (; t + 1 <= pc; t += 2) {
                        r += num;
                        if (r >= per) r -= per;
                        od = fma(s_hs[t], ctab[r <= den ? r : per - r], od);
                        r += num;
                        if (r >= per) r -= per;
                        ev = fma(s_hs[t + 1], ctab[r <= den ? r : per - r], ev);
                    }
                    if (t <= pc) {
                        r += num;
                        if (r >= per) r -= per;
                        od = fma(s_hs[t], ctab[r <= den ? r : per - r], od);
                    }
                    acc = ev + od;
                    if (lead) dmir[mj] = ev - od;
                } else if (centred) {
                    // Re z = h_0 + sum_{t>0} (h_t + h_{-t}) cos(t theta), even and odd t apart
                    double ev = h[pc], od = 0.0;
                    int r = 0, t = 1;
                    for (; t + 1 <= pc; t += 2) {
                        r += num;
                        if (r >= per) r -= per;
                        od = fma(h[pc + t] + h[pc - t], ctab[r <= den ? r : per - r], od);
                        r += num;
                        if (r >= per) r -= per;
                        ev = fma(h[pc + t + 1] + h[pc - t - 1], ctab[r <= den ? r : per - r], ev);
                    }
                    if (t <= pc) {
                        r += num;
                        if (r >= per) r -= per;
                        od = fma(h[pc + t] + h[pc - t], ctab[r <= den ? r : per - r], od);
                    }
                    acc = ev + od;
                    if (lead) dmir[mj] = ev - od;
                } else {
                    int r = static_cast<int>((static_cast<int64_t>(per) * pl - static_cast<int64_t>(pc) * num) % per);
                    for (int t = 0; t < pl; ++t) {
                        const double cv = ctab[r <= den ? r : per - r];
                        acc = fma(h[t], cv, acc);
                        r += num;
                        if (r >= per) r -= per;
                    }
                }
                dj[k] = acc;
                const int rn = num % per;
                const int rc = rn <= den ? rn : per - rn;
                sj[k] = ident ? 1.0 : 2.0 - 2.0 * (staged ? ctab[rc] : dtab(ax.tcos, rc));
            }
        }
        __syncthreads();
        if (pair) {  // uniform: the mirrored halves, then LDS is free for the next phase
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N && j >= rank) {
                    const int mj = mirror(j);
                    if (mj < j && mj >= rank) dj[k] = dmir[j];
                }
            }
            __syncthreads();
        }

        __shared__ float s_feat[NFEAT];
        if constexpr (MODE == MODE_FEATURES || MODE == MODE_FUSED) {
            // band means of log10(|ghat_j|^2 + 1e-20) (64 bands) and log10(|d_j|^2 + 1e-20) (8 bands) over the
            // normalised core frequency j / N; band b holds j with floor(B j / N) = b
            // (float32 logarithms: the features are float32)
            double2* lg = lds;
            constexpr float LOG10_2 = 0.30102999566398120f;
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N) {
                    const float lc = MODE == MODE_FEATURES
                                         ? lcf[k]
                                         : __builtin_amdgcn_logf(static_cast<float>(c[k] * c[k] + 1e-20)) * LOG10_2;
                    const float ld = __builtin_amdgcn_logf(static_cast<float>(dj[k] * dj[k] + 1e-20)) * LOG10_2;
                    lg[j] = make_double2(lc, ld);
                    if (a.spec) a.spec[sg.off + 1 + j] = dj[k];
                }
            }
            if (a.spec && tid == 0) {
                a.spec[sg.off] = z0;
                a.spec[sg.off + n - 1] = z0;
            }
            __syncthreads();
            // band sums by groups of aligned lanes (a fixed-order butterfly per group):
            // 64 spectrum bands of ghat with BLOCK/64 lanes each, then 8 bands of d with up
            // to 64 lanes each
            {
                constexpr int G1 = BLOCK / NFEAT_G;
                const int b = tid / G1, r = tid - b * G1;
                const int j0 = static_cast<int>((static_cast<int64_t>(b) * N + NFEAT_G - 1) / NFEAT_G);
                const int j1 = static_cast<int>((static_cast<int64_t>(b + 1) * N + NFEAT_G - 1) / NFEAT_G);
                double acc = 0.0;
                for (int j = j0 + r; j < j1; j += G1) acc += lg[j].x;
#pragma unroll
                for (int o = G1 / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
                if (r == 0) {
                    const float v = static_cast<float>(acc / (j1 - j0));
                    if (MODE == MODE_FUSED) s_feat[b] = v;
                    if (a.feat) a.feat[static_cast<int64_t>(sg.item) * NFEAT + b] = v;
                }
            }
            {
                constexpr int G2 = BLOCK / NFEAT_D < 64 ? BLOCK / NFEAT_D : 64;
                if (tid < NFEAT_D * G2) {  // whole waves
                    const int b = tid / G2, r = tid - b * G2;
                    const int j0 = static_cast<int>((static_cast<int64_t>(b) * N + NFEAT_D - 1) / NFEAT_D);
                    const int j1 = static_cast<int>((static_cast<int64_t>(b + 1) * N + NFEAT_D - 1) / NFEAT_D);
                    double acc = 0.0;
                    for (int j = j0 + r; j < j1; j += G2) acc += lg[j].y;
#pragma unroll
                    for (int o = G2 / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
                    if (r == 0) {
                        const float v = static_cast<float>(acc / (j1 - j0));
                        if (MODE == MODE_FUSED) s_feat[NFEAT_G + b] = v;
                        if (a.feat) a.feat[static_cast<int64_t>(sg.item) * NFEAT + NFEAT_G + b] = v;
                    }
                }
            }
            __syncthreads();
            if constexpr (MODE == MODE_FEATURES) continue;
            // ---- the network's log10 mu for this signal (fused mode), computed in LDS:
            // activations at [0, 256) and [256, 512) floats, layer partial sums behind them
            float* act = reinterpret_cast<float*>(lds);
            float* part = act + 2 * MLP_H;
            for (int i = tid; i < NFEAT; i += BLOCK) act[i] = bf16_round((s_feat[i] - a.fmean[i]) / a.fstd[i]);
            __syncthreads();
            mlp_layer<BLOCK>(act, NFEAT, a.w[0], a.bias[0], act + MLP_H, part, 1);
            mlp_layer<BLOCK>(act + MLP_H, MLP_H, a.w[1], a.bias[1], act, part, 1);
            mlp_layer<BLOCK>(act, MLP_H, a.w[2], a.bias[2], act + MLP_H, part, 1);
            if (tid < 64) {  // output layer: four inputs per lane, then a fixed-order butterfly
                float y = 0.0f;
#pragma unroll
                for (int k = 4 * tid; k < 4 * tid + 4; ++k) y = fmaf(act[MLP_H + k], bf16_load(a.w[3], k), y);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, 64);
                if (tid == 0) {
                    y += a.bias[3][0];
                    s_pred = y;
                    if (a.pred_out) a.pred_out[sg.item] = y;
                }
            }
            __syncthreads();
        }

        __builtin_amdgcn_sched_barrier(0);
        // ---- GCV: stage t_i = |d_i|^2 / |s_i|^2, w_i = |ghat_i|^2 (s_i = 0: no contribution)
        double2* stage = lds;
        // lean pass: d_j from the feature pass's spectrum, s_j from the cosine table
        auto lean_ds = [&](int j, double& d, double& sv) {
            d = a.spec[sg.off + 1 + j];
            if (j < rank) {
                sv = s_poly;
            } else {
                const int rn = (kind == HT_KIND_C ? j : j + 1) % per;
                sv = ident ? 1.0 : 2.0 - 2.0 * dtab(ax.tcos, rn <= den ? rn : per - rn);
            }
        };
        auto stage_fill = [&]() {
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N) {
                    double d = dj[k], sv = sj[k], cj = c[k];
                    if (LEAN) {
                        lean_ds(j, d, sv);
                        cj = f[j + 1];
                    }
                    const double s2 = sv * sv;
                    stage[j] = s2 != 0.0 ? make_double2(d * d / s2, cj * cj) : make_double2(1e150, 0.0);
                }
            }
            if (tid == 0) {
                const double s2 = s_poly * s_poly;
                stage[N] = s2 != 0.0 ? make_double2(z0 * z0 / s2, x1 * x1) : make_double2(1e150, 0.0);
                stage[N + 1] = s2 != 0.0 ? make_double2(z0 * z0 / s2, xn * xn) : make_double2(1e150, 0.0);
            }
            __syncthreads();
        };
        const int K = a.K;
        const double* mus = a.mus + static_cast<int64_t>(sg.item) * K;
        // G_k for k in [klo, khi] into Gs (and a.G), two grid values per evaluation.  Long
        // ranges: the lanes take different pairs and the workgroup splits the elements into
        // at most MAX_PARTS parts (all lanes of a part read the same staged element), the
        // parts are added in order through LDS (this overwrites the staged pairs).  Short
        // ranges (would need more parts): one wave per pair, its lanes striding over the
        // elements, a fixed-order butterfly across the lanes; the staged pairs survive.
        // Returns whether the staged pairs are still in place.
        double2* red = lds;
        auto eval_range = [&](int klo, int khi) -> bool {
            constexpr int MAX_PARTS = 16;
            const int cnt = khi - klo + 1;
            const int Kh = (cnt + 1) / 2;
            const int Kb = Kh < BLOCK ? Kh : BLOCK;
            const int nparts = BLOCK / Kb;
            if (nparts <= MAX_PARTS) {
                const int part = tid / Kb, kl = tid - part * Kb;
                const bool one_pass = Kh <= Kb;
                double2* rbuf = one_pass ? red : red_small;
                for (int k0 = 0; k0 < Kh; k0 += Kb) {
                    const int kk = k0 + kl;
                    double Na = 0.0, Da = 0.0, Nb = 0.0, Db = 0.0;
                    if (part < nparts && kk < Kh) {
                        const int ka = klo + 2 * kk, kb2 = ka + 1 <= khi ? ka + 1 : ka;
                        gcv_two(stage, n, part, nparts, mus[ka], mus[kb2], Na, Da, Nb, Db);
                    }
                    if (one_pass) __syncthreads();
                    rbuf[2 * tid] = make_double2(Na, Da);
                    rbuf[2 * tid + 1] = make_double2(Nb, Db);
                    __syncthreads();
                    if (part == 0 && kk < Kh) {
                        double2 A = rbuf[2 * kl], B = rbuf[2 * kl + 1];
                        for (int p = 1; p < nparts; ++p) {
                            const double2 va = rbuf[2 * (p * Kb + kl)], vb = rbuf[2 * (p * Kb + kl) + 1];
                            A.x += va.x;
                            A.y += va.y;
                            B.x += vb.x;
                            B.y += vb.y;
                        }
                        const int ka = klo + 2 * kk;
                        Gs[ka] = A.x / (A.y * A.y);
                        if (a.G) a.G[static_cast<int64_t>(sg.item) * K + ka] = Gs[ka];
                        if (ka + 1 <= khi) {
                            Gs[ka + 1] = B.x / (B.y * B.y);
                            if (a.G) a.G[static_cast<int64_t>(sg.item) * K + ka + 1] = Gs[ka + 1];
                        }
                    }
                    __syncthreads();
                }
                return !one_pass;  // red_small leaves the staged pairs alone
            }
            constexpr int NW = BLOCK / 64;
            const int wv = tid >> 6, lane = tid & 63;
            // whole rounds of one pair per wave; a short remainder (at most a quarter of
            // the waves' worth of pairs, after at least one whole round) is not left to a
            // few waves while the rest wait: every wave takes a share of its elements
            // (certificate brackets only: the scan's grids fill whole rounds)
            const int full = Kh / NW * NW, rem = Kh - full;
            const bool spread = CERT && full > 0 && rem > 0 && 4 * rem <= NW;
            const int kwhole = spread ? full : Kh;
            for (int k0 = 0; k0 < kwhole; k0 += NW) {
                const int kk = k0 + wv;
                if (kk < kwhole) {  // uniform across the wave
                    const int ka = klo + 2 * kk, kb2 = ka + 1 <= khi ? ka + 1 : ka;
                    double Na, Da, Nb, Db;
                    gcv_two(stage, n, lane, 64, mus[ka], mus[kb2], Na, Da, Nb, Db);
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        Na += __shfl_xor(Na, o, 64);
                        Da += __shfl_xor(Da, o, 64);
                        Nb += __shfl_xor(Nb, o, 64);
                        Db += __shfl_xor(Db, o, 64);
                    }
                    if (lane == 0) {
                        Gs[ka] = Na / (Da * Da);
                        if (a.G) a.G[static_cast<int64_t>(sg.item) * K + ka] = Gs[ka];
                        if (ka + 1 <= khi) {
                            Gs[ka + 1] = Nb / (Db * Db);
                            if (a.G) a.G[static_cast<int64_t>(sg.item) * K + ka + 1] = Gs[ka + 1];
                        }
                    }
                }
            }
            if (spread) {
                for (int q = 0; q < rem; ++q) {
                    const int ka = klo + 2 * (full + q), kb2 = ka + 1 <= khi ? ka + 1 : ka;
                    double Na, Da, Nb, Db;
                    // elements 64 wv + lane, + BLOCK, ...: lanes, then waves, added in order
                    gcv_two(stage, n, tid, BLOCK, mus[ka], mus[kb2], Na, Da, Nb, Db);
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        Na += __shfl_xor(Na, o, 64);
                        Da += __shfl_xor(Da, o, 64);
                        Nb += __shfl_xor(Nb, o, 64);
                        Db += __shfl_xor(Db, o, 64);
                    }
                    if (lane == 0) {
                        s_spread[2 * wv] = make_double2(Na, Da);
                        s_spread[2 * wv + 1] = make_double2(Nb, Db);
                    }
                    __syncthreads();
                    if (tid == 0) {
                        double2 A = s_spread[0], B = s_spread[1];
                        for (int w = 1; w < NW; ++w) {
                            A.x += s_spread[2 * w].x;
                            A.y += s_spread[2 * w].y;
                            B.x += s_spread[2 * w + 1].x;
                            B.y += s_spread[2 * w + 1].y;
                        }
                        Gs[ka] = A.x / (A.y * A.y);
                        if (a.G) a.G[static_cast<int64_t>(sg.item) * K + ka] = Gs[ka];
                        if (ka + 1 <= khi) {
                            Gs[ka + 1] = B.x / (B.y * B.y);
                            if (a.G) a.G[static_cast<int64_t>(sg.item) * K + ka + 1] = Gs[ka + 1];
                        }
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
            return true;
        };
        // first minimum over [klo, khi]; -1 if some G is not finite
        auto argmin_range = [&](int klo, int khi) {
            if (tid < 64) {
                double best = 0.0;
                int bk = -1, bad = 0;
                for (int k = klo + tid; k <= khi; k += 64) {
                    const double gv = Gs[k];
                    if (!isfinite(gv)) bad = 1;
                    if (bk < 0 || gv < best) {
                        best = gv;
                        bk = k;
                    }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 64);
                    const int ok = __shfl_xor(bk, off, 64);
                    bad |= __shfl_xor(bad, off, 64);
                    if (ok >= 0 && (bk < 0 || ob < best || (ob == best && ok < bk))) {
                        best = ob;
                        bk = ok;
                    }
                }
                if (tid == 0) s_kbest = bad ? -1 : bk;
            }
            __syncthreads();
            return __builtin_amdgcn_readfirstlane(s_kbest);
        };
        int kstar;
        if constexpr (CERT) {
            // nearest grid index to the prediction, then the certificate bracket
            if (tid < 64) {  // wave 0: lane-strided scan, then a first-index argmin across lanes
                const double pr = static_cast<double>(MODE == MODE_FUSED ? s_pred : a.pred[sg.item]);
                int kh = K;
                double bd = __builtin_inf();
                for (int k = tid; k < K; k += 64) {
                    const double dd = fabs(log10(mus[k]) - pr);
                    if (dd < bd) {
                        bd = dd;
                        kh = k;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    const double od = __shfl_xor(bd, o);
                    const int ok = __shfl_xor(kh, o);
                    if (od < bd || (od == bd && ok < kh)) {
                        bd = od;
                        kh = ok;
                    }
                }
                if (tid == 0) s_item = kh;  // reused as a broadcast slot (the queue index was already read)
            }
            __syncthreads();
            const int khat = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            const int half = a.cert_half;
            const int lo = khat - half < 0 ? 0 : khat - half;
            const int hi = khat + half > K - 1 ? K - 1 : khat + half;
            stage_fill();
            const bool staged = eval_range(lo, hi);
            const int km = argmin_range(lo, hi);
            const bool edge = (km == lo && lo > 0) || (km == hi && hi < K - 1);
            const bool ok = km >= 0 && !edge && Gs[khat] <= CERT_SLACK * Gs[km];
            if (ok) {
                kstar = km;
            } else {
                if (!staged) stage_fill();  // the part sums went through the staging buffer
                eval_range(0, K - 1);
                kstar = argmin_range(0, K - 1);
            }
            if (tid == 0) a.fallback[sg.item] = ok ? 0 : 1;
        } else {
            stage_fill();
            eval_range(0, K - 1);
            kstar = argmin_range(0, K - 1);
        }
        if (tid == 0) {
            a.kbest[sg.item] = kstar;
            a.mubest[sg.item] = kstar >= 0 ? mus[kstar] : __builtin_nan("");
        }
        __syncthreads();
        const int kb = kstar;
        const double mu_s = kb >= 0 ? mus[kb] : __builtin_nan("");

        __builtin_amdgcn_sched_barrier(0);
        // ---- Tikhonov filter at mu*: fhat = d ghat / (d^2 + mu s^2)
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            if constexpr (LEAN) {
                const int j = tid + k * BLOCK;
                c[k] = 0.0;
                if (j < N) {
                    double d, sv;
                    lean_ds(j, d, sv);
                    c[k] = d * f[j + 1] / fma(mu_s, sv * sv, d * d);
                }
            } else {
                c[k] = dj[k] * c[k] / fma(mu_s, sj[k] * sj[k], dj[k] * dj[k]);
            }
        }
        const double fpoly = z0 / fma(mu_s, s_poly * s_poly, z0 * z0);
        const double fx1 = fpoly * x1, fxn = fpoly * xn;
        if (tid < rank) bc[tid].x = c[0];
        if (S == 2) {  // the second half of the split reads the coefficients again
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N) scratch[j] = c[k];
            }
        }
        __syncthreads();
        const double beta0 = rank > 0 ? bc[0].x : 0.0;
        const double beta1 = rank > 1 ? bc[1].x : 0.0;

        __builtin_amdgcn_sched_barrier(0);
        // ---- forward transform of the filtered coefficients
        {
            auto in_fwd = [&](int k, int j) {
                const double v = S == 2 ? scratch[j] : c[k];
                return make_double2(j >= rank ? v : 0.0, 0.0);
            };
            auto park = [&](int j, double y) { f[j + 1] = y; };
            auto unpark = [&](int j) { return f[j + 1]; };
            double u[SL];
            bool done = false;
            if constexpr (S == 1) {
                if (ax.half) {  // uniform per signal; the coefficients go through LDS
                    double* ys = reinterpret_cast<double*>(lds);
#pragma unroll
                    for (int k = 0; k < SL; ++k) {
                        const int j = tid + k * BLOCK;
                        if (j < N) ys[j] = j >= rank ? c[k] : 0.0;
                    }
                    __syncthreads();
                    auto yr = [&](int j) { return ys[j]; };
                    if (kind == HT_KIND_C)
                        half_dct3<LOGP, SL>(u, ax, lds, tw, yr);
                    else
                        half_dst<LOGP, SL>(u, ax, lds, tw, yr, s_wsum);
                    done = true;
                }
            }
            if (!done) chirp_core<LOGP, S, SL, true>(u, ax.syn, ax.syn.mode, N, lds, tw, in_fwd, park, unpark);
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int j = tid + k * BLOCK;
                if (j < N) {
                    double y = u[k] + dtab(ax.q, j + 1) * fx1 + dtab(ax.q, N - j) * fxn;
                    if (rank > 0) y += dtab(ax.bub, j) * beta0;
                    if (rank > 1) y += dtab(ax.bub, N + j) * beta1;
                    f[j + 1] = y;
                    if (kind == HT_KIND_C) {
                        if (j == 0) f[0] = q1 * fx1 + u[k];
                        if (j == N - 1) f[n - 1] = q1 * fxn + u[k];
                    }
                }
            }
            if (tid == 0 && kind != HT_KIND_C) {
                f[0] = q1 * fx1;
                f[n - 1] = q1 * fxn;
            }
        }
    }
}


// Launch of the persistent kernel of size class c in mode MODE (the variant picks 8 or 16
// points per thread for the 4096- and 8192-point classes).  Each mode's kernels are
// instantiated in a source file of their own (ht_batch_k_*.hip), compiled in parallel.
template <int MODE>
void launch_mode(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream) {
#define HT_LAUNCH(LOGP, S, SL) \
    hipLaunchKernelGGL((k_restore<LOGP, S, SL, MODE>), dim3(static_cast<unsigned>(grid)), dim3((1 << LOGP) / SL), 0, \
                       stream, a, c, start, cnt)
    switch (c) {
        case 0: HT_LAUNCH(9, 1, 8); break;
        case 1: HT_LAUNCH(10, 1, 8); break;
        case 2: HT_LAUNCH(11, 1, 8); break;
        case 3:
            if (variant) HT_LAUNCH(12, 1, 16);
            else HT_LAUNCH(12, 1, 8);
            break;
        case 4:
            if (variant) HT_LAUNCH(13, 1, 16);
            else HT_LAUNCH(13, 1, 8);
            break;
        default:
            if (variant) HT_LAUNCH(13, 2, 16);
            else HT_LAUNCH(13, 2, 8);
            break;
    }
#undef HT_LAUNCH
}

void batch_launch_scan(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream);
void batch_launch_features(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream);
void batch_launch_learned(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream);
void batch_launch_learned_rc(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid,
                             hipStream_t stream);
void batch_launch_fused(const RaggedArgs& a, int c, int variant, int start, int cnt, int grid, hipStream_t stream);
// persistent workgroups that fill the device for class c (occupancy of the scan kernel)
int batch_full_grid(int cls, int variant, int device);

}  // namespace ht
