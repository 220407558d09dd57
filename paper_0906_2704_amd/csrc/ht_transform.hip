// Forward and inverse high-order boundary transforms (eqs. ART, Tc, Tf; Theorem th:inv).
//
// One workgroup handles one 1D transform of length n.  The core (DST-I, DCT-II/III or
// DFT of order N = n - 2) is computed as a chirp-z transform by FFT convolution in LDS
// (any N, no restriction to smooth lengths); the boundary work is float64 closed form:
//
//   inverse  (T_X x = y)   [x_1, x_n] from the 2x2 boundary system (C, F; for the
//            antireflective family the boundary rows decouple: x_1 = y_1/p_1,
//            x_n = y_n/p_1), then x_mid = X (y_mid - q^ x_1 - J q^ x_n), and for the DST
//            family x_mid -= U (E^T K)^{-1} E^T x_mid.
//   forward  (y = T_X x)   u = X^{-1} x_mid, y_mid = u + q^ x_1 + J q^ x_n (+ bubbles),
//            y_1 / y_n from the extension of the core columns to the ghost grid points
//            (zero for the sine core, mirror for the cosine core, periodic wrap for the
//            exponential core) plus q_1 x_1 / q_1 x_n.
// The comparators (periodic, reflective; Section 2.1) have no boundary columns: the whole
// vector is the core of order n.
#include <hip/hip_runtime.h>

#include "chirp_core.h"
#include "ht_internal.h"

namespace ht {

__device__ __forceinline__ double2 vload(const View& v, int64_t base, int64_t i) {
    const int64_t off = base + i * v.elem_stride;
    if (v.cplx) return static_cast<const double2*>(v.ptr)[off];
    return make_double2(static_cast<const double*>(v.ptr)[off], 0.0);
}

__device__ __forceinline__ void vstore(const View& v, int64_t base, int64_t i, double2 x) {
    const int64_t off = base + i * v.elem_stride;
    if (v.cplx)
        static_cast<double2*>(v.ptr)[off] = x;
    else
        static_cast<double*>(v.ptr)[off] = x.x;
}

__device__ __forceinline__ int64_t vbase(const View& v, int64_t b) {
    return (b / v.per_img) * v.img_stride + (b % v.per_img) * v.sig_stride;
}

// Workgroups are handed to the 8 XCDs round-robin in launch order; give each XCD a
// contiguous range of vectors instead, so that the column passes of a 2D transform (one
// column per workgroup, elements n1 apart) share their cache lines within one XCD's L2.
// A bijection on [0, gridDim.x): the first 8 floor(g / 8) ids are permuted, the tail kept.
__device__ __forceinline__ int64_t xcd_vector(unsigned w, unsigned g) {
    const unsigned per = g / 8;
    if (w >= 8 * per) return w;
    return static_cast<int64_t>(w % 8) * per + w / 8;
}

__device__ __forceinline__ bool is_comparator(int kind) { return kind == HT_KIND_P || kind == HT_KIND_R; }
__device__ __forceinline__ bool is_fourier(int kind) { return kind == HT_KIND_F || kind == HT_KIND_P || kind == HT_KIND_F3; }
// the kind whose boundary columns and core a kind uses (F3 is T_F plus a rank-2 change)
__device__ __forceinline__ int base_kind(int kind) { return kind == HT_KIND_F3 ? HT_KIND_F : kind; }

// The core's tables for the element type C (float64 or float32 copies).
template <class C>
__device__ __forceinline__ const ChirpT<C>& core_of(const Axis& ax, bool analysis);
template <>
__device__ __forceinline__ const Chirp& core_of<double2>(const Axis& ax, bool analysis) {
    return analysis ? ax.ana : ax.syn;
}
template <>
__device__ __forceinline__ const Chirp32& core_of<float2>(const Axis& ax, bool analysis) {
    return analysis ? ax.ana32 : ax.syn32;
}

template <int LOGP, int S, class C>
__global__ __launch_bounds__(fft_block_for(LOGP)) void k_inverse(Axis ax, View in, View out,
                                                             const C* __restrict__ tw) {
    constexpr int P = 1 << LOGP;
    constexpr int SL = fft_slots_for(LOGP);
    constexpr int BLOCK = fft_block_for(LOGP);
    __shared__ C lds[P];
    __shared__ double2 corr[2];
    const int tid = threadIdx.x;
    const int64_t b = xcd_vector(blockIdx.x, gridDim.x);
    const int n = ax.n, N = ax.N;
    const int64_t ib = vbase(in, b), ob = vbase(out, b);
    const bool cmp = is_comparator(ax.kind);
    const int off = cmp ? 0 : 1;  // position of core entry 0 in the vectors
    const int kb = base_kind(ax.kind);

    // boundary coefficients (float64 closed form)
    const double2 y0 = vload(in, ib, 0), y1 = vload(in, ib, 1);
    const double2 yN = vload(in, ib, n - 2), yL = vload(in, ib, n - 1);
    double2 x1 = make_double2(0.0, 0.0), xn = x1;
    if (cmp) {
    } else if (kb == HT_KIND_C || kb == HT_KIND_F) {
        const double2 r1 = kb == HT_KIND_C ? csub(y0, y1) : csub(y0, yN);
        const double2 r2 = kb == HT_KIND_C ? csub(yL, yN) : csub(yL, y1);
        x1 = make_double2(ax.minv[0] * r1.x + ax.minv[1] * r2.x, ax.minv[0] * r1.y + ax.minv[1] * r2.y);
        xn = make_double2(ax.minv[2] * r1.x + ax.minv[3] * r2.x, ax.minv[2] * r1.y + ax.minv[3] * r2.y);
    } else {
        const double inv = 1.0 / ax.q1;
        x1 = cscale(y0, inv);
        xn = cscale(yL, inv);
    }
    // interior correction r_j = y_{j+1} - q^_j x_1 - (J q^)_j x_n, then the core analysis
    auto in_fn = [&](int, int j) {
        double2 r = vload(in, ib, j + off);
        if (!cmp) {
            const double qa = ax.q[j + 1], qb = ax.q[N - j];
            r.x = r.x - qa * x1.x - qb * xn.x;
            r.y = r.y - qa * x1.y - qb * xn.y;
        }
        return r;
    };
    auto park = [&](int j, double2 y) { vstore(out, ob, j + off, y); };
    auto unpark = [&](int j) { return vload(out, ob, j + off); };
    const int mode = (is_fourier(ax.kind) && out.cplx) ? MODE_CPLX : ax.ana.mode;
    double2 acc[SL];
    chirp_core<LOGP, S, SL>(acc, core_of<C>(ax, true), mode, N, lds, tw, in_fn, park, unpark);
    if (ax.rank > 0) {  // DST family: x_mid -= U (E^T K)^{-1} E^T x_mid
        if (tid < ax.rank) corr[tid] = acc[0];
        __syncthreads();
        const double2 s0 = corr[0];
        const double2 s1 = ax.rank > 1 ? corr[1] : make_double2(0.0, 0.0);
        const double2 a0 = make_double2(ax.Gm[0] * s0.x + ax.Gm[1] * s1.x, ax.Gm[0] * s0.y + ax.Gm[1] * s1.y);
        const double2 a1 = make_double2(ax.Gm[2] * s0.x + ax.Gm[3] * s1.x, ax.Gm[2] * s0.y + ax.Gm[3] * s1.y);
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j < N) {
                const double u0 = ax.U[j];
                acc[k].x -= u0 * a0.x;
                acc[k].y -= u0 * a0.y;
                if (ax.rank > 1) {
                    const double u1 = ax.U[N + j];
                    acc[k].x -= u1 * a1.x;
                    acc[k].y -= u1 * a1.y;
                }
            }
        }
    }
    if (ax.kind == HT_KIND_F3) {  // rank-2 correction of the T_F inverse
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j == 1) corr[0] = acc[k];
            if (j == N - 1) corr[1] = acc[k];
        }
        __syncthreads();
        const double2 e0 = corr[0], e1 = corr[1];
        const double2 a0 = cadd(cmul(ax.f3vi[0], e0), cmul(ax.f3vi[1], e1));
        const double2 a1 = cadd(cmul(ax.f3vi[2], e0), cmul(ax.f3vi[3], e1));
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j < N) acc[k] = j == 1 ? a0 : (j == N - 1 ? a1 : csub(acc[k], cmul(ax.f3v[j + 1], a1)));
        }
        x1 = csub(x1, cmul(ax.f3v[0], a1));
        xn = csub(xn, cmul(ax.f3v[n - 1], a1));
    }
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        if (j < N) vstore(out, ob, j + off, acc[k]);
    }
    if (tid == 0 && !cmp) {
        vstore(out, ob, 0, x1);
        vstore(out, ob, n - 1, xn);
    }
}

template <int LOGP, int S, class C>
__global__ __launch_bounds__(fft_block_for(LOGP)) void k_forward(Axis ax, View in, View out,
                                                             const C* __restrict__ tw) {
    constexpr int P = 1 << LOGP;
    constexpr int SL = fft_slots_for(LOGP);
    constexpr int BLOCK = fft_block_for(LOGP);
    __shared__ C lds[P];
    const int tid = threadIdx.x;
    const int64_t b = xcd_vector(blockIdx.x, gridDim.x);
    const int n = ax.n, N = ax.N;
    const int64_t ib = vbase(in, b), ob = vbase(out, b);
    const bool cmp = is_comparator(ax.kind);
    const bool f3 = ax.kind == HT_KIND_F3;
    const int off = cmp ? 0 : 1;  // position of core entry 0 in the vectors
    const int kb = base_kind(ax.kind);

    const double2 zero = make_double2(0.0, 0.0);
    const double2 x1 = cmp ? zero : vload(in, ib, 0), xn = cmp ? zero : vload(in, ib, n - 1);
    const double2 beta0 = ax.rank > 0 ? vload(in, ib, 1) : zero;
    const double2 beta1 = ax.rank > 1 ? vload(in, ib, 2) : zero;
    // F3: the coefficients of the cosine and cubic columns (positions 2 and n-2)
    const double2 g0 = f3 ? vload(in, ib, 2) : zero, g1 = f3 ? vload(in, ib, n - 2) : zero;
    // the replaced (bubble, cosine, cubic) columns are added explicitly, not through the core
    auto in_fn = [&](int, int j) {
        const bool replaced = j < ax.rank || (f3 && (j == 1 || j == N - 1));
        return replaced ? zero : vload(in, ib, j + off);
    };
    auto park = [&](int j, double2 y) { vstore(out, ob, j + off, y); };
    auto unpark = [&](int j) { return vload(out, ob, j + off); };
    const int mode = (is_fourier(ax.kind) && out.cplx) ? MODE_CPLX : ax.syn.mode;
    double2 u[SL];
    chirp_core<LOGP, S, SL>(u, core_of<C>(ax, false), mode, N, lds, tw, in_fn, park, unpark);
#pragma unroll
    for (int k = 0; k < SL; ++k) {
        const int j = tid + k * BLOCK;
        if (j < N && cmp) {
            vstore(out, ob, j, u[k]);
        } else if (j < N) {
            const double qa = ax.q[j + 1], qb = ax.q[N - j];
            double2 y = make_double2(u[k].x + qa * x1.x + qb * xn.x, u[k].y + qa * x1.y + qb * xn.y);
            if (ax.rank > 0) {
                const double b0 = ax.bub[j];
                y.x += b0 * beta0.x;
                y.y += b0 * beta0.y;
                if (ax.rank > 1) {
                    const double b1 = ax.bub[N + j];
                    y.x += b1 * beta1.x;
                    y.y += b1 * beta1.y;
                }
            }
            if (f3) {
                const double c0 = ax.f3b[j + 1], c1 = ax.f3b[n + j + 1];
                y.x += c0 * g0.x + c1 * g1.x;
                y.y += c0 * g0.y + c1 * g1.y;
            }
            vstore(out, ob, j + off, y);
            // boundary rows: extension of the core columns to the two ghost grid points
            if (kb == HT_KIND_C || kb == HT_KIND_F) {
                const bool first_src = kb == HT_KIND_C ? (j == 0) : (j == N - 1);
                const bool last_src = kb == HT_KIND_C ? (j == N - 1) : (j == 0);
                double2 b0v = make_double2(ax.q1 * x1.x + u[k].x, ax.q1 * x1.y + u[k].y);
                double2 bnv = make_double2(ax.q1 * xn.x + u[k].x, ax.q1 * xn.y + u[k].y);
                if (f3) {
                    b0v.x += ax.f3b[0] * g0.x + ax.f3b[n] * g1.x;
                    b0v.y += ax.f3b[0] * g0.y + ax.f3b[n] * g1.y;
                    bnv.x += ax.f3b[n - 1] * g0.x + ax.f3b[2 * n - 1] * g1.x;
                    bnv.y += ax.f3b[n - 1] * g0.y + ax.f3b[2 * n - 1] * g1.y;
                }
                if (first_src) vstore(out, ob, 0, b0v);
                if (last_src) vstore(out, ob, n - 1, bnv);
            }
        }
    }
    if (tid == 0 && !cmp && !(kb == HT_KIND_C || kb == HT_KIND_F)) {
        vstore(out, ob, 0, cscale(x1, ax.q1));
        vstore(out, ob, n - 1, cscale(xn, ax.q1));
    }
}

template <int LOGP, class C>
static hipError_t launch_one(const Axis& ax, const C* tw, bool inverse, const View& in, const View& out,
                             int64_t count, hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>(count)), block(fft_block_for(LOGP));
    if constexpr (LOGP == MAX_LOGP) {  // split convolutions (M = 16384)
        if (ax.S == 2) {
            if (inverse)
                hipLaunchKernelGGL((k_inverse<LOGP, 2, C>), grid, block, 0, stream, ax, in, out, tw);
            else
                hipLaunchKernelGGL((k_forward<LOGP, 2, C>), grid, block, 0, stream, ax, in, out, tw);
            return hipGetLastError();
        }
    }
    {
        if (inverse)
            hipLaunchKernelGGL((k_inverse<LOGP, 1, C>), grid, block, 0, stream, ax, in, out, tw);
        else
            hipLaunchKernelGGL((k_forward<LOGP, 1, C>), grid, block, 0, stream, ax, in, out, tw);
    }
    return hipGetLastError();
}

template <int LOGP>
static hipError_t launch_prec(const Axis& ax, const double2* tw, bool inverse, const View& in, const View& out,
                              int64_t count, hipStream_t stream, bool f32) {
    if (f32) return launch_one<LOGP, float2>(ax, ax.tw32, inverse, in, out, count, stream);
    return launch_one<LOGP, double2>(ax, tw, inverse, in, out, count, stream);
}

ht_status launch_core(const Axis& ax, const double2* tw, bool inverse, const View& in,
                      const View& out, int64_t count, hipStream_t stream, bool f32) {
    if (count <= 0) return HT_OK;
    if (count > 0x7fffffffLL) return fail(HT_ERR_INVALID_ARG, "too many transforms in one call");
    hipError_t e;
    switch (ax.logP) {
        case 9: e = launch_prec<9>(ax, tw, inverse, in, out, count, stream, f32); break;
        case 10: e = launch_prec<10>(ax, tw, inverse, in, out, count, stream, f32); break;
        case 11: e = launch_prec<11>(ax, tw, inverse, in, out, count, stream, f32); break;
        case 12: e = launch_prec<12>(ax, tw, inverse, in, out, count, stream, f32); break;
        case 13: e = launch_prec<13>(ax, tw, inverse, in, out, count, stream, f32); break;
        default: return fail(HT_ERR_INVALID_ARG, "internal: FFT size out of range");
    }
    return check_hip(e, "transform launch");
}

}  // namespace ht

using namespace ht;

extern "C" ht_status ht_transform_inv(const ht_plan* plan, const double* signal, void* coeff,
                                      int64_t batch, hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_transform_inv: null plan");
    if (batch < 0) return fail(HT_ERR_INVALID_ARG, "ht_transform_inv: negative batch");
    if (batch == 0) return HT_OK;
    if (!signal || !coeff) return fail(HT_ERR_INVALID_ARG, "ht_transform_inv: null argument");
    if (plan->gemm) {
        if (signal == coeff) return fail(HT_ERR_INVALID_ARG, "ht_transform_inv: signal and coeff must not overlap");
        return gemm_transform(plan, true, signal, static_cast<double*>(coeff), batch, stream);
    }
    const int cp = plan->cplx;
    if (plan->ndim == 1) {
        const Axis& a = plan->ax[0];
        View in{const_cast<double*>(signal), 0, a.n, 1, batch, 0};
        View out{coeff, 0, a.n, 1, batch, cp};
        return launch_core(a, plan->tw, true, in, out, batch, stream, plan->f32 != 0);
    }
    if (batch > plan->max_batch) return fail(HT_ERR_INVALID_ARG, "ht_transform_inv: batch exceeds the plan's max_batch");
    const Axis& a0 = plan->ax[0];
    const Axis& a1 = plan->ax[1];
    const int64_t img = static_cast<int64_t>(a0.n) * a1.n;
    // axis 1: every row, signal -> workspace
    View r_in{const_cast<double*>(signal), 0, a1.n, 1, batch * a0.n, 0};
    View r_out{plan->work, 0, a1.n, 1, batch * a0.n, cp};
    ht_status st = launch_core(a1, plan->tw, true, r_in, r_out, batch * a0.n, stream, plan->f32 != 0);
    if (st != HT_OK) return st;
    // axis 0: every column, workspace -> coeff
    View c_in{plan->work, img, 1, a1.n, a1.n, cp};
    View c_out{coeff, img, 1, a1.n, a1.n, cp};
    return launch_core(a0, plan->tw, true, c_in, c_out, batch * a1.n, stream, plan->f32 != 0);
}

extern "C" ht_status ht_transform_fwd(const ht_plan* plan, const void* coeff, double* signal,
                                      int64_t batch, hipStream_t stream) {
    if (!plan) return fail(HT_ERR_INVALID_ARG, "ht_transform_fwd: null plan");
    if (batch < 0) return fail(HT_ERR_INVALID_ARG, "ht_transform_fwd: negative batch");
    if (batch == 0) return HT_OK;
    if (!signal || !coeff) return fail(HT_ERR_INVALID_ARG, "ht_transform_fwd: null argument");
    if (plan->gemm) {
        if (signal == coeff) return fail(HT_ERR_INVALID_ARG, "ht_transform_fwd: signal and coeff must not overlap");
        return gemm_transform(plan, false, static_cast<const double*>(coeff), signal, batch, stream);
    }
    const int cp = plan->cplx;
    if (plan->ndim == 1) {
        const Axis& a = plan->ax[0];
        View in{const_cast<void*>(coeff), 0, a.n, 1, batch, cp};
        View out{signal, 0, a.n, 1, batch, 0};
        return launch_core(a, plan->tw, false, in, out, batch, stream, plan->f32 != 0);
    }
    if (batch > plan->max_batch) return fail(HT_ERR_INVALID_ARG, "ht_transform_fwd: batch exceeds the plan's max_batch");
    const Axis& a0 = plan->ax[0];
    const Axis& a1 = plan->ax[1];
    const int64_t img = static_cast<int64_t>(a0.n) * a1.n;
    // axis 0: every column, coeff -> workspace (complex for F, real otherwise)
    View c_in{const_cast<void*>(coeff), img, 1, a1.n, a1.n, cp};
    View c_out{plan->work, img, 1, a1.n, a1.n, cp};
    ht_status st = launch_core(a0, plan->tw, false, c_in, c_out, batch * a1.n, stream, plan->f32 != 0);
    if (st != HT_OK) return st;
    // axis 1: every row, workspace -> signal (real part)
    View r_in{plan->work, 0, a1.n, 1, batch * a0.n, cp};
    View r_out{signal, 0, a1.n, 1, batch * a0.n, 0};
    return launch_core(a1, plan->tw, false, r_in, r_out, batch * a0.n, stream, plan->f32 != 0);
}
