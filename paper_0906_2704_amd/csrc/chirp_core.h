// Chirp-z evaluation of the trigonometric cores on the LDS FFT (device code).
//
// Every core (DST-I, DCT-II, DCT-III, DFT, inverse DFT of order N) is written as
//   Y_k = post_k * sum_j b_{k-j} (pre_j x_j),  k < N,
// a circular convolution of length M >= 2N - 1 done as FFT, pointwise product with the
// precomputed spectrum B = FFT_M(b) / M, inverse FFT.  M = S * P with P = 2^LOGP held in
// LDS; for S = 2 (M = 2P > 8192) the length-M transforms are split by even / odd
// frequency into two length-P halves (the input occupies the first P points only, and
// only the first N <= P outputs are kept).  The first half's finished values are parked
// by the caller (in its output buffer) and added back after the second half, so only
// the eight slot values are live across an FFT.
#pragma once

#include "fft_lds.h"

namespace ht {

__device__ __forceinline__ double2 select_out(double2 y, int mode) {
    if (mode == MODE_RE) return make_double2(y.x, 0.0);
    if (mode == MODE_IM) return make_double2(y.y, 0.0);
    return y;
}

// in(k, j) returns x_j for the slot k holding j = tid + k * BLOCK < N; the result goes to
// out[k].  OutT = double2 keeps the complex result (selected by `mode`), OutT = double the
// real or imaginary part only.  The workgroup has 2^LOGP / SL threads.
template <int LOGP, int S, int SL, bool FRESH = false, class OutT, class In, class Park, class Unpark, class C>
__device__ __forceinline__ void chirp_core(OutT (&out)[SL], const ChirpT<C>& ch, int mode, int N, C* lds,
                                           const C* __restrict__ tw, In in, Park park, Unpark unpark) {
    constexpr int BLOCK = (1 << LOGP) / SL;
    constexpr bool REAL = sizeof(OutT) == sizeof(double);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        // FRESH (persistent kernels): a fresh thread index per phase, so that no lane offset
        // is held across the FFTs
        int tid = FRESH ? local_tid() : static_cast<int>(threadIdx.x);
        C v[SL];
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j < N) {
                const double2 x = in(k, j);  // float64 input, rounded to the core's type
                v[k] = cmul(cmake<C>(x.x, x.y), tload(ch.pre, j));
            } else {
                v[k] = cmake<C>(0.0, 0.0);
            }
            if (s == 1) v[k] = cmul(v[k], tload(tw, j * (TWN >> (LOGP + 1))));  // exp(-2 pi i j / M)
        }
        __builtin_amdgcn_sched_barrier(0);
        fft_slots<LOGP, -1, SL, FRESH>(v, lds, tw);
        __builtin_amdgcn_sched_barrier(0);
        if (FRESH) tid = local_tid();
#pragma unroll
        for (int k = 0; k < SL; ++k) v[k] = cmul(v[k], tload(ch.B, static_cast<unsigned>(s * (1 << LOGP) + tid + k * BLOCK)));
        __builtin_amdgcn_sched_barrier(0);
        fft_slots<LOGP, 1, SL, FRESH>(v, lds, tw);
        __builtin_amdgcn_sched_barrier(0);
        if (FRESH) tid = local_tid();
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int j = tid + k * BLOCK;
            if (j < N) {
                C c = v[k];
                if (s == 1) c = cmulc(c, tload(tw, j * (TWN >> (LOGP + 1))));  // exp(+2 pi i j / M)
                const C yc = cmul(c, tload(ch.post, j));
                const double2 y2 = make_double2(yc.x, yc.y);
                OutT y;
                if constexpr (REAL)
                    y = mode == MODE_IM ? y2.y : y2.x;
                else
                    y = select_out(y2, mode);
                if (S == 2 && s == 0)
                    park(j, y);
                else if (S == 2)
                    out[k] = y + unpark(j);
                else
                    out[k] = y;
            }
        }
    }
}

}  // namespace ht
