// Workgroup-wide complex FFT (float64, or float32 for the reduced-precision core) of a
// power-of-two length P held in LDS.
//
// Layout: the workgroup has BLOCK = P / SLOTS threads (SLOTS = 8 or 16); thread t owns
// the "slots" t + s * BLOCK, s = 0..SLOTS-1, held in registers between passes.  Each pass is a Stockham
// autosort step of radix 8 (a final radix 2 or 4 pass covers the remaining bits): every
// pass reads the thread's own slots, applies the pass twiddles, does a radix-R DFT in
// registers and scatters the results to their positions for the next pass.  The first
// pass therefore takes its input straight from registers and the last pass leaves its
// output in registers, already in natural order, so a full FFT costs (passes - 1) LDS
// round trips.  Twiddles come from the global table tw[m] = exp(-2 pi i m / TWN).
//
// DIR = -1: X_k = sum_j x_j e^{-2 pi i jk/P};  DIR = +1: unnormalised inverse.
#pragma once

#include <hip/hip_runtime.h>

#include "ht_internal.h"

namespace ht {

// Complex arithmetic for float64 (double2) and float32 (float2) elements.
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

template <class C>
__device__ __forceinline__ C cmake(double re, double im);
template <>
__device__ __forceinline__ double2 cmake<double2>(double re, double im) { return make_double2(re, im); }
template <>
__device__ __forceinline__ float2 cmake<float2>(double re, double im) {
    return make_float2(static_cast<float>(re), static_cast<float>(im));
}

// Table read with a 32-bit unsigned element index through a global-memory pointer: the
// tables are device allocations whose addresses reach the kernels inside records, so the
// compiler cannot infer their address space and would emit flat loads (64-bit address per
// lane, counted against the LDS wait counter too).  As a global pointer with a uniform
// base the load is scalar base + 32-bit lane offset.
typedef double gdbl2_t __attribute__((ext_vector_type(2)));
typedef float gflt2_t __attribute__((ext_vector_type(2)));
#define HT_GLOBAL __attribute__((address_space(1)))
// element i >= 0 of a float64 device table
__device__ __forceinline__ double dtab(const double* __restrict__ base, int i) {
    return *(const HT_GLOBAL double*)((const HT_GLOBAL char*)base + (static_cast<unsigned>(i) << 3));
}
__device__ __forceinline__ double2 tload(const double2* __restrict__ base, unsigned idx) {
    const gdbl2_t v = *(const HT_GLOBAL gdbl2_t*)((const HT_GLOBAL char*)base + (idx << 4));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 tload(const float2* __restrict__ base, unsigned idx) {
    const gflt2_t v = *(const HT_GLOBAL gflt2_t*)((const HT_GLOBAL char*)base + (idx << 3));
    return make_float2(v.x, v.y);
}

// threadIdx.x as a value the compiler cannot equate with other reads of it.  Addresses
// and table offsets derived from it are then computed where they are used: otherwise they
// are hoisted out of the persistent kernels' queue loops, held across a whole signal and,
// under a register cap, spilled and reloaded before every use.
__device__ __forceinline__ int local_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// multiply by exp(DIR * i pi / 2): -i for the forward direction, +i for the inverse
template <int DIR, class C>
__device__ __forceinline__ C rot90(C a) {
    C r;
    if (DIR < 0) {
        r.x = a.y;
        r.y = -a.x;
    } else {
        r.x = -a.y;
        r.y = a.x;
    }
    return r;
}

template <int DIR, class C>
__device__ __forceinline__ void dft2(C& a, C& b) {
    C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR, class C>
__device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
    C a = cadd(x0, x2), b = csub(x0, x2);
    C c = cadd(x1, x3), d = rot90<DIR>(csub(x1, x3));
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, d);
    x3 = csub(b, d);
}

// multiply by exp(DIR * i pi / 4)
template <int DIR, class C>
__device__ __forceinline__ C rot45(C a) {
    using R = decltype(a.x);
    const R h = static_cast<R>(0.70710678118654752440);  // 1 / sqrt(2)
    C r;
    if (DIR < 0) {
        r.x = (a.x + a.y) * h;
        r.y = (a.y - a.x) * h;
    } else {
        r.x = (a.x - a.y) * h;
        r.y = (a.x + a.y) * h;
    }
    return r;
}

template <int DIR, class C>
__device__ __forceinline__ void dft8(C (&u)[8]) {
    C e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
    C o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = rot45<DIR>(o1);
    o2 = rot90<DIR>(o2);
    o3 = rot90<DIR>(rot45<DIR>(o3));
    u[0] = cadd(e0, o0); u[4] = csub(e0, o0);
    u[1] = cadd(e1, o1); u[5] = csub(e1, o1);
    u[2] = cadd(e2, o2); u[6] = csub(e2, o2);
    u[3] = cadd(e3, o3); u[7] = csub(e3, o3);
}

template <int R, int DIR, class C>
__device__ __forceinline__ void dftR(C (&u)[R]) {
    if constexpr (R == 2)
        dft2<DIR>(u[0], u[1]);
    else if constexpr (R == 4)
        dft4<DIR>(u[0], u[1], u[2], u[3]);
    else
        dft8<DIR>(u);
}

// Threads per workgroup for an LDS FFT of 2^LOGP points: 8 points per thread up to 4096
// points, 16 per thread for 8192 (512 threads, so that each wave may use 256 VGPRs).
__host__ __device__ constexpr int fft_slots_for(int logp) { return logp >= 13 ? 16 : 8; }
__host__ __device__ constexpr int fft_block_for(int logp) { return (1 << logp) / fft_slots_for(logp); }

// One Stockham pass of radix R with Ns = product of the radices of earlier passes (Ns = 1:
// no twiddles).  LAST: the outputs stay in the thread's own slots.
//
// FIRST (the Ns = 1 pass, radix 8): thread t writes its eight outputs to the contiguous
// elements 8t .. 8t+7, so in a plain layout the lanes of one store instruction are 128
// bytes apart and meet in the same LDS banks.  This pass stores element e at
// e ^ ((e >> 3) & 7) instead -- a permutation inside each aligned group of eight elements
// that puts the eight lanes of a 128-byte row in eight different 16-byte bank groups --
// and its read-back applies the same permutation (BLOCK is a multiple of 64, so every
// read element tid + s * BLOCK has (e >> 3) & 7 = (tid >> 3) & 7).
//
// FRESH: the pass takes its own copy of the thread index (local_tid) -- for the persistent
// kernels, whose loop-invariant offsets would otherwise be held (and spilled) across signals.
template <int R, int DIR, int BLOCK, int SLOTS, bool LAST, class C, bool FIRST = false, bool FRESH = false>
__device__ __forceinline__ void stockham_pass(C (&v)[SLOTS], C* lds, const C* __restrict__ tw, int Ns) {
    static_assert(!FIRST || (R == 8 && !LAST && BLOCK % 64 == 0), "permuted first pass: radix 8, 64-aligned");
    constexpr int NB = SLOTS / R;  // butterflies per thread
    const int tid = FRESH ? local_tid() : static_cast<int>(threadIdx.x);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int t = tid + c * BLOCK;
        C u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[c + r * NB];
        const int k = t & (Ns - 1);
        if (Ns > 1) {
            // w^r, r = 1..R-1, w = exp(-2 pi i k / (Ns R)): powers 1, 2, 4 from the table,
            // the others as products of two of them (a few ulp, far below the tolerance)
            const unsigned step = static_cast<unsigned>((TWN / R) / Ns * k);
            const C w1 = tload(tw, step);
            if constexpr (R == 2) {
                u[1] = DIR < 0 ? cmul(u[1], w1) : cmulc(u[1], w1);
            } else {
                const C w2 = tload(tw, 2u * step);
                u[1] = DIR < 0 ? cmul(u[1], w1) : cmulc(u[1], w1);
                u[2] = DIR < 0 ? cmul(u[2], w2) : cmulc(u[2], w2);
                const C w3 = cmul(w1, w2);
                u[3] = DIR < 0 ? cmul(u[3], w3) : cmulc(u[3], w3);
                if constexpr (R == 8) {
                    const C w4 = tload(tw, 4u * step);
                    u[4] = DIR < 0 ? cmul(u[4], w4) : cmulc(u[4], w4);
                    const C w5 = cmul(w1, w4);
                    u[5] = DIR < 0 ? cmul(u[5], w5) : cmulc(u[5], w5);
                    const C w6 = cmul(w2, w4);
                    u[6] = DIR < 0 ? cmul(u[6], w6) : cmulc(u[6], w6);
                    const C w7 = cmul(w3, w4);
                    u[7] = DIR < 0 ? cmul(u[7], w7) : cmulc(u[7], w7);
                }
            }
        }
        dftR<R, DIR>(u);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[c + r * NB] = u[r];
        } else if constexpr (FIRST) {
            const int sw = t & 7;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[t * R + (r ^ sw)] = u[r];
        } else {
            const int base = (t - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[base + r * Ns] = u[r];
        }
    }
    if (!LAST) {
        __syncthreads();
        const int rd = FIRST ? tid ^ ((tid >> 3) & 7) : tid;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) v[s] = lds[rd + s * BLOCK];
        __syncthreads();
    }
}


// Full FFT of length P = 2^LOGP on the slots v (natural order in, natural order out),
// SL points per thread, P / SL threads.  The radix-8 passes run as a loop that is not
// unrolled, so only one pass's addresses are live at a time.
template <int LOGP, int DIR, int SL = fft_slots_for(LOGP), bool FRESH = false, class C>
__device__ __forceinline__ void fft_slots(C (&v)[SL], C* lds, const C* __restrict__ tw) {
    constexpr int BL = (1 << LOGP) / SL;
    static_assert(SL == 8 || SL == 16, "8 or 16 points per thread");
    static_assert(LOGP >= 9 && LOGP <= 13, "FFT length out of range");
    constexpr int NR8 = LOGP / 3;
    constexpr int REM = LOGP % 3;
    constexpr int NMID = REM ? NR8 : NR8 - 1;  // radix-8 passes that go through LDS
    static_assert(NMID >= 1, "the first pass goes through LDS");
    stockham_pass<8, DIR, BL, SL, false, C, true, FRESH>(v, lds, tw, 1);
    int Ns = 8;
#pragma unroll 1
    for (int p = 1; p < NMID; ++p) {
        stockham_pass<8, DIR, BL, SL, false, C, false, FRESH>(v, lds, tw, Ns);
        Ns *= 8;
    }
    if constexpr (REM == 0)
        stockham_pass<8, DIR, BL, SL, true, C, false, FRESH>(v, lds, tw, Ns);
    else
        stockham_pass<(1 << REM), DIR, BL, SL, true, C, false, FRESH>(v, lds, tw, Ns);
}

}  // namespace ht
