// Split-precision matrix-core form of the real transform cores (DCT-II/III for T_C, DST-I
// for the antireflective transform, DST-I with replaced columns for the DST family).
//
// Every core pass is one GEMM over all vectors of a call.  With A_inv (N x N, the inverse
// of the interior core block, Theorem th:inv) and A_fwd (n x N, the core columns of T_X on
// the whole grid, eqs. ART and Tc) dense float64 matrices built once per plan from exactly
// reduced angles, and the float64 vectors c = A_inv q^, c' = A_inv J q^, b = q - A_fwd c,
// b' = J q - A_fwd c', the two directions are
//
//   inverse  [x_1, x_n] from the 2x2 boundary system, x_mid = A_inv y_mid - x_1 c - x_n c'
//   forward  v = x_mid + x_1 c + x_n c',               y = A_fwd v + x_1 b + x_n b'
//
// (the same maps as "correct, then transform": A_inv (y_mid - q^ x_1 - J q^ x_n) and
// A_fwd x_mid + q x_1 + J q x_n).  The GEMM only ever sees y_mid or v, which have the size
// of the data, while x_1, x_n and x_mid can be larger by the condition number of T_X
// (about 6e4 for T_C at n = 2048) and cancel in the forward transform; the rank-2 terms
// that carry them are float64.
//
// Both GEMM operands are split into a high and a low 16-bit part (bfloat16 or float16),
// x = x_hi + x_lo, and the product is accumulated in float32 on the matrix cores as
// A_hi B_hi + A_hi B_lo + A_lo B_hi (v_mfma_f32_16x16x32_{bf16,f16}).  The dropped
// A_lo B_lo term and the representation error x - x_hi - x_lo are both of order u^2
// relative, u the 16-bit unit roundoff.  For float16 every operand row is scaled by a
// power of two that puts its largest entry in [2^13, 2^14): nothing overflows and the low
// parts stay normal; the epilogue undoes both row scales.
//
// 2D tensor products (Section 6) run rows first (axis 1) and then columns (axis 0); the
// column pass transposes through LDS in its operand preparation so that both GEMM
// operands are always stored row-major with the contraction index contiguous.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "ht_internal.h"
#include "plan_build.h"

namespace ht {

constexpr int GT_M = 256;  // GEMM block tile (rows of A and rows of B)
constexpr int GEMM_THREADS = 512;  // eight waves per GEMM workgroup
constexpr int GT_K = 32;   // contraction tile (one v_mfma_f32_16x16x32 step)
constexpr int K_ALIGN = 64;
// LDS rows of GT_K elements (64 bytes, four 16-byte chunks), chunk c of row r stored at
// chunk c ^ lds_swz(r).  A 16-byte access by 8 consecutive lanes covers 128 bytes and by 16
// consecutive lanes 256 bytes; both the fragment reads (16 consecutive rows, one chunk) and
// the tile stores (4 consecutive rows, all chunks) then touch distinct banks whether the
// LDS serves 32 or 64 four-byte banks per cycle.
constexpr int LDS_ROW = GT_K;
__device__ __forceinline__ int lds_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// One split matrix: rows padded to a multiple of GT_M, contraction padded with zeros to Kp.
struct GemmMat {
    const uint16_t* hi = nullptr;
    const uint16_t* lo = nullptr;
    const float* scale = nullptr;  // per row: 2^-e (1 for bfloat16)
    int rows = 0, rows_p = 0, Kp = 0;
};

// float64 rank-2 terms of one axis (see the top of this file)
struct GemmVecs {
    const double* c = nullptr;    // [N] A_inv q^
    const double* cj = nullptr;   // [N] A_inv J q^
    const double* nc = nullptr;   // [N] -c
    const double* ncj = nullptr;  // [N] -c'
    const double* b = nullptr;    // [n] q - A_fwd c
    const double* bj = nullptr;   // [n] J q - A_fwd c'
    const double* u0 = nullptr;   // [n] e_1 - c (c placed on the interior)
    const double* u1 = nullptr;   // [n] e_n - c'
};

struct GemmState {
    int prec = 0;
    GemmMat inv[2], fwd[2];
    GemmVecs vec[2];
    void* arena = nullptr;
    uint16_t* vhi = nullptr;   // vector operand workspace (high parts)
    uint16_t* vlo = nullptr;   // (low parts)
    float* vscale = nullptr;   // per vector row
    int64_t vcap = 0, vrows = 0;
    double* side_r = nullptr;  // 2D: [batch][n0][2] boundary coefficients of the rows
    double* side_z = nullptr;  // 2D: [batch][n0][2] their axis-0 transforms
    double* side_x = nullptr;  // 2D: [batch][2][n1] boundary values of the column pass
};

static int round_up(int x, int m) { return (x + m - 1) / m * m; }
static int64_t round_up64(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------------ 16-bit conversions

static __host__ __device__ __forceinline__ uint16_t bf16_bits_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

static __host__ __device__ __forceinline__ float bf16_value(uint16_t h) {
    const uint32_t u = static_cast<uint32_t>(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

static __host__ __device__ __forceinline__ uint16_t f16_bits_rne(float x) {
    const _Float16 h = static_cast<_Float16>(x);
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

static __host__ __device__ __forceinline__ float f16_value(uint16_t u) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return static_cast<float>(h);
}

// x (already scaled) -> high and low 16-bit parts
template <int PREC>
static __host__ __device__ __forceinline__ void split16(double x, uint16_t& hi, uint16_t& lo) {
    if constexpr (PREC == HT_PRECISION_BF16X3) {
        hi = bf16_bits_rne(static_cast<float>(x));
        lo = bf16_bits_rne(static_cast<float>(x - static_cast<double>(bf16_value(hi))));
    } else {
        hi = f16_bits_rne(static_cast<float>(x));
        lo = f16_bits_rne(static_cast<float>(x - static_cast<double>(f16_value(hi))));
    }
}

// Power-of-two row scale for float16 (largest entry into [2^13, 2^14)); 1 for bfloat16.
template <int PREC>
static __host__ __device__ __forceinline__ double row_scale_exp(double mx, int* e_out) {
    int e = 0;
    if constexpr (PREC == HT_PRECISION_F16X3) {
        if (mx > 0.0 && mx < 1e300) {
            int ex;
            (void)frexp(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
            e = 14 - ex;
        }
    }
    *e_out = e;
    return ldexp(1.0, e);
}

// --------------------------------------------------------------- operand preparation

// Boundary coefficients of one real vector (closed form of the capacitance system).
__device__ __forceinline__ void boundary_solve(const Axis& ax, double y0, double y1, double yN, double yL,
                                               double& x1, double& xn) {
    if (ax.kind == HT_KIND_C) {
        const double r1 = y0 - y1, r2 = yL - yN;
        x1 = ax.minv[0] * r1 + ax.minv[1] * r2;
        xn = ax.minv[2] * r1 + ax.minv[3] * r2;
    } else {
        const double inv = 1.0 / ax.q1;
        x1 = y0 * inv;
        xn = yL * inv;
    }
}

// Operand preparation modes.
enum PrepMode {
    ROW_INV = 0,  // boundary solve of the vector; operand y_mid
    ROW_FWD = 1,  // operand v = x_mid + x_1 c + x_n c' of a coefficient vector
    ROW_RAW = 2,  // operand = the first N entries as they are
    COL_INV = 3,  // column of an image: boundary solve; operand y_mid
    COL_FWD = 4   // column k of H = X V1^T (axis-1 forms of the rows of a coefficient
                  // image X), then its axis-0 form v as for ROW_FWD
};

// The cross rank-2 term of the 2D passes: zc[(z zc_img + row) 2 + t] w_t[col].
struct Cross {
    const double* zc;  // null: no term
    int64_t zc_img;
    const double* w0;
    const double* w1;
};

__device__ __forceinline__ double cross_at(const Cross& x, int64_t zrow, int col) {
    if (!x.zc) return 0.0;
    const double* zr = x.zc + zrow * 2;
    return fma(zr[0], x.w0[col], zr[1] * x.w1[col]);
}

struct PrepRows {
    int mode;          // ROW_INV, ROW_FWD or ROW_RAW
    const double* in;  // vector v at in + v * in_ld
    int64_t in_ld;
    const double* c;   // ROW_FWD: v = x_mid + x_1 c + x_n c'
    const double* cj;
    double* bout;      // ROW_INV: x_1 at bout + v * bout_ld, x_n at + bout_last
    int64_t bout_ld, bout_last;
    double* zout;      // ROW_INV (2D): zero entries 0 and n-1 of zout + v * zout_ld
    int64_t zout_ld;
    uint16_t* hi;
    uint16_t* lo;
    float* scale;
    int Kp;
};

// One workgroup per vector: the operand row v (row scale, split into 16-bit parts).
template <int PREC>
__global__ __launch_bounds__(256) void k_prep_rows(Axis ax, PrepRows p) {
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int64_t v = blockIdx.x;
    const int n = ax.n, N = ax.N;
    const double* y = p.in + v * p.in_ld;
    double x1 = 0.0, xn = 0.0;
    if (p.mode == ROW_INV) {
        boundary_solve(ax, y[0], y[1], y[n - 2], y[n - 1], x1, xn);
    } else if (p.mode == ROW_FWD) {
        x1 = y[0];
        xn = y[n - 1];
    }
    const int off = p.mode == ROW_RAW ? 0 : 1;
    auto r_at = [&](int k) {
        double r = y[k + off];
        if (p.mode == ROW_FWD) r = fma(x1, p.c[k], fma(xn, p.cj[k], r));
        return r;
    };
    double s = 1.0;
    int e = 0;
    if constexpr (PREC == HT_PRECISION_F16X3) {
        double mx = 0.0;
        for (int k = tid; k < N; k += 256) mx = fmax(mx, fabs(r_at(k)));
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        s = row_scale_exp<PREC>(mx, &e);
    }
    uint16_t* hrow = p.hi + v * p.Kp;
    uint16_t* lrow = p.lo + v * p.Kp;
    for (int k0 = tid * 8; k0 < p.Kp; k0 += 256 * 8) {
        uint16_t h[8], l[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = k0 + t;
            split16<PREC>(k < N ? r_at(k) * s : 0.0, h[t], l[t]);
        }
        u32x4 hv, lv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            hv[t] = static_cast<uint32_t>(h[2 * t]) | (static_cast<uint32_t>(h[2 * t + 1]) << 16);
            lv[t] = static_cast<uint32_t>(l[2 * t]) | (static_cast<uint32_t>(l[2 * t + 1]) << 16);
        }
        *reinterpret_cast<u32x4*>(hrow + k0) = hv;
        *reinterpret_cast<u32x4*>(lrow + k0) = lv;
    }
    if (tid == 0) {
        p.scale[v] = static_cast<float>(ldexp(1.0, -e));
        if (p.mode == ROW_INV) {
            p.bout[v * p.bout_ld] = x1;
            p.bout[v * p.bout_ld + p.bout_last] = xn;
            if (p.zout) {
                p.zout[v * p.zout_ld] = 0.0;
                p.zout[v * p.zout_ld + n - 1] = 0.0;
            }
        }
    }
}

struct PrepCols {
    int mode;          // COL_INV or COL_FWD
    const double* in;  // image z: element (i, j) at in + z * img + i * ld + j
    int64_t img, ld;
    int ncols;         // columns of the pass (n1 for COL_INV, N1 for COL_FWD)
    const double* c;   // axis-0 c, c' (COL_FWD)
    const double* cj;
    const double* c1;  // axis-1 c, c' (COL_FWD: H = X V1^T)
    const double* cj1;
    int n1;            // row length of the images
    double* xbuf;      // x_1 of column j at xbuf + z * xb_img + j, x_n at + xb_last
    int64_t xb_img, xb_last;
    double* bout;      // COL_INV: rows 0 and n-1 of the output image, plus the cross term
    Cross cross;
    uint16_t* hi;
    uint16_t* lo;
    float* scale;
    int Kp;
    int64_t rows_per_img;  // operand row of column j of image z: z * rows_per_img + j
};

// 64 columns of one image per workgroup: boundary values per column, column scale, then
// the columns' operand vectors transposed through LDS into operand rows.
template <int PREC>
__global__ __launch_bounds__(256) void k_prep_cols(Axis ax, PrepCols p) {
    __shared__ double tile[64][65];
    __shared__ double sx1[64], sxn[64];
    __shared__ double smax[4][64];
    // ty (the wave) is uniform across a wave: the per-row terms (row[0], row[n1 - 1], c[k],
    // c'[k]) then go through scalar loads
    const int tid = threadIdx.x, tx = tid & 63, ty = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = ax.n, N = ax.N;
    const int64_t z = blockIdx.y;
    const int j = blockIdx.x * 64 + tx;
    const bool ok = j < p.ncols;
    const double* __restrict__ base = p.in + z * p.img;
    const double* __restrict__ c0 = p.c;
    const double* __restrict__ cj0 = p.cj;
    const double* __restrict__ c1 = p.c1;
    const double* __restrict__ cj1 = p.cj1;
    // COL_FWD: the column's axis-1 factors, loaded once
    const bool fwd = p.mode == COL_FWD;
    const double c1j = (fwd && ok) ? c1[j] : 0.0, cj1j = (fwd && ok) ? cj1[j] : 0.0;
    // entry i of this thread's column (ok threads only)
    auto col = [&](int i) {
        const double* __restrict__ row = base + i * p.ld;
        if (!fwd) return row[j];
        return fma(row[0], c1j, fma(row[p.n1 - 1], cj1j, row[1 + j]));
    };
    // blockIdx.z: a range of the contraction (the bfloat16 parts need no per-row scale, so
    // their rows are split over several blocks); the first range writes the per-column data
    const bool first = blockIdx.z == 0;
    if (ty == 0) {
        double x1 = 0.0, xn = 0.0;
        if (ok) {
            if (p.mode == COL_INV) {
                boundary_solve(ax, col(0), col(1), col(n - 2), col(n - 1), x1, xn);
                if (first) {
                    p.bout[z * p.img + j] = x1 + cross_at(p.cross, z * p.cross.zc_img, j);
                    p.bout[z * p.img + (n - 1) * p.ld + j] = xn + cross_at(p.cross, z * p.cross.zc_img + n - 1, j);
                }
            } else {
                x1 = col(0);
                xn = col(n - 1);
            }
            if (first) {
                p.xbuf[z * p.xb_img + j] = x1;
                p.xbuf[z * p.xb_img + p.xb_last + j] = xn;
            }
        }
        sx1[tx] = x1;
        sxn[tx] = xn;
    }
    __syncthreads();
    const double x1 = sx1[tx], xn = sxn[tx];
    auto r_at = [&](int k) {
        double r = col(k + 1);
        if (fwd) r = fma(x1, c0[k], fma(xn, cj0[k], r));
        return r;
    };
    double s = 1.0;
    int e = 0;
    if constexpr (PREC == HT_PRECISION_F16X3) {
        double mx = 0.0;
        if (ok)
            for (int k = ty; k < N; k += 4) mx = fmax(mx, fabs(r_at(k)));
        smax[ty][tx] = mx;
        __syncthreads();
        mx = fmax(fmax(smax[0][tx], smax[1][tx]), fmax(smax[2][tx], smax[3][tx]));
        s = row_scale_exp<PREC>(mx, &e);
    }
    if (ty == 0 && ok && first) p.scale[z * p.rows_per_img + j] = static_cast<float>(ldexp(1.0, -e));
    const int jj = tid >> 2, ks = (tid & 3) * 16;
    const int jw = blockIdx.x * 64 + jj;
    const int64_t orow = z * p.rows_per_img + jw;
    const int nchunk = p.Kp / 64, per = (nchunk + gridDim.z - 1) / gridDim.z;
    const int kbeg = blockIdx.z * per * 64;
    const int kend = (blockIdx.z + 1) * per * 64 < p.Kp ? (blockIdx.z + 1) * per * 64 : p.Kp;
    for (int k0 = kbeg; k0 < kend; k0 += 64) {
#pragma unroll 4
        for (int t = 0; t < 16; ++t) {
            const int kl = ty + 4 * t, k = k0 + kl;
            tile[kl][tx] = (ok && k < N) ? r_at(k) * s : 0.0;
        }
        __syncthreads();
        if (jw < p.ncols) {
            u32x4 hv[2], lv[2];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                uint16_t h0, l0, h1, l1;
                split16<PREC>(tile[ks + 2 * t][jj], h0, l0);
                split16<PREC>(tile[ks + 2 * t + 1][jj], h1, l1);
                hv[t >> 2][t & 3] = static_cast<uint32_t>(h0) | (static_cast<uint32_t>(h1) << 16);
                lv[t >> 2][t & 3] = static_cast<uint32_t>(l0) | (static_cast<uint32_t>(l1) << 16);
            }
            u32x4* hd = reinterpret_cast<u32x4*>(p.hi + orow * p.Kp + k0 + ks);
            u32x4* ld = reinterpret_cast<u32x4*>(p.lo + orow * p.Kp + k0 + ks);
            hd[0] = hv[0];
            hd[1] = hv[1];
            ld[0] = lv[0];
            ld[1] = lv[1];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------- the GEMM

struct GemmSplitArgs {
    const uint16_t* a_hi;
    const uint16_t* a_lo;
    const float* a_scale;
    int64_t a_img, a_simg;  // per-image offsets (elements, scale entries); 0 when shared
    const uint16_t* b_hi;
    const uint16_t* b_lo;
    const float* b_scale;
    int64_t b_img, b_simg;
    int Kp;
    int tiles_m, tiles_n, nz;
    int vec_is_a;  // which operand holds the vectors (its panels are visited in order)
    // epilogue: out[z o_img + m o_ldm + n + o_off] = D[m][n] sa_m sb_n
    //                      + e1[pos] x_1(vec) + e2[pos] x_n(vec)   (if e1)
    //                      + cross term of row z zc_img + m + zc_off, column n
    double* out;
    int64_t o_img, o_ldm, o_off;
    int m_lim, n_lim;
    const double* e1;  // float64 rank-2 terms along the output position (or null)
    const double* e2;
    Cross cross;
    int64_t zc_off;
    int pos_is_m;      // 1: position = m, vector = n; 0: the reverse
    const double* xb;  // x_1 at xb + z xb_img + vec xb_vs, x_n at + xb_last
    int64_t xb_img, xb_vs, xb_last;
};

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
    if constexpr (PREC == HT_PRECISION_BF16X3)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
}

// D = A B^T for A [rows_a][Kp], B [rows_b][Kp] (high and low parts), one 256 x 256 tile per
// workgroup of eight waves (4 x 2; 64 x 128 each, 4 x 8 MFMA tiles of 16 x 16).  Lane l
// supplies A row l % 16 and B row l % 16 with the contraction slice 8 (l / 16) + 0..7, and
// holds D rows 4 (l / 16) + 0..3 of column l % 16.  The operand slices of a contraction step
// go from global memory straight into LDS (global_load_lds_dwordx4: no register staging, no
// LDS store instructions), double-buffered: the loads of step k + 1 run under the fragment
// reads and matrix-core work of step k, one barrier per step.  The B fragments are read in
// two halves so that at most 16 fragments are live.
typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef const __attribute__((address_space(1))) void* global_void_ptr;

template <int PREC>
__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_split(GemmSplitArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t sm[2][4][GT_M][LDS_ROW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;

    // Tile order: consecutive ids go to different XCDs, so hand each XCD a contiguous
    // range of tiles; inside it, the panel of the vector operand changes slowest.
    const int per_z = g.tiles_m * g.tiles_n;
    const int nb = per_z * g.nz;
    int t = blockIdx.x;
    if ((nb & 7) == 0) t = (t & 7) * (nb >> 3) + (t >> 3);
    const int z = t / per_z;
    const int r = t - z * per_z;
    int tm, tn;
    if (g.vec_is_a) {
        tm = r / g.tiles_n;
        tn = r - tm * g.tiles_n;
    } else {
        tn = r / g.tiles_m;
        tm = r - tn * g.tiles_m;
    }

    const int Kp = g.Kp;
    const int64_t a_row0 = static_cast<int64_t>(tm) * GT_M, b_row0 = static_cast<int64_t>(tn) * GT_M;
    const uint16_t* src[4] = {g.a_hi + z * g.a_img + a_row0 * Kp, g.a_lo + z * g.a_img + a_row0 * Kp,
                              g.b_hi + z * g.b_img + b_row0 * Kp, g.b_lo + z * g.b_img + b_row0 * Kp};
    // Each operand slice (GT_M rows x 64 bytes) is 16 blocks of 1 KB (16 rows); wave w loads
    // blocks 2w and 2w + 1 of each, lane l filling the block's 16-byte slot l = (row l / 4,
    // stored chunk l % 4), i.e. reading logical chunk (l % 4) ^ lds_swz(row).
    static_assert(GEMM_THREADS / 64 * 2 * 16 == GT_M, "two 16-row blocks per wave and operand");
    int64_t goff[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int row = 16 * (2 * w + h) + (lane >> 2);
        goff[h] = static_cast<int64_t>(row) * Kp + 8 * ((lane & 3) ^ lds_swz(row));
    }
    auto dload = [&](int buf, int k0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                __builtin_amdgcn_global_load_lds((global_void_ptr)(src[a] + goff[h] + k0),
                                                 (lds_void_ptr)(&sm[buf][a][16 * (2 * w + h)][0]), 16, 0, 0);
        }
    };

    f32x4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nk = Kp / GT_K;
    dload(0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        // buffer buf ^ 1 was last read in step kt - 1, which ended with a barrier
        if (kt + 1 < nk) dload(buf ^ 1, (kt + 1) * GT_K);
        u32x4 ah[4], al[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ra = wm * 64 + i * 16 + fr;
            const int ca = fk ^ (8 * lds_swz(ra));
            ah[i] = *reinterpret_cast<const u32x4*>(&sm[buf][0][ra][ca]);
            al[i] = *reinterpret_cast<const u32x4*>(&sm[buf][1][ra][ca]);
        }
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {
            u32x4 bh[4], bl[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int rb = wn * 128 + (hb * 4 + j) * 16 + fr;
                const int cb = fk ^ (8 * lds_swz(rb));
                bh[j] = *reinterpret_cast<const u32x4*>(&sm[buf][2][rb][cb]);
                bl[j] = *reinterpret_cast<const u32x4*>(&sm[buf][3][rb][cb]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][hb * 4 + j] = mfma16<PREC>(ah[i], bh[j], acc[i][hb * 4 + j]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][hb * 4 + j] = mfma16<PREC>(ah[i], bl[j], acc[i][hb * 4 + j]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][hb * 4 + j] = mfma16<PREC>(al[i], bh[j], acc[i][hb * 4 + j]);
        }
        // this wave's loads of step kt + 1 have landed; the barrier makes every wave's visible
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }

    // epilogue (float64): for each 16-row group i, the row terms (scale, rank-2 and cross
    // factors of the lane's four rows) are loaded once, then every column tile j; the inputs
    // are read through restrict-qualified pointers so that the stores do not force reloads
    const float* __restrict__ sa = g.a_scale + z * g.a_simg;
    const float* __restrict__ sb = g.b_scale + z * g.b_simg;
    const double* __restrict__ e1 = g.e1;
    const double* __restrict__ e2 = g.e2;
    const double* __restrict__ xb = g.xb ? g.xb + z * g.xb_img : nullptr;
    const double* __restrict__ zc = g.cross.zc ? g.cross.zc + 2 * (z * g.cross.zc_img + g.zc_off) : nullptr;
    const double* __restrict__ w0 = g.cross.w0;
    const double* __restrict__ w1 = g.cross.w1;
    double* __restrict__ out = g.out + z * g.o_img + g.o_off;
    const bool pos_m = g.pos_is_m != 0;
    const int m0 = tm * GT_M + wm * 64 + (lane >> 4) * 4;
    const int n0 = tn * GT_M + wn * 128 + fr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double rs[4], r1[4], r2[4], c0[4], c1[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m0 + i * 16 + e;
            const bool ok = m < g.m_lim;
            rs[e] = ok ? static_cast<double>(sa[m]) : 0.0;
            // rank-2 factors that depend on the row: e1/e2 at position m, or x_1/x_n of vector m
            r1[e] = r2[e] = 0.0;
            if (ok && e1) {
                if (pos_m) {
                    r1[e] = e1[m];
                    r2[e] = e2[m];
                } else {
                    r1[e] = xb[static_cast<int64_t>(m) * g.xb_vs];
                    r2[e] = xb[static_cast<int64_t>(m) * g.xb_vs + g.xb_last];
                }
            }
            c0[e] = (ok && zc) ? zc[2 * m] : 0.0;
            c1[e] = (ok && zc) ? zc[2 * m + 1] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int n = n0 + j * 16;
            if (n >= g.n_lim) continue;
            const double sbn = static_cast<double>(sb[n]);
            double q1 = 0.0, q2 = 0.0;
            if (e1) {
                if (pos_m) {
                    q1 = xb[static_cast<int64_t>(n) * g.xb_vs];
                    q2 = xb[static_cast<int64_t>(n) * g.xb_vs + g.xb_last];
                } else {
                    q1 = e1[n];
                    q2 = e2[n];
                }
            }
            const double wa = zc ? w0[n] : 0.0, wb = zc ? w1[n] : 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + i * 16 + e;
                if (m >= g.m_lim) continue;
                double v = static_cast<double>(acc[i][j][e]) * (rs[e] * sbn);
                if (e1) v = fma(r1[e], q1, fma(r2[e], q2, v));
                if (zc) v += fma(c0[e], wa, c1[e] * wb);
                out[static_cast<int64_t>(m) * g.o_ldm + n] = v;
            }
        }
    }
}

// ---------------------------------------------------------------- host: the matrices

using ldbl = long double;
static const ldbl PI_LD = 3.141592653589793238462643383279502884L;

// c = A_inv q^, c' = A_inv J q^ (N), -c, -c', b = q - A_fwd c, b' = J q - A_fwd c' (n) and
// u0 = e_1 - c, u1 = e_n - c' on the whole grid (n), with long-double accumulation.
static void rank2_terms(const HostAxis& h, const std::vector<double>& Ainv, const std::vector<double>& Afwd,
                        std::vector<double>& out) {
    const int n = h.ax.n, N = h.ax.N;
    std::vector<ldbl> c(N, 0.0L), cj(N, 0.0L);
    for (int r = 0; r < N; ++r) {
        ldbl a = 0.0L, b = 0.0L;
        for (int k = 0; k < N; ++k) {
            const ldbl m = Ainv[static_cast<size_t>(r) * N + k];
            a += m * h.q[k + 1];
            b += m * h.q[N - k];
        }
        c[r] = a;
        cj[r] = b;
    }
    out.assign(4 * static_cast<size_t>(N) + 4 * static_cast<size_t>(n), 0.0);
    for (int r = 0; r < N; ++r) {
        out[r] = static_cast<double>(c[r]);
        out[N + r] = static_cast<double>(cj[r]);
        out[2 * N + r] = -static_cast<double>(c[r]);
        out[3 * N + r] = -static_cast<double>(cj[r]);
    }
    for (int i = 0; i < n; ++i) {
        ldbl a = h.q[i], b = h.q[n - 1 - i];
        for (int k = 0; k < N; ++k) {
            const ldbl m = Afwd[static_cast<size_t>(i) * N + k];
            a -= m * c[k];
            b -= m * cj[k];
        }
        out[4 * N + i] = static_cast<double>(a);
        out[4 * N + n + i] = static_cast<double>(b);
    }
    for (int i = 0; i < n; ++i) {
        const bool interior = i >= 1 && i <= N;
        out[4 * N + 2 * n + i] = (i == 0 ? 1.0 : 0.0) - (interior ? static_cast<double>(c[i - 1]) : 0.0);
        out[4 * N + 3 * n + i] = (i == n - 1 ? 1.0 : 0.0) - (interior ? static_cast<double>(cj[i - 1]) : 0.0);
    }
}

// Dense A_inv (N x N, row-major) and A_fwd (n x N) of one real axis.
static void dense_core(const HostAxis& h, std::vector<double>& Ainv, std::vector<double>& Afwd) {
    const Axis& a = h.ax;
    const int n = a.n, N = a.N;
    Ainv.assign(static_cast<size_t>(N) * N, 0.0);
    Afwd.assign(static_cast<size_t>(n) * N, 0.0);
    if (a.kind == HT_KIND_C) {
        // C[c][k] = w_c cos(pi c (2k+1) / (2N)); T_C core column c at grid point i (0-based,
        // x_i = (2i-1) pi / (2N)): w_c cos(pi c (2i-1) / (2N)).
        const int64_t P = 4LL * N;
        std::vector<double> ct(P);
        for (int64_t r = 0; r < P; ++r) ct[r] = static_cast<double>(cosl(PI_LD * static_cast<ldbl>(r) / (2.0L * N)));
        const double w0 = static_cast<double>(sqrtl(1.0L / N)), w1 = static_cast<double>(sqrtl(2.0L / N));
        for (int c = 0; c < N; ++c) {
            const double wc = c == 0 ? w0 : w1;
            for (int k = 0; k < N; ++k) Ainv[static_cast<size_t>(c) * N + k] = wc * ct[(static_cast<int64_t>(c) * (2 * k + 1)) % P];
            for (int i = 0; i < n; ++i) {
                int64_t m = (static_cast<int64_t>(c) * (2 * i - 1)) % P;
                if (m < 0) m += P;
                Afwd[static_cast<size_t>(i) * N + c] = wc * ct[m];
            }
        }
        return;
    }
    // sine core: Q[c][k] = sqrt(2/(N+1)) sin(pi (c+1)(k+1) / (N+1)); core column c of T at
    // grid point i (0-based) is sqrt(2/(N+1)) sin(pi (c+1) i / (N+1)), zero at both ends.
    const int64_t P = 2LL * (N + 1);
    std::vector<double> st(P);
    const ldbl w = sqrtl(2.0L / (N + 1));
    for (int64_t r = 0; r < P; ++r) st[r] = static_cast<double>(w * sinl(PI_LD * static_cast<ldbl>(r) / (N + 1)));
    std::vector<double> Q(static_cast<size_t>(N) * N);
    for (int c = 0; c < N; ++c)
        for (int k = 0; k < N; ++k) Q[static_cast<size_t>(c) * N + k] = st[(static_cast<int64_t>(c + 1) * (k + 1)) % P];
    for (int i = 1; i <= N; ++i)
        for (int c = 0; c < N; ++c) Afwd[static_cast<size_t>(i) * N + c] = Q[static_cast<size_t>(c) * N + (i - 1)];
    Ainv = Q;
    if (a.rank > 0) {
        // replaced columns: the bubbles (zero on the boundary rows)
        for (int c = 0; c < a.rank; ++c)
            for (int i = 1; i <= N; ++i) Afwd[static_cast<size_t>(i) * N + c] = h.bub[static_cast<size_t>(c) * N + (i - 1)];
        // A_inv = (I - U Gm E^T) Q: row j gets - sum_c U[c][j] (Gm Q[0..rank-1])[c]
        std::vector<double> GQ(static_cast<size_t>(a.rank) * N, 0.0);
        for (int c = 0; c < a.rank; ++c)
            for (int c2 = 0; c2 < a.rank; ++c2) {
                const double gm = a.Gm[c * 2 + c2];
                for (int k = 0; k < N; ++k) GQ[static_cast<size_t>(c) * N + k] += gm * Q[static_cast<size_t>(c2) * N + k];
            }
        for (int j = 0; j < N; ++j)
            for (int c = 0; c < a.rank; ++c) {
                const double u = h.U[static_cast<size_t>(c) * N + j];
                for (int k = 0; k < N; ++k) Ainv[static_cast<size_t>(j) * N + k] -= u * GQ[static_cast<size_t>(c) * N + k];
            }
    }
}

template <int PREC>
static void split_matrix(const std::vector<double>& A, int rows, int cols, int rows_p, int Kp, uint16_t* hi,
                         uint16_t* lo, float* scale) {
    std::memset(hi, 0, sizeof(uint16_t) * static_cast<size_t>(rows_p) * Kp);
    std::memset(lo, 0, sizeof(uint16_t) * static_cast<size_t>(rows_p) * Kp);
    for (int r = 0; r < rows_p; ++r) scale[r] = 1.0f;
    for (int r = 0; r < rows; ++r) {
        const double* x = &A[static_cast<size_t>(r) * cols];
        double mx = 0.0;
        for (int k = 0; k < cols; ++k) mx = std::fmax(mx, std::fabs(x[k]));
        int e = 0;
        const double s = row_scale_exp<PREC>(mx, &e);
        scale[r] = static_cast<float>(std::ldexp(1.0, -e));
        for (int k = 0; k < cols; ++k)
            split16<PREC>(x[k] * s, hi[static_cast<size_t>(r) * Kp + k], lo[static_cast<size_t>(r) * Kp + k]);
    }
}

void gemm_release(GemmState* g) {
    if (!g) return;
    if (g->arena) (void)hipFree(g->arena);
    if (g->vhi) (void)hipFree(g->vhi);
    if (g->vlo) (void)hipFree(g->vlo);
    if (g->vscale) (void)hipFree(g->vscale);
    if (g->side_r) (void)hipFree(g->side_r);
    if (g->side_z) (void)hipFree(g->side_z);
    if (g->side_x) (void)hipFree(g->side_x);
    delete g;
}

static ht_status build_gemm(const ht_plan* p, int prec, GemmState** out) {
    GemmState* g = new (std::nothrow) GemmState();
    if (!g) return fail(HT_ERR_OOM, "ht_plan_set_precision: host allocation failed");
    g->prec = prec;
    struct Host {
        std::vector<uint16_t> hi, lo;
        std::vector<float> sc;
        int rows, rows_p, Kp;
    };
    std::vector<Host> mats;
    std::vector<double> vecs[2];
    for (int a = 0; a < p->ndim; ++a) {
        HostAxis h;
        ht_status st = build_axis(p->ax[a].n, p->ax[a].kind, h);
        if (st != HT_OK) {
            delete g;
            return st;
        }
        std::vector<double> Ainv, Afwd;
        dense_core(h, Ainv, Afwd);
        rank2_terms(h, Ainv, Afwd, vecs[a]);
        const int n = h.ax.n, N = h.ax.N, Kp = round_up(N, K_ALIGN);
        for (int which = 0; which < 2; ++which) {
            Host m;
            m.rows = which == 0 ? N : n;
            m.rows_p = round_up(m.rows, GT_M);
            m.Kp = Kp;
            m.hi.resize(static_cast<size_t>(m.rows_p) * Kp);
            m.lo.resize(static_cast<size_t>(m.rows_p) * Kp);
            m.sc.resize(m.rows_p);
            const std::vector<double>& A = which == 0 ? Ainv : Afwd;
            if (prec == HT_PRECISION_BF16X3)
                split_matrix<HT_PRECISION_BF16X3>(A, m.rows, N, m.rows_p, Kp, m.hi.data(), m.lo.data(), m.sc.data());
            else
                split_matrix<HT_PRECISION_F16X3>(A, m.rows, N, m.rows_p, Kp, m.hi.data(), m.lo.data(), m.sc.data());
            mats.push_back(std::move(m));
        }
    }
    size_t bytes = 0;
    for (const Host& m : mats) bytes += 2 * m.hi.size() * sizeof(uint16_t) + round_up64(m.sc.size() * 4, 256);
    for (int a = 0; a < p->ndim; ++a) bytes += round_up64(vecs[a].size() * sizeof(double), 256);
    char* dev = nullptr;
    if (hipMalloc(&dev, bytes) != hipSuccess) {
        delete g;
        return fail(HT_ERR_OOM, "ht_plan_set_precision: matrix allocation failed");
    }
    g->arena = dev;
    size_t off = 0;
    for (size_t i = 0; i < mats.size(); ++i) {
        const Host& m = mats[i];
        GemmMat gm;
        const size_t eb = m.hi.size() * sizeof(uint16_t);
        hipError_t e1 = hipMemcpy(dev + off, m.hi.data(), eb, hipMemcpyHostToDevice);
        gm.hi = reinterpret_cast<const uint16_t*>(dev + off);
        off += eb;
        hipError_t e2 = hipMemcpy(dev + off, m.lo.data(), eb, hipMemcpyHostToDevice);
        gm.lo = reinterpret_cast<const uint16_t*>(dev + off);
        off += eb;
        hipError_t e3 = hipMemcpy(dev + off, m.sc.data(), m.sc.size() * 4, hipMemcpyHostToDevice);
        gm.scale = reinterpret_cast<const float*>(dev + off);
        off += round_up64(m.sc.size() * 4, 256);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            gemm_release(g);
            return fail(HT_ERR_HIP, "ht_plan_set_precision: matrix upload failed");
        }
        gm.rows = m.rows;
        gm.rows_p = m.rows_p;
        gm.Kp = m.Kp;
        if (i % 2 == 0)
            g->inv[i / 2] = gm;
        else
            g->fwd[i / 2] = gm;
    }
    for (int a = 0; a < p->ndim; ++a) {
        const int n = p->ax[a].n, N = p->ax[a].N;
        const size_t vb = vecs[a].size() * sizeof(double);
        if (hipMemcpy(dev + off, vecs[a].data(), vb, hipMemcpyHostToDevice) != hipSuccess) {
            gemm_release(g);
            return fail(HT_ERR_HIP, "ht_plan_set_precision: vector upload failed");
        }
        const double* d = reinterpret_cast<const double*>(dev + off);
        g->vec[a].c = d;
        g->vec[a].cj = d + N;
        g->vec[a].nc = d + 2 * N;
        g->vec[a].ncj = d + 3 * N;
        g->vec[a].b = d + 4 * N;
        g->vec[a].bj = d + 4 * N + n;
        g->vec[a].u0 = d + 4 * N + 2 * n;
        g->vec[a].u1 = d + 4 * N + 3 * n;
        off += round_up64(vb, 256);
    }
    // vector operand workspace, large enough for every pass
    const int64_t B = p->max_batch;
    int64_t rows = 0, cap = 0;
    auto need = [&](int64_t r, int Kp) {
        rows = r > rows ? r : rows;
        cap = r * Kp > cap ? r * Kp : cap;
    };
    if (p->ndim == 1) {
        need(round_up64(B, GT_M), g->inv[0].Kp);
    } else {
        const int n0 = p->ax[0].n, n1 = p->ax[1].n;
        need(round_up64(B * n0, GT_M), g->inv[1].Kp);       // rows of every image
        need(B * round_up64(n1, GT_M), g->inv[0].Kp);       // columns of every image
    }
    if (hipMalloc(&g->vhi, sizeof(uint16_t) * cap) != hipSuccess ||
        hipMalloc(&g->vlo, sizeof(uint16_t) * cap) != hipSuccess ||
        hipMalloc(&g->vscale, sizeof(float) * rows) != hipSuccess) {
        gemm_release(g);
        return fail(HT_ERR_OOM, "ht_plan_set_precision: workspace allocation failed");
    }
    if (hipMemset(g->vhi, 0, sizeof(uint16_t) * cap) != hipSuccess ||
        hipMemset(g->vlo, 0, sizeof(uint16_t) * cap) != hipSuccess ||
        hipMemset(g->vscale, 0, sizeof(float) * rows) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        gemm_release(g);
        return fail(HT_ERR_HIP, "ht_plan_set_precision: workspace initialisation failed");
    }
    if (p->ndim == 2) {
        const int64_t n0 = p->ax[0].n, n1 = p->ax[1].n;
        if (hipMalloc(&g->side_r, sizeof(double) * 2 * B * n0) != hipSuccess ||
            hipMalloc(&g->side_z, sizeof(double) * 2 * B * n0) != hipSuccess ||
            hipMalloc(&g->side_x, sizeof(double) * 2 * B * n1) != hipSuccess) {
            gemm_release(g);
            return fail(HT_ERR_OOM, "ht_plan_set_precision: workspace allocation failed");
        }
    }
    g->vcap = cap;
    g->vrows = rows;
    *out = g;
    return HT_OK;
}

// ---------------------------------------------------------------- host: the passes

template <int PREC>
static ht_status run_prep_rows(const Axis& ax, const PrepRows& pr, int64_t count, hipStream_t s) {
    if (count <= 0) return HT_OK;
    hipLaunchKernelGGL((k_prep_rows<PREC>), dim3(static_cast<unsigned>(count)), dim3(256), 0, s, ax, pr);
    return check_hip(hipGetLastError(), "operand preparation launch");
}

template <int PREC>
static ht_status run_prep_cols(const Axis& ax, const PrepCols& pc, int64_t batch, hipStream_t s) {
    // float16 parts carry a per-row scale from the whole row: one block per column tile
    const unsigned ksplit = PREC == HT_PRECISION_F16X3 ? 1u : static_cast<unsigned>(std::min(8, pc.Kp / 64));
    const dim3 grid(static_cast<unsigned>((pc.ncols + 63) / 64), static_cast<unsigned>(batch), ksplit);
    hipLaunchKernelGGL((k_prep_cols<PREC>), grid, dim3(256), 0, s, ax, pc);
    return check_hip(hipGetLastError(), "operand preparation launch");
}

template <int PREC>
static ht_status run_gemm(GemmSplitArgs g, hipStream_t s) {
    const int64_t nb = static_cast<int64_t>(g.tiles_m) * g.tiles_n * g.nz;
    if (nb <= 0) return HT_OK;
    if (nb > 0x7fffffffLL) return fail(HT_ERR_INVALID_ARG, "GEMM grid too large");
    hipLaunchKernelGGL((k_gemm_split<PREC>), dim3(static_cast<unsigned>(nb)), dim3(GEMM_THREADS), 0, s, g);
    return check_hip(hipGetLastError(), "GEMM launch");
}

// GEMM over `count` contiguous operand rows (A = vectors) against the matrix M (B).
static GemmSplitArgs rows_gemm(const GemmState* G, const GemmMat& M, int64_t count) {
    GemmSplitArgs g{};
    g.a_hi = G->vhi;
    g.a_lo = G->vlo;
    g.a_scale = G->vscale;
    g.b_hi = M.hi;
    g.b_lo = M.lo;
    g.b_scale = M.scale;
    g.Kp = M.Kp;
    g.tiles_m = static_cast<int>((count + GT_M - 1) / GT_M);
    g.tiles_n = M.rows_p / GT_M;
    g.nz = 1;
    g.vec_is_a = 1;
    g.m_lim = static_cast<int>(count);
    return g;
}

// GEMM of the matrix M (A) against `batch` blocks of rpi operand rows (B = vectors).
static GemmSplitArgs cols_gemm(const GemmState* G, const GemmMat& M, int64_t rpi, int64_t batch) {
    GemmSplitArgs g{};
    g.a_hi = M.hi;
    g.a_lo = M.lo;
    g.a_scale = M.scale;
    g.b_hi = G->vhi;
    g.b_lo = G->vlo;
    g.b_scale = G->vscale;
    g.b_img = rpi * M.Kp;
    g.b_simg = rpi;
    g.Kp = M.Kp;
    g.tiles_m = M.rows_p / GT_M;
    g.tiles_n = static_cast<int>(rpi / GT_M);
    g.nz = static_cast<int>(batch);
    g.vec_is_a = 0;
    return g;
}

// 1D transforms of `count` contiguous vectors: in [count][n] -> out [count][n].
template <int PREC>
static ht_status pass_1d(const GemmState* G, const Axis& ax, bool inverse, const double* in, double* out,
                         int64_t count, hipStream_t s) {
    const GemmMat& A = inverse ? G->inv[0] : G->fwd[0];
    const GemmVecs& V = G->vec[0];
    PrepRows pr{};
    pr.mode = inverse ? ROW_INV : ROW_FWD;
    pr.in = in;
    pr.in_ld = ax.n;
    pr.c = V.c;
    pr.cj = V.cj;
    pr.bout = out;  // x_1, x_n go straight to the coefficient vector
    pr.bout_ld = ax.n;
    pr.bout_last = ax.n - 1;
    pr.hi = G->vhi;
    pr.lo = G->vlo;
    pr.scale = G->vscale;
    pr.Kp = A.Kp;
    ht_status st = run_prep_rows<PREC>(ax, pr, count, s);
    if (st != HT_OK) return st;
    GemmSplitArgs g = rows_gemm(G, A, count);
    g.out = out;
    g.o_ldm = ax.n;
    g.o_off = inverse ? 1 : 0;
    g.n_lim = inverse ? ax.N : ax.n;
    g.e1 = inverse ? V.nc : V.b;
    g.e2 = inverse ? V.ncj : V.bj;
    g.pos_is_m = 0;
    g.xb = inverse ? out : in;
    g.xb_vs = ax.n;
    g.xb_last = ax.n - 1;
    return run_gemm<PREC>(g, s);
}

// 2D inverse (T0^{-1} (x) T1^{-1}) with T^{-1} = M + U B^T per axis (M: the core GEMM on
// y_mid, U = [e_1 - c, e_n - c'], B^T y = [x_1, x_n] from the boundary solve):
//   R   = G B1            boundary solve of every row                   (float64)
//   W   = G M1^T          row GEMM; zero boundary columns
//   Z   = T0^{-1} R       two columns per image, float64 chirp-z core
//   out = T0^{-1} W + Z U1^T   column GEMM; the axis-0 and the cross rank-2 terms are
//                              added in float64 in its epilogue and its boundary rows
template <int PREC>
static ht_status inverse_2d(const ht_plan* p, const double* in, double* out, int64_t batch, hipStream_t s) {
    const GemmState* G = p->gemm;
    const Axis& a0 = p->ax[0];
    const Axis& a1 = p->ax[1];
    const int n0 = a0.n, n1 = a1.n;
    const int64_t img = static_cast<int64_t>(n0) * n1, rows = batch * n0;
    double* W = reinterpret_cast<double*>(p->work);
    // rows
    PrepRows pr{};
    pr.mode = ROW_INV;
    pr.in = in;
    pr.in_ld = n1;
    pr.bout = G->side_r;
    pr.bout_ld = 2;
    pr.bout_last = 1;
    pr.zout = W;
    pr.zout_ld = n1;
    pr.hi = G->vhi;
    pr.lo = G->vlo;
    pr.scale = G->vscale;
    pr.Kp = G->inv[1].Kp;
    ht_status st = run_prep_rows<PREC>(a1, pr, rows, s);
    if (st != HT_OK) return st;
    GemmSplitArgs g = rows_gemm(G, G->inv[1], rows);
    g.out = W;
    g.o_ldm = n1;
    g.o_off = 1;
    g.n_lim = a1.N;
    st = run_gemm<PREC>(g, s);
    if (st != HT_OK) return st;
    // the two boundary-coefficient columns in float64
    const View zin{G->side_r, 2LL * n0, 1, 2, 2, 0};
    const View zout{G->side_z, 2LL * n0, 1, 2, 2, 0};
    st = launch_core(a0, p->tw, true, zin, zout, 2 * batch, s);
    if (st != HT_OK) return st;
    // columns
    const Cross cr{G->side_z, n0, G->vec[1].u0, G->vec[1].u1};
    const int64_t rpi = round_up64(n1, GT_M);
    PrepCols pc{};
    pc.mode = COL_INV;
    pc.in = W;
    pc.img = img;
    pc.ld = n1;
    pc.ncols = n1;
    pc.n1 = n1;
    pc.xbuf = G->side_x;
    pc.xb_img = 2LL * n1;
    pc.xb_last = n1;
    pc.bout = out;
    pc.cross = cr;
    pc.hi = G->vhi;
    pc.lo = G->vlo;
    pc.scale = G->vscale;
    pc.Kp = G->inv[0].Kp;
    pc.rows_per_img = rpi;
    st = run_prep_cols<PREC>(a0, pc, batch, s);
    if (st != HT_OK) return st;
    g = cols_gemm(G, G->inv[0], rpi, batch);
    g.out = out;
    g.o_img = img;
    g.o_ldm = n1;
    g.o_off = n1;
    g.m_lim = a0.N;
    g.n_lim = n1;
    g.e1 = G->vec[0].nc;
    g.e2 = G->vec[0].ncj;
    g.pos_is_m = 1;
    g.xb = G->side_x;
    g.xb_img = 2LL * n1;
    g.xb_vs = 1;
    g.xb_last = n1;
    g.cross = cr;
    g.zc_off = 1;
    return run_gemm<PREC>(g, s);
}

// 2D forward (T0 (x) T1) with T = A V + [b, b'] [e_1, e_n]^T per axis (V x = x_mid +
// x_1 c + x_n c'):
//   Z   = T0 X E1         the two boundary columns of X, float64 chirp-z core
//   W   = T0 (X V1^T)     column GEMM on the axis-0 forms v of the columns of X V1^T
//   out = W A1^T + Z [b1, b1']^T   row GEMM; the cross rank-2 term in its epilogue
template <int PREC>
static ht_status forward_2d(const ht_plan* p, const double* in, double* out, int64_t batch, hipStream_t s) {
    const GemmState* G = p->gemm;
    const Axis& a0 = p->ax[0];
    const Axis& a1 = p->ax[1];
    const int n0 = a0.n, n1 = a1.n;
    const int64_t img = static_cast<int64_t>(n0) * n1, rows = batch * n0;
    double* W = reinterpret_cast<double*>(p->work);
    const View zin{const_cast<double*>(in), img, n1 - 1, n1, 2, 0};
    const View zout{G->side_z, 2LL * n0, 1, 2, 2, 0};
    ht_status st = launch_core(a0, p->tw, false, zin, zout, 2 * batch, s);
    if (st != HT_OK) return st;
    // columns of X V1^T
    const int64_t rpi = round_up64(a1.N, GT_M);
    PrepCols pc{};
    pc.mode = COL_FWD;
    pc.in = in;
    pc.img = img;
    pc.ld = n1;
    pc.ncols = a1.N;
    pc.c = G->vec[0].c;
    pc.cj = G->vec[0].cj;
    pc.c1 = G->vec[1].c;
    pc.cj1 = G->vec[1].cj;
    pc.n1 = n1;
    pc.xbuf = G->side_x;
    pc.xb_img = 2LL * n1;
    pc.xb_last = n1;
    pc.hi = G->vhi;
    pc.lo = G->vlo;
    pc.scale = G->vscale;
    pc.Kp = G->fwd[0].Kp;
    pc.rows_per_img = rpi;
    st = run_prep_cols<PREC>(a0, pc, batch, s);
    if (st != HT_OK) return st;
    GemmSplitArgs g = cols_gemm(G, G->fwd[0], rpi, batch);
    g.out = W;
    g.o_img = img;
    g.o_ldm = n1;
    g.o_off = 0;
    g.m_lim = n0;
    g.n_lim = a1.N;
    g.e1 = G->vec[0].b;
    g.e2 = G->vec[0].bj;
    g.pos_is_m = 1;
    g.xb = G->side_x;
    g.xb_img = 2LL * n1;
    g.xb_vs = 1;
    g.xb_last = n1;
    st = run_gemm<PREC>(g, s);
    if (st != HT_OK) return st;
    // rows: W is already in axis-1 form (first N1 entries of each row)
    PrepRows pr{};
    pr.mode = ROW_RAW;
    pr.in = W;
    pr.in_ld = n1;
    pr.hi = G->vhi;
    pr.lo = G->vlo;
    pr.scale = G->vscale;
    pr.Kp = G->fwd[1].Kp;
    st = run_prep_rows<PREC>(a1, pr, rows, s);
    if (st != HT_OK) return st;
    g = rows_gemm(G, G->fwd[1], rows);
    g.out = out;
    g.o_ldm = n1;
    g.o_off = 0;
    g.n_lim = n1;
    g.cross = Cross{G->side_z, 0, G->vec[1].b, G->vec[1].bj};
    g.zc_off = 0;
    return run_gemm<PREC>(g, s);
}

template <int PREC>
static ht_status gemm_transform_t(const ht_plan* p, bool inverse, const double* in, double* out, int64_t batch,
                                  hipStream_t s) {
    if (p->ndim == 1) return pass_1d<PREC>(p->gemm, p->ax[0], inverse, in, out, batch, s);
    return inverse ? inverse_2d<PREC>(p, in, out, batch, s) : forward_2d<PREC>(p, in, out, batch, s);
}

ht_status gemm_transform(const ht_plan* p, bool inverse, const double* in, double* out, int64_t batch,
                         hipStream_t s) {
    if (batch > p->max_batch) return fail(HT_ERR_INVALID_ARG, "batch exceeds the plan's max_batch");
    if (p->gemm->prec == HT_PRECISION_BF16X3) return gemm_transform_t<HT_PRECISION_BF16X3>(p, inverse, in, out, batch, s);
    return gemm_transform_t<HT_PRECISION_F16X3>(p, inverse, in, out, batch, s);
}

}  // namespace ht

using namespace ht;

extern "C" ht_status ht_plan_set_precision(ht_plan* p, int precision) {
    if (!p) return fail(HT_ERR_INVALID_ARG, "ht_plan_set_precision: null plan");
    if (precision != HT_PRECISION_F64 && precision != HT_PRECISION_BF16X3 && precision != HT_PRECISION_F16X3 &&
        precision != HT_PRECISION_F32)
        return fail(HT_ERR_INVALID_ARG, "ht_plan_set_precision: unknown precision");
    if (precision != HT_PRECISION_F64) {
        if (precision != HT_PRECISION_F32)
            for (int a = 0; a < p->ndim; ++a)
                if (p->ax[a].kind == HT_KIND_F || p->ax[a].kind == HT_KIND_P || p->ax[a].kind == HT_KIND_R ||
                    p->ax[a].kind == HT_KIND_F3)
                    return fail(HT_ERR_UNSUPPORTED,
                                "ht_plan_set_precision: the split-precision core needs a real boundary transform "
                                "(not T_F or a comparator)");
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
            return fail(HT_ERR_INVALID_ARG, "ht_plan_set_precision: the plan's device must be current");
    }
    if (precision == HT_PRECISION_F32) {
        ht_status st = plan_build_f32(p);
        if (st != HT_OK) return st;
        gemm_release(p->gemm);
        p->gemm = nullptr;
        return HT_OK;
    }
    GemmState* g = nullptr;
    if (precision != HT_PRECISION_F64) {
        ht_status st = build_gemm(p, precision, &g);
        if (st != HT_OK) return st;
    }
    gemm_release(p->gemm);
    p->gemm = g;
    plan_release_f32(p);
    return HT_OK;
}

extern "C" int ht_plan_precision(const ht_plan* p) {
    if (!p) return -1;
    if (p->f32) return HT_PRECISION_F32;
    return p->gemm ? p->gemm->prec : HT_PRECISION_F64;
}
