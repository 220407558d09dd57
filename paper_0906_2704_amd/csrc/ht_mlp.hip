// Kernels of the learned-mu predictor: a small MLP trained and evaluated on the GPU.
//
//   GEMM      C = act(A B + bias) with A, B in bfloat16 and float32 accumulation on the
//             matrix cores: 64 x 64 blocks of four waves with the contraction staged
//             through LDS; unit-stride operands as 16-byte vectors on
//             v_mfma_f32_16x16x32_bf16, strided ones (the transposed operands of the
//             backward pass, which need no copy) element by element on
//             v_mfma_f32_16x16x16bf16_1k
//   GELU      exact, 0.5 x (1 + erf(x / sqrt 2)); derivative Phi(x) + x phi(x)
//   reductions column sums (bias gradients) in a fixed order: deterministic
//   Adam      float32 master weights and moments, bfloat16 copies for the GEMMs
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ht_internal.h"

namespace ht {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float x) {
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
    return cdf + x * pdf;
}

struct Gemm {
    int M, N, K;
    const uint16_t* A;
    int64_t sa_i, sa_k;
    const uint16_t* B;
    int64_t sb_k, sb_j;
    const float* bias;  // [N] or null
    int act;            // 0: none, 1: GELU
    float* Z;           // pre-activation out (may be null)
    float* C;           // activated out (may be null)
    int64_t ldc;
    uint16_t* Cb;       // bfloat16 copy of the activated out (may be null)
};

// A workgroup of four waves computes a 64 x 64 block of C; wave w owns rows 16w .. 16w+15
// (four 16 x 16 MFMA tiles).  The contraction runs in chunks of 64 staged in LDS: A as
// [row][k], B transposed to [col][k], so that every lane reads its four consecutive k in
// one 8-byte access.  Lane l supplies A row l % 16, k = 4 (l / 16) + 0..3 and B column
// l % 16, same k, and receives D rows 4 (l / 16) + 0..3 of column l % 16.  Operands
// outside the matrices read 0.
constexpr int GB = 64, GKC = 64, GPAD = GKC + 4;

__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
    __shared__ __attribute__((aligned(8))) uint16_t sA[GB][GPAD];
    __shared__ __attribute__((aligned(8))) uint16_t sB[GB][GPAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nbj = (g.N + GB - 1) / GB;
    const int bi = blockIdx.x / nbj, bj = blockIdx.x - bi * nbj;
    const int64_t row0 = static_cast<int64_t>(bi) * GB, col0 = static_cast<int64_t>(bj) * GB;
    const int r = lane & 15, q = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < g.K; k0 += GKC) {
        // stage: element e = tid + 256 u of the 64 x 64 chunk; k fastest for A, column
        // fastest for B (the contiguous direction of the usual layouts)
#pragma unroll 4
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u;
            const int ar = e >> 6, ak = e & 63;
            const int64_t gi = row0 + ar;
            const int gk = k0 + ak;
            sA[ar][ak] = (gi < g.M && gk < g.K) ? g.A[gi * g.sa_i + gk * g.sa_k] : static_cast<uint16_t>(0);
            const int bk = e >> 6, bc = e & 63;
            const int64_t gj = col0 + bc;
            const int gk2 = k0 + bk;
            sB[bc][bk] = (gj < g.N && gk2 < g.K) ? g.B[gk2 * g.sb_k + gj * g.sb_j] : static_cast<uint16_t>(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GKC; kk += 16) {
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(&sA[16 * w + r][kk + 4 * q]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bf16x4 b = *reinterpret_cast<const bf16x4*>(&sB[16 * t + r][kk + 4 * q]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t cj = col0 + 16 * t + r;
        if (cj >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t ci = row0 + 16 * w + 4 * q + i;
            if (ci >= g.M) continue;
            float z = acc[t][i] + (g.bias ? g.bias[cj] : 0.0f);
            if (g.Z) g.Z[ci * g.ldc + cj] = z;
            const float y = g.act ? gelu(z) : z;
            const uint16_t yb = f32_to_bf16(y);
            if (g.C) g.C[ci * g.ldc + cj] = g.Cb ? bf16_to_f32(yb) : y;
            if (g.Cb) g.Cb[ci * g.ldc + cj] = yb;
        }
    }
}

// Unit-stride operands (A row-major [M][K], B row-major [K][N], K and N multiples of 8,
// 16-byte aligned rows): the same 64 x 64 block per workgroup of four waves, but the
// operands arrive as 16-byte vectors (eight bfloat16) and the contraction runs in steps of
// 32 on v_mfma_f32_16x16x32_bf16.  A is staged as [row][k]; B is transposed into [col][k]
// as it is staged.  Rows of 72 elements (144 bytes) keep the 16-byte fragment reads of
// the 16 rows of a lane group in distinct banks.  Lane l supplies A row l % 16 and B
// column l % 16 with k = 8 (l / 16) + 0..7, and receives D rows 4 (l / 16) + 0..3 of
// column l % 16.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
constexpr int VKC = 64, VPAD = VKC + 8;

template <bool BT>  // BT: B is given transposed (B(k, j) = B[j sb_j + k]), staged without a transpose
__global__ __launch_bounds__(256) void k_gemm_vec(Gemm g) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[GB][VPAD];
    __shared__ __attribute__((aligned(16))) uint16_t sB[GB][VPAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nbj = (g.N + GB - 1) / GB;
    const int bi = blockIdx.x / nbj, bj = blockIdx.x - bi * nbj;
    const int64_t row0 = static_cast<int64_t>(bi) * GB, col0 = static_cast<int64_t>(bj) * GB;
    const int r = lane & 15, q = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < g.K; k0 += VKC) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int v = tid + 256 * u;
            const int ar = v >> 3, seg = (v & 7) * 8;
            const int64_t gi = row0 + ar;
            const int gk = k0 + seg;
            u32x4v va = u32x4v{0u, 0u, 0u, 0u};
            if (gi < g.M && gk < g.K) va = *reinterpret_cast<const u32x4v*>(g.A + gi * g.sa_i + gk);
            *reinterpret_cast<u32x4v*>(&sA[ar][seg]) = va;
            if constexpr (BT) {  // column ar of C, contraction slice seg .. seg + 7
                const int64_t gj = col0 + ar;
                u32x4v vb = u32x4v{0u, 0u, 0u, 0u};
                if (gj < g.N && gk < g.K) vb = *reinterpret_cast<const u32x4v*>(g.B + gj * g.sb_j + gk);
                *reinterpret_cast<u32x4v*>(&sB[ar][seg]) = vb;
            } else {
                const int bk = v >> 3;
                const int64_t gj = col0 + seg;
                const int gk2 = k0 + bk;
                u32x4v vb = u32x4v{0u, 0u, 0u, 0u};
                if (gj < g.N && gk2 < g.K) vb = *reinterpret_cast<const u32x4v*>(g.B + gk2 * g.sb_k + gj);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    sB[seg + 2 * i][bk] = static_cast<uint16_t>(vb[i] & 0xffffu);
                    sB[seg + 2 * i + 1][bk] = static_cast<uint16_t>(vb[i] >> 16);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < VKC; kk += 32) {
            const u32x4v a = *reinterpret_cast<const u32x4v*>(&sA[16 * w + r][kk + 8 * q]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const u32x4v b = *reinterpret_cast<const u32x4v*>(&sB[16 * t + r][kk + 8 * q]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a),
                                                                 __builtin_bit_cast(bf16x8v, b), acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t cj = col0 + 16 * t + r;
        if (cj >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t ci = row0 + 16 * w + 4 * q + i;
            if (ci >= g.M) continue;
            float z = acc[t][i] + (g.bias ? g.bias[cj] : 0.0f);
            if (g.Z) g.Z[ci * g.ldc + cj] = z;
            const float y = g.act ? gelu(z) : z;
            const uint16_t yb = f32_to_bf16(y);
            if (g.C) g.C[ci * g.ldc + cj] = g.Cb ? bf16_to_f32(yb) : y;
            if (g.Cb) g.Cb[ci * g.ldc + cj] = yb;
        }
    }
}

// dst[c][r] = src[r][c] for a [rows][cols] bfloat16 matrix (32 x 32 tiles through LDS)
__global__ __launch_bounds__(256) void k_transpose16(const uint16_t* src, uint16_t* dst, int rows, int cols) {
    __shared__ uint16_t t[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8)
        if (r0 + i < rows && c0 + tx < cols) t[i][tx] = src[static_cast<int64_t>(r0 + i) * cols + c0 + tx];
    __syncthreads();
    for (int i = ty; i < 32; i += 8)
        if (c0 + i < cols && r0 + tx < rows) dst[static_cast<int64_t>(c0 + i) * rows + r0 + tx] = t[tx][i];
}

// dst = bf16((src - mean[col]) / std[col]) (mean/std may be null: plain conversion)
__global__ void k_to_bf16(const float* src, uint16_t* dst, int64_t rows, int cols, const float* mean,
                          const float* stdv) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const int c = static_cast<int>(i % cols);
    float v = src[i];
    if (mean) v = (v - mean[c]) / stdv[c];
    dst[i] = f32_to_bf16(v);
}

__global__ void k_from_bf16(const uint16_t* src, float* dst, int64_t count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = bf16_to_f32(src[i]);
}

// dz = dh * GELU'(z); also the bfloat16 copy used by the next GEMMs
__global__ void k_gelu_bwd(const float* z, const float* dh, float* dz, uint16_t* dzb, int64_t count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = dh[i] * gelu_grad(z[i]);
    dz[i] = v;
    if (dzb) dzb[i] = f32_to_bf16(v);
}

// out[j] = sum_i X[i][j] (rows summed in a fixed tree order): one block per column
__global__ __launch_bounds__(256) void k_colsum(const float* X, int64_t rows, int cols, float* out) {
    __shared__ float part[256];
    const int j = blockIdx.x;
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < rows; i += 256) s += X[i * cols + j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = part[0];
}

// dy = 2 (y - t) / B (mean squared error), and the per-row squared errors
__global__ void k_mse_grad(const float* y, const float* t, float* dy, float* sq, int64_t rows) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const float e = y[i] - t[i];
    dy[i] = 2.0f * e / static_cast<float>(rows);
    sq[i] = e * e;
}

// dh[i][j] = dy[i] * w[j]  (gradient through the last, one-output layer)
__global__ void k_outer(const float* dy, const float* w, float* dh, int64_t rows, int cols) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    dh[i] = dy[i / cols] * w[i % cols];
}

// X[i][j] * y[i] summed over i: gradient of a one-output layer's weights
__global__ __launch_bounds__(256) void k_weighted_colsum(const float* X, const float* y, int64_t rows, int cols,
                                                         float* out) {
    __shared__ float part[256];
    const int j = blockIdx.x;
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < rows; i += 256) s += X[i * cols + j] * y[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = part[0];
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* pb) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    const float pi = p[i] - upd;
    p[i] = pi;
    if (pb) pb[i] = f32_to_bf16(pi);
}

static unsigned blocks_for(int64_t n, int t = 256) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace ht

using namespace ht;

extern "C" ht_status ht_gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sa_i, int64_t sa_k,
                                  const uint16_t* B, int64_t sb_k, int64_t sb_j, const float* bias, int act,
                                  float* Z, float* C, int64_t ldc, uint16_t* Cb, hipStream_t stream) {
    if (M < 0 || N < 0 || K < 0 || (act != 0 && act != 1)) return fail(HT_ERR_INVALID_ARG, "ht_gemm_bf16: bad sizes");
    if (M == 0 || N == 0) return HT_OK;
    if (!A || !B || (!Z && !C && !Cb) || ldc < N) return fail(HT_ERR_INVALID_ARG, "ht_gemm_bf16: null argument or ldc < N");
    const int64_t blocks = static_cast<int64_t>((M + GB - 1) / GB) * ((N + GB - 1) / GB);
    if (blocks > 0x7fffffffLL) return fail(HT_ERR_INVALID_ARG, "ht_gemm_bf16: too large");
    Gemm g{M, N, K, A, sa_i, sa_k, B, sb_k, sb_j, bias, act, Z, C, ldc, Cb};
    const bool avec = sa_k == 1 && K % 8 == 0 && sa_i % 8 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(B) & 15) == 0;
    const bool brow = sb_j == 1 && N % 8 == 0 && sb_k % 8 == 0;       // B row-major [K][N]
    const bool bcol = sb_k == 1 && sb_j % 8 == 0;                     // B^T row-major [N][K]
    if (avec && bcol)
        hipLaunchKernelGGL(k_gemm_vec<true>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g);
    else if (avec && brow)
        hipLaunchKernelGGL(k_gemm_vec<false>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g);
    else
        hipLaunchKernelGGL(k_gemm, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, g);
    return check_hip(hipGetLastError(), "ht_gemm_bf16 launch");
}

extern "C" ht_status ht_to_bf16(const float* src, uint16_t* dst, int64_t rows, int cols, const float* mean,
                                const float* stdv, hipStream_t stream) {
    if (rows < 0 || cols < 1 || (!mean) != (!stdv)) return fail(HT_ERR_INVALID_ARG, "ht_to_bf16: bad argument");
    if (rows == 0) return HT_OK;
    if (!src || !dst) return fail(HT_ERR_INVALID_ARG, "ht_to_bf16: null argument");
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(rows * cols)), dim3(256), 0, stream, src, dst, rows, cols, mean, stdv);
    return check_hip(hipGetLastError(), "ht_to_bf16 launch");
}

extern "C" ht_status ht_from_bf16(const uint16_t* src, float* dst, int64_t count, hipStream_t stream) {
    if (count < 0) return fail(HT_ERR_INVALID_ARG, "ht_from_bf16: bad count");
    if (count == 0) return HT_OK;
    if (!src || !dst) return fail(HT_ERR_INVALID_ARG, "ht_from_bf16: null argument");
    hipLaunchKernelGGL(k_from_bf16, dim3(blocks_for(count)), dim3(256), 0, stream, src, dst, count);
    return check_hip(hipGetLastError(), "ht_from_bf16 launch");
}

extern "C" ht_status ht_gelu_backward(const float* z, const float* dh, float* dz, uint16_t* dzb, int64_t count,
                                      hipStream_t stream) {
    if (count < 0) return fail(HT_ERR_INVALID_ARG, "ht_gelu_backward: bad count");
    if (count == 0) return HT_OK;
    if (!z || !dh || !dz) return fail(HT_ERR_INVALID_ARG, "ht_gelu_backward: null argument");
    hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for(count)), dim3(256), 0, stream, z, dh, dz, dzb, count);
    return check_hip(hipGetLastError(), "ht_gelu_backward launch");
}

extern "C" ht_status ht_colsum(const float* X, int64_t rows, int cols, const float* weight, float* out,
                               hipStream_t stream) {
    if (rows < 0 || cols < 1 || cols > 65535 || !X || !out) return fail(HT_ERR_INVALID_ARG, "ht_colsum: bad argument");
    if (weight)
        hipLaunchKernelGGL(k_weighted_colsum, dim3(cols), dim3(256), 0, stream, X, weight, rows, cols, out);
    else
        hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, stream, X, rows, cols, out);
    return check_hip(hipGetLastError(), "ht_colsum launch");
}

extern "C" ht_status ht_mse_grad(const float* y, const float* t, float* dy, float* sq, int64_t rows,
                                 hipStream_t stream) {
    if (rows < 1 || !y || !t || !dy || !sq) return fail(HT_ERR_INVALID_ARG, "ht_mse_grad: bad argument");
    hipLaunchKernelGGL(k_mse_grad, dim3(blocks_for(rows)), dim3(256), 0, stream, y, t, dy, sq, rows);
    return check_hip(hipGetLastError(), "ht_mse_grad launch");
}

extern "C" ht_status ht_outer(const float* dy, const float* w, float* dh, int64_t rows, int cols, hipStream_t stream) {
    if (rows < 0 || cols < 1 || !dy || !w || !dh) return fail(HT_ERR_INVALID_ARG, "ht_outer: bad argument");
    if (rows == 0) return HT_OK;
    hipLaunchKernelGGL(k_outer, dim3(blocks_for(rows * cols)), dim3(256), 0, stream, dy, w, dh, rows, cols);
    return check_hip(hipGetLastError(), "ht_outer launch");
}

extern "C" ht_status ht_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float beta1,
                             float beta2, float eps, int64_t step, uint16_t* pb, hipStream_t stream) {
    if (count < 0 || step < 1 || !p || !g || !m || !v) return fail(HT_ERR_INVALID_ARG, "ht_adam: bad argument");
    if (count == 0) return HT_OK;
    const float c1 = 1.0f - powf(beta1, static_cast<float>(step));
    const float c2 = 1.0f - powf(beta2, static_cast<float>(step));
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(count)), dim3(256), 0, stream, p, g, m, v, count, lr, beta1, beta2, eps,
                       c1, c2, pb);
    return check_hip(hipGetLastError(), "ht_adam launch");
}

extern "C" ht_status ht_transpose_bf16(const uint16_t* src, uint16_t* dst, int rows, int cols, hipStream_t stream) {
    if (rows < 0 || cols < 0 || (rows > 0 && cols > 0 && (!src || !dst)) || src == dst)
        return fail(HT_ERR_INVALID_ARG, "ht_transpose_bf16: bad argument");
    if (rows == 0 || cols == 0) return HT_OK;
    hipLaunchKernelGGL(k_transpose16, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, stream, src, dst, rows,
                       cols);
    return check_hip(hipGetLastError(), "ht_transpose_bf16 launch");
}
