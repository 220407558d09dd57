// The learned-mu predictor as a library object: a 72 -> 256 -> 256 -> 256 -> 1 network with
// exact GELU (float32 master weights, bfloat16 copies for the matrix-core GEMMs, Adam
// moments) and its forward pass, backward pass, Adam step, minibatch training step,
// feature standardisation and the batched prediction of log10 mu.  Every step runs in the
// library's kernels (the network kernels of ht_mlp.hip and the gathers, reductions and
// conversions below); the object owns every buffer, sized at creation, so the calls only
// launch kernels.  Not in the paper: an accelerator of its GCV choice of mu (Section 4).
//
// Parameter layout (one float32 vector, HT_MLP_PARAMS entries): W1 [72][256], b1 [256],
// W2 [256][256], b2, W3 [256][256], b3, W4 [256][1], b4 [1]; W row-major [in][out].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "ht_internal.h"

namespace ht {

constexpr int MLP_IN = 72, MLP_H = 256;
constexpr int64_t MLP_DIMS[5] = {MLP_IN, MLP_H, MLP_H, MLP_H, 1};

struct MlpLayout {
    int64_t w[4], b[4], total;
    MlpLayout() {
        int64_t off = 0;
        for (int l = 0; l < 4; ++l) {
            w[l] = off;
            off += MLP_DIMS[l] * MLP_DIMS[l + 1];
            b[l] = off;
            off += MLP_DIMS[l + 1];
        }
        total = off;
    }
};
static const MlpLayout LAYOUT;

// rows of the feature matrix are gathered by a device index list
__global__ void k_gather_rows(const float* src, const float* tsrc, const int32_t* idx, int64_t rows, int cols,
                              float* dst, float* tdst) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const int64_t r = i / cols;
    const int c = static_cast<int>(i - r * cols);
    const int64_t s = idx[r];
    dst[i] = src[s * cols + c];
    if (c == 0) tdst[r] = tsrc[s];
}

// per-column mean and standard deviation (population, floored at 1e-6) of a [rows][cols]
// float32 matrix: one block per column, float64 sums over rows in a fixed order (strided
// per thread, then a fixed tree), two passes (mean, then the squared deviations)
__global__ __launch_bounds__(256) void k_col_mean_std(const float* X, int64_t rows, int cols, float* mean,
                                                      float* stdv) {
    __shared__ double part[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) s += static_cast<double>(X[i * cols + j]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double mu = part[0] / static_cast<double>(rows);
    __syncthreads();
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
        const double e = static_cast<double>(X[i * cols + j]) - mu;
        v += e * e;
    }
    part[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mean[j] = static_cast<float>(mu);
        stdv[j] = static_cast<float>(fmax(sqrt(part[0] / static_cast<double>(rows)), 1e-6));
    }
}

// loss = mean of the per-row squared errors (float64 sum in a fixed order)
__global__ __launch_bounds__(256) void k_mean(const float* sq, int64_t rows, float* out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) s += static_cast<double>(sq[i]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = static_cast<float>(part[0] / static_cast<double>(rows));
}

__global__ void k_log10(const double* x, float* y, int64_t count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) y[i] = static_cast<float>(log10(x[i]));
}

static unsigned nblocks(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace ht

using namespace ht;

struct ht_mlp {
    int device = 0;
    int64_t max_rows = 0;
    int64_t steps = 0;          // Adam steps taken
    int64_t fwd_rows = 0;       // rows of the last forward pass (backward needs the same)
    void* arena = nullptr;
    float* P = nullptr;         // [HT_MLP_PARAMS] float32 masters
    float* G = nullptr;         // gradients
    float* M = nullptr;         // Adam first moments
    float* V = nullptr;         // Adam second moments
    uint16_t* Pb = nullptr;     // bfloat16 copies (every entry; the GEMMs read the weights)
    uint16_t* Wt = nullptr;     // the bfloat16 weights transposed ([out][in] per layer, at the
                                // offsets of LAYOUT.w): contiguous along the contraction for the
                                // forward GEMMs
    float* mean = nullptr;      // [72]
    float* stdv = nullptr;      // [72]
    float* w4r = nullptr;       // [256] float32 value of the bfloat16 W4
    // activations and gradients for max_rows rows
    uint16_t* Xb = nullptr;     // [R][72]
    float* Z[3]{};              // [R][256] pre-activations
    uint16_t* Hb[3]{};          // [R][256] bfloat16 activations
    float* H3 = nullptr;        // [R][256] float32 value of Hb[2]
    float* y = nullptr;         // [R]
    float* dy = nullptr;
    float* sq = nullptr;
    float* dH = nullptr;        // [R][256]
    float* dZ = nullptr;
    uint16_t* dZb = nullptr;
    float* Xg = nullptr;        // [R][72] gathered minibatch
    float* tg = nullptr;        // [R]
};

namespace {

// keep: write the pre-activations and the float32 last hidden layer that the backward pass
// reads (training); inference writes only the bfloat16 activations the next layer reads
ht_status mlp_forward_rows(ht_mlp* m, const float* X, int64_t B, float* pred, hipStream_t st, bool keep = true) {
    const MlpLayout& L = LAYOUT;
    const int H = MLP_H;
    ht_status s = ht_to_bf16(X, m->Xb, B, MLP_IN, m->mean, m->stdv, st);
    if (s) return s;
    // B(k, j) = W[k][j] read from the transposed copy Wt[j][k] (sb_k = 1, sb_j = fan_in)
    s = ht_gemm_bf16(static_cast<int>(B), H, MLP_IN, m->Xb, MLP_IN, 1, m->Wt + L.w[0], 1, MLP_IN, m->P + L.b[0], 1,
                     keep ? m->Z[0] : nullptr, nullptr, H, m->Hb[0], st);
    if (s) return s;
    s = ht_gemm_bf16(static_cast<int>(B), H, H, m->Hb[0], H, 1, m->Wt + L.w[1], 1, H, m->P + L.b[1], 1,
                     keep ? m->Z[1] : nullptr, nullptr, H, m->Hb[1], st);
    if (s) return s;
    s = ht_gemm_bf16(static_cast<int>(B), H, H, m->Hb[1], H, 1, m->Wt + L.w[2], 1, H, m->P + L.b[2], 1,
                     keep ? m->Z[2] : nullptr, keep ? m->H3 : nullptr, H, m->Hb[2], st);
    if (s) return s;
    return ht_gemm_bf16(static_cast<int>(B), 1, H, m->Hb[2], H, 1, m->Wt + L.w[3], 1, H, m->P + L.b[3], 0, nullptr,
                        pred, 1, nullptr, st);
}

ht_status mlp_backward_rows(ht_mlp* m, const float* t, int64_t B, float* loss, hipStream_t st) {
    const MlpLayout& L = LAYOUT;
    const int H = MLP_H;
    ht_status s = ht_mse_grad(m->y, t, m->dy, m->sq, B, st);
    if (s) return s;
    if ((s = ht_colsum(m->H3, B, H, m->dy, m->G + L.w[3], st))) return s;
    if ((s = ht_colsum(m->dy, B, 1, nullptr, m->G + L.b[3], st))) return s;
    if ((s = ht_from_bf16(m->Pb + L.w[3], m->w4r, H, st))) return s;
    if ((s = ht_outer(m->dy, m->w4r, m->dH, B, H, st))) return s;
    const uint16_t* ins[3] = {m->Xb, m->Hb[0], m->Hb[1]};
    for (int l = 2; l >= 0; --l) {
        if ((s = ht_gelu_backward(m->Z[l], m->dH, m->dZ, m->dZb, B * H, st))) return s;
        const int fan_in = static_cast<int>(MLP_DIMS[l]);
        // dW = H_in^T dZ (fan_in x 256), the contraction over the minibatch
        if ((s = ht_gemm_bf16(fan_in, H, static_cast<int>(B), ins[l], 1, fan_in, m->dZb, H, 1, nullptr, 0, nullptr,
                              m->G + L.w[l], H, nullptr, st)))
            return s;
        if ((s = ht_colsum(m->dZ, B, H, nullptr, m->G + L.b[l], st))) return s;
        if (l > 0) {  // dH_in = dZ W^T
            if ((s = ht_gemm_bf16(static_cast<int>(B), H, H, m->dZb, H, 1, m->Pb + L.w[l], 1, H, nullptr, 0, nullptr,
                                  m->dH, H, nullptr, st)))
                return s;
        }
    }
    if (loss) {
        hipLaunchKernelGGL(k_mean, dim3(1), dim3(256), 0, st, m->sq, B, loss);
        return check_hip(hipGetLastError(), "ht_mlp_backward loss");
    }
    return HT_OK;
}

// the transposed bfloat16 weights, after every change of the bfloat16 copies
ht_status refresh_wt(ht_mlp* m, hipStream_t st) {
    for (int l = 0; l < 4; ++l) {
        ht_status s = ht_transpose_bf16(m->Pb + LAYOUT.w[l], m->Wt + LAYOUT.w[l], static_cast<int>(MLP_DIMS[l]),
                                        static_cast<int>(MLP_DIMS[l + 1]), st);
        if (s) return s;
    }
    return HT_OK;
}

ht_status mlp_adam(ht_mlp* m, float lr, hipStream_t st) {
    m->steps += 1;
    ht_status s = ht_adam(m->P, m->G, m->M, m->V, LAYOUT.total, lr, 0.9f, 0.999f, 1e-8f, m->steps, m->Pb, st);
    return s ? s : refresh_wt(m, st);
}

ht_status check_rows(const ht_mlp* m, int64_t rows, const char* what) {
    if (!m) return fail(HT_ERR_INVALID_ARG, std::string(what) + ": null network");
    if (rows < 1 || rows > m->max_rows)
        return fail(HT_ERR_INVALID_ARG, std::string(what) + ": rows must be in [1, max_rows]");
    return HT_OK;
}

}  // namespace

extern "C" int64_t ht_mlp_param_count(void) { return LAYOUT.total; }

extern "C" ht_status ht_mlp_create(int64_t max_rows, ht_mlp** out) {
    if (!out) return fail(HT_ERR_INVALID_ARG, "ht_mlp_create: null output");
    *out = nullptr;
    if (max_rows < 1 || max_rows > (int64_t{1} << 24)) return fail(HT_ERR_INVALID_ARG, "ht_mlp_create: max_rows");
    ht_mlp* m = new (std::nothrow) ht_mlp;
    if (!m) return fail(HT_ERR_OOM, "ht_mlp_create: host allocation");
    ht_status s = check_hip(hipGetDevice(&m->device), "ht_mlp_create: hipGetDevice");
    if (s) {
        delete m;
        return s;
    }
    const int64_t P = LAYOUT.total, R = max_rows, H = MLP_H;
    // arena: float32 blocks then bfloat16 blocks, each block 256-byte aligned
    int64_t f32[] = {P, P, P, P, MLP_IN, MLP_IN, H, R * H, R * H, R * H, R * H, R, R, R, R * H, R * H, R * MLP_IN, R};
    int64_t b16[] = {P, P, R * MLP_IN, R * H, R * H, R * H, R * H};
    size_t bytes = 0;
    auto pad = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    for (int64_t e : f32) bytes += pad(static_cast<size_t>(e) * 4);
    for (int64_t e : b16) bytes += pad(static_cast<size_t>(e) * 2);
    if (hipMalloc(&m->arena, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete m;
        return fail(HT_ERR_OOM, "ht_mlp_create: device allocation");
    }
    char* c = static_cast<char*>(m->arena);
    auto take = [&](int64_t elems, size_t es) {
        void* p = c;
        c += pad(static_cast<size_t>(elems) * es);
        return p;
    };
    m->P = static_cast<float*>(take(P, 4));
    m->G = static_cast<float*>(take(P, 4));
    m->M = static_cast<float*>(take(P, 4));
    m->V = static_cast<float*>(take(P, 4));
    m->mean = static_cast<float*>(take(MLP_IN, 4));
    m->stdv = static_cast<float*>(take(MLP_IN, 4));
    m->w4r = static_cast<float*>(take(H, 4));
    for (int l = 0; l < 3; ++l) m->Z[l] = static_cast<float*>(take(R * H, 4));
    m->H3 = static_cast<float*>(take(R * H, 4));
    m->y = static_cast<float*>(take(R, 4));
    m->dy = static_cast<float*>(take(R, 4));
    m->sq = static_cast<float*>(take(R, 4));
    m->dH = static_cast<float*>(take(R * H, 4));
    m->dZ = static_cast<float*>(take(R * H, 4));
    m->Xg = static_cast<float*>(take(R * MLP_IN, 4));
    m->tg = static_cast<float*>(take(R, 4));
    m->Pb = static_cast<uint16_t*>(take(P, 2));
    m->Wt = static_cast<uint16_t*>(take(P, 2));
    m->Xb = static_cast<uint16_t*>(take(R * MLP_IN, 2));
    for (int l = 0; l < 3; ++l) m->Hb[l] = static_cast<uint16_t*>(take(R * H, 2));
    m->dZb = static_cast<uint16_t*>(take(R * H, 2));
    m->max_rows = max_rows;
    // zero parameters and moments, identity standardisation
    s = check_hip(hipMemset(m->arena, 0, bytes), "ht_mlp_create: clear");
    if (!s) {
        float ones[MLP_IN];
        for (float& v : ones) v = 1.0f;
        s = check_hip(hipMemcpy(m->stdv, ones, sizeof(ones), hipMemcpyHostToDevice), "ht_mlp_create: std");
    }
    if (s) {
        (void)hipFree(m->arena);
        delete m;
        return s;
    }
    *out = m;
    return HT_OK;
}

extern "C" ht_status ht_mlp_destroy(ht_mlp* m) {
    if (!m) return HT_OK;
    ht_status s = HT_OK;
    if (m->arena) s = check_hip(hipFree(m->arena), "ht_mlp_destroy");
    delete m;
    return s;
}

extern "C" ht_status ht_mlp_set_params(ht_mlp* m, const float* params, hipStream_t st) {
    if (!m || !params) return fail(HT_ERR_INVALID_ARG, "ht_mlp_set_params: null argument");
    ht_status s = check_hip(hipMemcpyAsync(m->P, params, LAYOUT.total * 4, hipMemcpyDeviceToDevice, st),
                            "ht_mlp_set_params: copy");
    if (s) return s;
    s = ht_to_bf16(m->P, m->Pb, LAYOUT.total, 1, nullptr, nullptr, st);
    return s ? s : refresh_wt(m, st);
}

extern "C" ht_status ht_mlp_get(const ht_mlp* m, int what, float* out, hipStream_t st) {
    if (!m || !out) return fail(HT_ERR_INVALID_ARG, "ht_mlp_get: null argument");
    const float* src = nullptr;
    int64_t n = LAYOUT.total;
    switch (what) {
        case HT_MLP_PARAMS_VEC: src = m->P; break;
        case HT_MLP_GRADS_VEC: src = m->G; break;
        case HT_MLP_ADAM_M_VEC: src = m->M; break;
        case HT_MLP_ADAM_V_VEC: src = m->V; break;
        case HT_MLP_MEAN_VEC: src = m->mean; n = MLP_IN; break;
        case HT_MLP_STD_VEC: src = m->stdv; n = MLP_IN; break;
        default: return fail(HT_ERR_INVALID_ARG, "ht_mlp_get: unknown vector");
    }
    return check_hip(hipMemcpyAsync(out, src, n * 4, hipMemcpyDeviceToDevice, st), "ht_mlp_get: copy");
}

extern "C" ht_status ht_mlp_set_state(ht_mlp* m, const float* adam_m, const float* adam_v, int64_t steps,
                                      const float* mean, const float* stdv, hipStream_t st) {
    if (!m || steps < 0 || (!adam_m) != (!adam_v) || (!mean) != (!stdv))
        return fail(HT_ERR_INVALID_ARG, "ht_mlp_set_state: bad argument");
    ht_status s = HT_OK;
    if (adam_m) {
        if ((s = check_hip(hipMemcpyAsync(m->M, adam_m, LAYOUT.total * 4, hipMemcpyDeviceToDevice, st), "m")))
            return s;
        if ((s = check_hip(hipMemcpyAsync(m->V, adam_v, LAYOUT.total * 4, hipMemcpyDeviceToDevice, st), "v")))
            return s;
    }
    if (mean) {
        if ((s = check_hip(hipMemcpyAsync(m->mean, mean, MLP_IN * 4, hipMemcpyDeviceToDevice, st), "mean")))
            return s;
        if ((s = check_hip(hipMemcpyAsync(m->stdv, stdv, MLP_IN * 4, hipMemcpyDeviceToDevice, st), "std")))
            return s;
    }
    m->steps = steps;
    return HT_OK;
}

extern "C" int64_t ht_mlp_steps(const ht_mlp* m) { return m ? m->steps : -1; }

extern "C" ht_status ht_mlp_fit_standardisation(ht_mlp* m, const float* features, int64_t rows, hipStream_t st) {
    if (!m || !features || rows < 1) return fail(HT_ERR_INVALID_ARG, "ht_mlp_fit_standardisation: bad argument");
    hipLaunchKernelGGL(k_col_mean_std, dim3(MLP_IN), dim3(256), 0, st, features, rows, MLP_IN, m->mean, m->stdv);
    return check_hip(hipGetLastError(), "ht_mlp_fit_standardisation launch");
}

extern "C" ht_status ht_mlp_forward(ht_mlp* m, const float* features, int64_t rows, float* pred, hipStream_t st) {
    ht_status s = check_rows(m, rows, "ht_mlp_forward");
    if (s) return s;
    if (!features) return fail(HT_ERR_INVALID_ARG, "ht_mlp_forward: null features");
    m->fwd_rows = rows;
    s = mlp_forward_rows(m, features, rows, m->y, st);
    if (s || !pred || pred == m->y) return s;
    return check_hip(hipMemcpyAsync(pred, m->y, rows * 4, hipMemcpyDeviceToDevice, st), "ht_mlp_forward: copy");
}

extern "C" ht_status ht_mlp_predict(ht_mlp* m, const float* features, int64_t rows, float* pred, hipStream_t st) {
    if (!m || !features || !pred || rows < 0) return fail(HT_ERR_INVALID_ARG, "ht_mlp_predict: bad argument");
    m->fwd_rows = 0;  // the activations left behind are not those of an ht_mlp_forward
    for (int64_t r0 = 0; r0 < rows; r0 += m->max_rows) {
        const int64_t r = rows - r0 < m->max_rows ? rows - r0 : m->max_rows;
        ht_status s = mlp_forward_rows(m, features + r0 * MLP_IN, r, pred + r0, st, false);
        if (s) return s;
    }
    return HT_OK;
}

extern "C" ht_status ht_mlp_backward(ht_mlp* m, const float* target, int64_t rows, float* loss, hipStream_t st) {
    ht_status s = check_rows(m, rows, "ht_mlp_backward");
    if (s) return s;
    if (!target) return fail(HT_ERR_INVALID_ARG, "ht_mlp_backward: null target");
    if (rows != m->fwd_rows) return fail(HT_ERR_INVALID_ARG, "ht_mlp_backward: rows differ from the last forward pass");
    return mlp_backward_rows(m, target, rows, loss, st);
}

extern "C" ht_status ht_mlp_adam_step(ht_mlp* m, float lr, hipStream_t st) {
    if (!m || !(lr > 0.0f)) return fail(HT_ERR_INVALID_ARG, "ht_mlp_adam_step: bad argument");
    return mlp_adam(m, lr, st);
}

extern "C" ht_status ht_mlp_train_step(ht_mlp* m, const float* features, const float* target, const int32_t* idx,
                                       int64_t rows, float lr, float* loss, hipStream_t st) {
    ht_status s = check_rows(m, rows, "ht_mlp_train_step");
    if (s) return s;
    if (!features || !target || !idx || !(lr > 0.0f)) return fail(HT_ERR_INVALID_ARG, "ht_mlp_train_step: bad argument");
    hipLaunchKernelGGL(k_gather_rows, dim3(nblocks(rows * MLP_IN)), dim3(256), 0, st, features, target, idx, rows,
                       MLP_IN, m->Xg, m->tg);
    if ((s = check_hip(hipGetLastError(), "ht_mlp_train_step gather"))) return s;
    m->fwd_rows = rows;
    if ((s = mlp_forward_rows(m, m->Xg, rows, m->y, st))) return s;
    if ((s = mlp_backward_rows(m, m->tg, rows, loss, st))) return s;
    return mlp_adam(m, lr, st);
}

extern "C" ht_status ht_mlp_weights_of(const ht_mlp* m, ht_mlp_weights* out) {
    if (!m || !out) return fail(HT_ERR_INVALID_ARG, "ht_mlp_weights_of: null argument");
    for (int l = 0; l < 4; ++l) {
        out->w[l] = m->Pb + LAYOUT.w[l];
        out->b[l] = m->P + LAYOUT.b[l];
    }
    out->mean = m->mean;
    out->std = m->stdv;
    return HT_OK;
}

extern "C" ht_status ht_log10_labels(const double* mu, float* labels, int64_t count, hipStream_t st) {
    if (count < 0 || (count > 0 && (!mu || !labels))) return fail(HT_ERR_INVALID_ARG, "ht_log10_labels: bad argument");
    if (count == 0) return HT_OK;
    hipLaunchKernelGGL(k_log10, dim3(nblocks(count)), dim3(256), 0, st, mu, labels, count);
    return check_hip(hipGetLastError(), "ht_log10_labels launch");
}

extern "C" ht_status ht_lambda_predict(const ht_batch* bt, ht_mlp* m, const double* signal, const double* psf,
                                       double* coeff, float* features, double* spectrum, float* pred,
                                       hipStream_t st) {
    if (!bt || !m || !pred) return fail(HT_ERR_INVALID_ARG, "ht_lambda_predict: null argument");
    const int64_t count = ht_batch_count(bt);
    ht_status s = ht_batch_features(bt, signal, psf, coeff, features, spectrum, st);
    if (s) return s;
    return ht_mlp_predict(m, features, count, pred, st);
}
