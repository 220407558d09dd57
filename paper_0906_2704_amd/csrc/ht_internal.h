// Internal definitions shared by the host plan code and the HIP kernels of libht.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ht.h"

namespace ht {

// Size of the global FFT twiddle table: tw[m] = exp(-2 pi i m / TWN).  Every FFT length
// used here divides TWN, so every twiddle is one exact table entry.
constexpr int TWN = 16384;
constexpr int MAX_N = 8192;
constexpr int MAX_LOGP = 13;  // largest LDS-resident FFT: 8192 complex doubles = 128 KiB
constexpr int MIN_LOGP = 9;   // smallest FFT (one wave of 64 threads, 8 points each)
// Convolution lengths M > 8192 run as two LDS-resident halves of M / 2 points (even and
// odd frequencies).  (Splitting M = 8192 as well halves its LDS but measured slower: the
// split kernel's registers then allow only one 512-thread workgroup per CU.)
constexpr int SPLIT_M = 16384;

enum OutMode { MODE_RE = 0, MODE_IM = 1, MODE_CPLX = 2 };

// Tables of one core direction (analysis X or synthesis X^{-1}) computed as a chirp-z
// transform: Y_k = post_k * sum_j b_{k-j} (pre_j x_j), evaluated by FFT convolution of
// length M = S * P with the precomputed spectrum B = FFT_M(b) / M.
template <class C>
struct ChirpT {
    const C* pre;         // [N]
    const C* post;        // [N]
    const C* B;           // [M]
    int mode;             // OutMode of the core output for a real result
};
using Chirp = ChirpT<double2>;
using Chirp32 = ChirpT<float2>;  // float32 copies (HT_PRECISION_F32 cores)

// Everything a kernel needs about one 1D transform of length n (passed by value).
struct Axis {
    int n, N;             // signal length, core order n - 2
    int kind;             // ht_kind
    int logP;             // FFT size P = 2^logP handled by BLOCK = P / 8 threads
    int S;                // split factor (1 or 2), M = S * P >= 2N - 1
    int rank;             // DST2 / DST3: number of replaced core columns (degree - 1)
    double q1;            // q_1 (p_1 for the antireflective family)
    double minv[4];       // inverse of the 2x2 boundary system (C, F), row-major
    double Gm[4];         // (E^T K)^{-1} of the DST correction, rank x rank, row-major
    const double* q;      // [n] polynomial column q (or p)
    const double* bub;    // [rank][N] bubble columns (DST2/3)
    const double* U;      // [rank][N] K - E, K = Q * bubbles
    Chirp ana, syn;
    Chirp32 ana32, syn32; // float32 tables, set by ht_plan_set_precision(HT_PRECISION_F32)
    const float2* tw32;   // float32 twiddle table (same)
    int den;              // eigenvalue grid: angles pi * r / den
    const double* tcos;   // [2 den] cos(pi r / den)
    const double* tsin;   // [2 den] sin(pi r / den)
    const double2* tw;    // the device's FFT twiddle table
    // degree 3 for any PSF (kind F3): the T_F inverse corrected by
    //   a = Vi (x[2], x[n-2]),  x[2] = a0, x[n-2] = a1, x[j] -= f3v[j] a1 elsewhere,
    // with f3v = T_F^{-1} (cubic column) and Vi the inverse of rows {2, n-2} of
    // [ (e_2 + e_{n-2})/sqrt 2 | f3v ]; the forward adds f3b[0] x[2] + f3b[1] x[n-2].
    const double2* f3v;   // [n]
    const double* f3b;    // [2][n]: cosine column, cubic column (all n rows)
    double2 f3vi[4];      // Vi, row-major
    // Half-length real cores (ragged batches, real kinds): the core is a real DFT of
    // length L (N for the cosine core, N + 1 for the sine core) of which only the outputs
    // k <= L/2 are needed.  half = 1 (L even): a complex DFT of H = L/2 packed pairs;
    // half = 2 (cosine core, N odd): a chirp-z DFT of length N that keeps H = (N + 1)/2
    // outputs (the synthesis: reads H inputs).  Tables in ana (analysis) / syn
    // (synthesis), pre- and post-processing on htw.  0: the full chirp-z core.
    int half;
    int H;
    double hw[2];         // cosine core: sqrt(1/N), sqrt(2/N); sine core: sqrt(2/(N+1)), 0
    const double2* htw;   // half = 1: [2][H + 1]: cosine core e^{-2 pi i k/N}, e^{-i pi k/(2N)};
                          //   sine core e^{2 pi i k/(N+1)}, (sin(pi k/(N+1)), 0).
                          // half = 2: [H]: e^{-i pi k/(2N)}.
};

// Strided view of a batch of 1D signals: signal b lives at
//   base = (b / per_img) * img_stride + (b % per_img) * sig_stride,
// element i at base + i * elem_stride (units: elements of the array's type).
struct View {
    void* ptr;
    int64_t img_stride, sig_stride, elem_stride;
    int64_t per_img;
    int cplx;             // 1: interleaved complex128, 0: float64
};

struct GemmState;  // split-precision matrix-core cores of a plan (ht_gemm.hip)

// Exact GCV of a 1D plan (eq. gcv): with T = [t0 | core columns | t_{n-1}], interior rows
// T_I = S v_mid + R_C v_C (S the orthonormal core of order N, R_C the interior parts of the
// boundary and replaced columns C) and the two boundary rows,
//   ||T v||^2 = ||v_mid||^2 + 2 Re sum_c conj(P_c) v_c + v_C^H Gam v_C + |y_0|^2 + |y_{n-1}|^2,
//   P_c = (S^H R_c)^H v_mid,  y_0 = t0_0 v_0 + tn_0 v_{n-1} + a . v_mid  (y_{n-1} with b).
// vec[k][j] (k < nv, j < N) holds the factors f with P_c = sum_j f_j v_j:
// conj(S^H R_c) for the columns of C, then a and b when the core has ghost rows.
constexpr int XG_MAXC = 4;
struct XgcvParams {
    const double2* vec;   // [nv][N]
    int nc, nv, rows;     // |C|, number of vectors, 1 if a and b are present
    int cidx[XG_MAXC];    // coefficient index of each column of C
    double gam[XG_MAXC][XG_MAXC];
    double t00, t0n, tn0, tnn;  // T[0][0], T[0][n-1], T[n-1][0], T[n-1][n-1]
};

}  // namespace ht

struct ht_plan {
    int ndim = 1;
    int device = 0;
    ht::Axis ax[2];
    int cplx = 0;                      // any axis of kind F
    int64_t max_batch = 1;
    void* arena = nullptr;             // device tables of both axes
    double2* work = nullptr;           // 2D: [max_batch][n0][n1] complex workspace
    double* gcv_part = nullptr;        // 2D GCV partial sums
    int64_t gcv_part_elems = 0;
    const double2* tw = nullptr;       // global twiddle table of this device
    ht::GemmState* gemm = nullptr;     // set by ht_plan_set_precision (null: float64 core)
    int f32 = 0;                       // float32 chirp-z cores (HT_PRECISION_F32)
    void* arena32 = nullptr;           // their tables
    ht::XgcvParams xg[2]{};            // exact GCV tables per axis (vec in xg_mem)
    void* xg_mem[2] = {nullptr, nullptr};
    // 2D exact GCV workspace (ht_gcv_scan_exact on 2D plans): row-pass outputs, column-pass
    // partials and the G values when the caller passes none, sized for grids of up to
    // xg2_max_k values (ht_plan_reserve_exact_gcv)
    void* xg2_mem = nullptr;
    int xg2_max_k = 0;
    int64_t xg2_rows_elems = 0, xg2_part_elems = 0, xg2_g_elems = 0;
};

namespace ht {

// error reporting (thread-local message, see ht_last_error)
ht_status fail(ht_status st, const std::string& msg);
ht_status check_hip(hipError_t e, const char* what);
const double2* device_twiddles(int device, ht_status* st);

// split-precision cores (ht_gemm.hip): in and out contiguous, must not overlap
ht_status gemm_transform(const ht_plan* p, bool inverse, const double* in, double* out, int64_t batch,
                         hipStream_t stream);
void gemm_release(GemmState* g);

// exact GCV tables of a 1D plan (ht_plan.hip)
struct HostAxis;
ht_status build_exact_gcv(const HostAxis& h, ht_plan* p, int axis);
// the 2D exact GCV workspace of a plan for grids of up to max_k values (ht_spectral.hip)
ht_status reserve_exact_gcv_2d(ht_plan* p, int max_k);
constexpr int XG2_DEFAULT_K = 128;  // grid size reserved at plan creation
// device address of the static scratch of ht_gcv_scan_exact_static on `device` (current)
ht_status static_scratch_init(int device, double** out);

// float32 chirp-z cores (ht_plan.hip)
ht_status plan_build_f32(ht_plan* p);
void plan_release_f32(ht_plan* p);

// launchers (ht_transform.hip)
ht_status launch_core(const Axis& ax, const double2* tw, bool inverse, const View& in,
                      const View& out, int64_t count, hipStream_t stream, bool f32 = false);

}  // namespace ht
