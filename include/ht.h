/*
 * ht.h -- C ABI of the MI355X (gfx950) library for spectral Tikhonov deblurring under
 * high-order (polynomial preserving) boundary conditions, after M. Donatelli, "Fast
 * transforms for high order boundary conditions".
 *
 * Problem statement (Sections 2 and 4 of the paper): an observed signal or image g, a PSF
 * mask h_{-m..m} with symbol z(t) = sum_j h_j e^{ijt} (eq. symbol), a boundary model that
 * preserves sampled polynomials of a given degree, a smoothing operator L (identity or
 * second difference / Laplacian) and a regularisation parameter mu > 0.  The blurring
 * matrix is A = T diag(d) T^{-1} for a fast transform T (eqs. ART, Tc, Tf), and the
 * restoration is f = T Phi D^{-1} T^{-1} g (eq. freg) with mu chosen by GCV (eq. mugcv).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller, except where a
 *     parameter is documented as a host array.  The library never frees caller memory.
 *   - Calls are asynchronous on the given HIP stream (0 = legacy default stream) and
 *     allocate nothing: a plan owns every table and workspace it needs (set-up calls -
 *     ht_plan_create, ht_plan_set_precision, ht_plan_reserve_exact_gcv, ht_batch_create,
 *     ht_mlp_create - allocate and may block).
 *   - Arguments are validated on the host before anything is launched; on error nothing
 *     is launched and a status other than HT_OK is returned.  ht_last_error() returns a
 *     thread-local message describing the most recent failure.  No exception crosses the
 *     ABI.  With batch = 0 a call validates its sizes, launches nothing and returns
 *     HT_OK; its array arguments may then be NULL.
 *   - Signals are real float64.  Coefficient vectors ("coeff"), filtered coefficients and
 *     eigenvalues d are float64 for the real kinds (AR, C, DST2, DST3, R) and interleaved
 *     complex128 (re, im) for the kinds F, P and F3.  Coefficients are ordered like the
 *     columns of T: [first polynomial column, the n-2 core columns, last polynomial
 *     column]; for the comparators P and R, the n core columns.
 *   - A batch of 1D signals is a contiguous [batch][n] array; a batch of images is
 *     [batch][n0][n1], row-major, coefficients in the same layout.
 *   - PSF convention: psf[idx] is the tap h_{idx - center}; the blur is the convolution
 *     g_i = sum_j h_j f_{i-j} (the PSF is the blur of a single pixel, Section 1).
 */
#ifndef HT_H
#define HT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HT_OK = 0,
    HT_ERR_INVALID_ARG = 1,   /* null pointer, size out of range, bad enum value          */
    HT_ERR_UNSUPPORTED = 2,   /* e.g. a nonsymmetric PSF with a degree that needs symmetry */
    HT_ERR_PSF_TOO_WIDE = 3,  /* 2m+1 > n-2 (eq. jcf requires 2m+1 <= n-2; n for P, R)     */
    HT_ERR_SINGULAR = 4,      /* a boundary capacitance matrix is singular                 */
    HT_ERR_NONFINITE = 5,     /* non-finite data detected                                  */
    HT_ERR_HIP = 6,           /* a HIP runtime call failed                                 */
    HT_ERR_OOM = 7            /* device or host allocation failed (plan creation only)     */
} ht_status;

/* Which transform family realises a boundary degree.
 *  HT_FAMILY_PAPER: degree 1 -> antireflective T (eq. ART, symmetric PSF);
 *                   degree 2 -> T_C (eq. Tc) for a symmetric PSF, T_F (eq. Tf) otherwise.
 *  HT_FAMILY_DST:   degree 1..3 -> the antireflective transform whose lowest degree-1
 *                   sine columns are replaced by polynomial "bubbles" (symmetric PSF);
 *                   degree 1 is identical to the antireflective transform.            */
/*  HT_FAMILY_PAPER_DST3: degrees 1 and 2 as HT_FAMILY_PAPER, degree 3 as HT_FAMILY_DST
 *                   for a symmetric PSF and as HT_KIND_F3 otherwise (the paper defines
 *                   no degree-3 transform of its own).
 *  HT_FAMILY_PERIODIC / HT_FAMILY_REFLECTIVE: the comparators of Section 2.1 (degree 0):
 *                   A_P = F^H diag(d) F (eq. permat, any PSF) and A_R = C^T diag(d) C
 *                   (eq. refm, symmetric PSF), cores of order n with no boundary columns.
 *                   Float64 and float32 cores; not in ragged batches or split precision. */
typedef enum {
    HT_FAMILY_PAPER = 0,
    HT_FAMILY_DST = 1,
    HT_FAMILY_PAPER_DST3 = 2,
    HT_FAMILY_PERIODIC = 3,
    HT_FAMILY_REFLECTIVE = 4
} ht_family;

/* Smoothing operator of eq. mintik: L = I, or the second difference with the same
 * boundary model (eq. L, L_C, L_F; in 2D the Laplacian L0 (x) I + I (x) L1).          */
typedef enum { HT_NORM_IDENTITY = 0, HT_NORM_SECOND_DIFF = 1 } ht_norm;

/* What a plan resolved to (per axis). */
typedef enum {
    HT_KIND_AR = 1, HT_KIND_C = 2, HT_KIND_F = 3, HT_KIND_DST2 = 4, HT_KIND_DST3 = 5,
    HT_KIND_P = 6,  /* periodic: unitary DFT of order n (eq. permat)        */
    HT_KIND_R = 7,  /* reflective: orthonormal DCT-II of order n (eq. refm) */
    HT_KIND_F3 = 8  /* degree 3, any PSF: T_F with its frequency +-1 pair replaced by the
                       real columns sqrt(2/N) cos x (eigenvalue Re z(x_1)) and the unit-norm
                       cubic x (x - pi)(x - 2 pi) (eigenvalue z(0)); complex coefficients,
                       real on those two columns for real signals; inverse = the T_F
                       inverse plus a rank-2 float64 correction.  Not in ragged batches,
                       split precision, ht_eigs2d or ht_gcv_scan_exact.                */
} ht_kind;

typedef struct ht_plan ht_plan;

/* Create a plan for signals of length n[0] (ndim = 1) or images n[0] x n[1] (ndim = 2).
 *   degree         preserved polynomial degree (1..3, see ht_family)
 *   psf_symmetric  nonzero if h_{-j} = h_j (selects T_C over T_F for degree 2)
 *   family         ht_family
 *   max_batch      number of images (2D) one call may process, sizing the plan's
 *                  workspace; in 1D it bounds the signals per call only for the
 *                  split-precision core (ht_plan_set_precision) and is otherwise ignored
 * Lengths must satisfy 5 <= n <= 8192.  The plan owns all device tables (boundary
 * vectors and 2x2 solves of Theorem th:inv in closed form, chirp and filter-spectrum
 * tables of the core transform, trigonometric tables of the exactly reduced angles).
 * Returns HT_ERR_UNSUPPORTED for combinations the paper does not define (degree 3 in
 * HT_FAMILY_PAPER, a nonsymmetric PSF with the antireflective or DST family).        */
ht_status ht_plan_create(int ndim, const int64_t* n /* host [ndim] */, int degree,
                         int psf_symmetric, int family, int64_t max_batch, ht_plan** out);
ht_status ht_plan_destroy(ht_plan* plan);
/* Kind of axis `axis` (0 or 1), or -1 on a bad argument. */
int ht_plan_kind(const ht_plan* plan, int axis);
/* 1 if coefficients / eigenvalues are complex128 (kinds F, P, F3), else 0. */
int ht_plan_is_complex(const ht_plan* plan);

/* Arithmetic of the core transform inside ht_transform_inv / ht_transform_fwd.
 *   HT_PRECISION_F64     float64 chirp-z FFT core (default).
 *   HT_PRECISION_BF16X3  the core as a dense GEMM on the matrix cores: the core matrix
 *                        (A_inv = inverse of the interior core block, A_fwd = the core
 *                        columns of T on the whole grid) and the vectors are each split
 *                        x = x_hi + x_lo into two bfloat16 parts, and the product is
 *                        A_hi B_hi + A_hi B_lo + A_lo B_hi accumulated in float32.
 *   HT_PRECISION_F16X3   the same with float16 parts and a power-of-two scale per row.
 *   HT_PRECISION_F32     the chirp-z FFT core in float32 (tables rounded from the float64
 *                        ones), any kind including T_F; the interior correction is rounded
 *                        to float32 on entry to the core, the result widened on exit.
 * The 2x2 boundary solve, the interior correction, the boundary columns of the forward
 * transform and all inputs and outputs stay float64.  Relative error of one 1D pass is
 * of order 2^-16 (bfloat16), 2^-21 (float16) or 2^-20 (float32 core) of the vector's
 * norm instead of 2^-52.                                                                */
typedef enum {
    HT_PRECISION_F64 = 0,
    HT_PRECISION_BF16X3 = 1,
    HT_PRECISION_F16X3 = 2,
    HT_PRECISION_F32 = 3
} ht_precision;

/* ht_plan_set_precision -- choose the core arithmetic of `plan` (ht_precision).  The
 * split-precision cores need real cores on every axis (T_C, antireflective, DST family;
 * HT_ERR_UNSUPPORTED for T_F) and the plan's device current.  Builds the dense split
 * core matrices (2 n^2 x 4 bytes per axis) and a workspace for max_batch signals or
 * images, or the float32 tables; blocking (synchronises the device).  Not to be called
 * while the plan is in use on a stream.  HT_PRECISION_F64 releases them.               */
ht_status ht_plan_set_precision(ht_plan* plan, int precision);
/* The plan's ht_precision, or -1 for a null plan. */
int ht_plan_precision(const ht_plan* plan);

/* ht_eigs -- eigenvalues d of the blurring matrix and s of the smoothing operator in the
 * plan's basis (eqs. jcf, Ac, Af; L_A, L_C, L_F of Section 4), computed from the PSF by
 * direct summation of z at exactly reduced angles.  The preserved-polynomial columns get
 * d = z(0) = sum_j h_j and s = 0 (s = 1 for L = I).
 *   1D: psf [batch][psf_len[0]] (device), d [batch][n], s [batch][n].
 *   2D: psf = [h0 (psf_len[0]) | h1 (psf_len[1])], a separable PSF h0 (x) h1; outputs are
 *       the 1D factors d = [d0 (n0) | d1 (n1)], s = [s0 (n0) | s1 (n1)] with
 *       d_ij = d0_i d1_j and s_ij = s0_i + s1_j (for L = I: s0 = 1, s1 = 0).  batch = 1.
 *   psf_len, psf_center: host arrays [ndim].  Requires 2m+1 <= n-2 per axis (2m+1 <= n
 *   for the comparators, whose core has order n), with m = max(center, len-1-center)
 *   (HT_ERR_PSF_TOO_WIDE otherwise).  The comparators have no polynomial columns: d is
 *   z on the grid 2 pi k/n (P, conjugated for the convolution model) or pi k/n (R), and
 *   s = 2 - 2 cos on the same grid.  For the real kinds
 *   the mask is used through Re z(t), i.e. its even part.                              */
ht_status ht_eigs(const ht_plan* plan, const double* psf, const int64_t* psf_len,
                  const int64_t* psf_center, int norm, void* d, double* s, int64_t batch,
                  hipStream_t stream);

/* ht_eigs2d -- eigenvalues for a general (non-separable) 2D PSF mask on a 2D plan, by
 * the three steps of Section 6: the marginal 1D masks (the sums of the columns and of the
 * rows of the mask) give the entries whose index along one axis is a preserved
 * polynomial column (the edges of the array; the corners get the mask's sum), and the 2D
 * transform of the mask at the grid frequencies of both axes gives the inner entries.
 * Computed as one formula: polynomial columns have frequency 0, where the 2D sum reduces
 * to the marginal's 1D sum.  Real kinds use the part of the mask even in each axis,
 * sum H[a,b] cos((a-c0) t_i) cos((b-c1) u_j) (the eigen relation needs a mask even in
 * each axis, e.g. a disk); T_F uses the 2D symbol at (-t_i, -u_j) (any mask, e.g. motion
 * blur).  Direct sums with exactly reduced angles, O(len0 n1 len1 + n0 n1 len0) per mask.
 *   psf: device [batch][len0][len1], tap (a, b) at offset (a - center0, b - center1).
 *   d: device [batch][n0][n1] (complex128 for T_F plans, else float64); s: [batch][n0][n1]
 *   with s_ij = s0_i + s1_j for HT_NORM_SECOND_DIFF (0 on polynomial columns), 1 for
 *   HT_NORM_IDENTITY.  The HT_SPECTRUM_FULL layout of ht_tikhonov_filter / ht_gcv_scan.
 *   1 <= batch <= the plan's max_batch; 2m+1 <= n-2 (n for P, R) per axis, m = max(center,
 *   len-1-center) (HT_ERR_PSF_TOO_WIDE).  Uses the plan's 2D workspace: calls on one plan
 *   must be ordered on one stream, as for its transforms.                               */
ht_status ht_eigs2d(const ht_plan* plan, const double* psf, int64_t psf_len0, int64_t psf_len1,
                    int64_t psf_center0, int64_t psf_center1, int norm, void* d, double* s,
                    int64_t batch, hipStream_t stream);

/* Layout of the spectra d and s of a 2D plan for ht_tikhonov_filter / ht_gcv_scan (1D
 * plans ignore it: their spectra are [eig_batch][n]).                                  */
typedef enum {
    HT_SPECTRUM_FACTORS = 0,  /* [d0 (n0) | d1 (n1)], [s0 | s1] of ht_eigs (separable mask) */
    HT_SPECTRUM_FULL = 1      /* [eig_batch][n0][n1] of ht_eigs2d (any mask)                */
} ht_spectrum_layout;

/* ht_transform_inv -- coeff = T^{-1} signal (Theorem th:inv): the 2x2 boundary system in
 * float64, the interior correction, one core analysis transform (DST-I, DCT-II or DFT of
 * order n-2) and, for DST2/DST3, the rank-(degree-1) correction.  In 2D the 1D transform
 * runs along axis 1 then axis 0 (Section 6).  signal and coeff must not overlap.  With
 * a split-precision core (ht_plan_set_precision) batch must not exceed max_batch.      */
ht_status ht_transform_inv(const ht_plan* plan, const double* signal, void* coeff,
                           int64_t batch, hipStream_t stream);

/* ht_transform_fwd -- signal = T coeff (the direct transform).  For kind F the result of
 * a Hermitian coefficient vector (the image of a real signal under T^{-1}, or any vector
 * the filter produces from one) is real; the library returns its real part.          */
ht_status ht_transform_fwd(const ht_plan* plan, const void* coeff, double* signal,
                           int64_t batch, hipStream_t stream);

/* ht_tikhonov_filter -- fhat_i = conj(d_i) coeff_i / (|d_i|^2 + mu |s_i|^2), i.e.
 * Phi D^{-1} coeff of eq. freg (reblurred Tikhonov, eq. nerebl), in float64.
 *   d, s: eig_batch = 1 (shared by every item) or eig_batch = batch (one per item); 2D
 *   plans: layout (ht_spectrum_layout) HT_SPECTRUM_FACTORS takes eig_batch = 1.
 *   mu:   device [batch], mu > 0.  fhat may alias coeff.                               */
ht_status ht_tikhonov_filter(const ht_plan* plan, const void* coeff, const void* d,
                             const double* s, int64_t eig_batch, int layout, const double* mu,
                             void* fhat, int64_t batch, hipStream_t stream);

/* ht_gcv_scan -- G(mu_k) = sum_i |sigma_i coeff_i|^2 / (sum_i sigma_i)^2 with
 * sigma_i = |s_i|^2 / (|d_i|^2 + mu_k |s_i|^2) (eqs. gcv2, mugcv) for every mu_k of the
 * grid, and the index of its first minimum.  Sums are float64 in a fixed order, so the
 * result is bitwise reproducible run to run.  d, s, eig_batch, layout as for
 * ht_tikhonov_filter.
 *   mu_grid: device [K] (grid_per_item = 0) or [batch][K] (grid_per_item = 1), mu_k > 0.
 *   G: device [batch][K] or NULL.  k_best: device int32 [batch] (-1 if some G_k is not
 *   finite).  mu_best: device [batch] or NULL (NaN when k_best = -1).  1 <= K <= 1024.  */
ht_status ht_gcv_scan(const ht_plan* plan, const void* coeff, const void* d, const double* s,
                      int64_t eig_batch, int layout, const double* mu_grid, int32_t K, int grid_per_item,
                      double* G, int32_t* k_best, double* mu_best, int64_t batch,
                      hipStream_t stream);

/* ht_gcv_scan_exact -- the exact GCV functional of eq. gcv,
 * G(mu_k) = ||T (sigma ghat)||^2 / (sum_i sigma_i)^2, i.e. ||g - A f_reg||^2 /
 * trace(I - A T Phi D^{-1} T^{-1})^2 with the factors mu^2 cancelled (the residual is
 * T (I - Phi) ghat and the trace sum_i (1 - Phi_i)), on the same scale as ht_gcv_scan,
 * which uses the approximation ||T v|| ~ ||v|| of eq. gcnum.  Arguments as for
 * ht_gcv_scan.  Float64 sums in a fixed order.
 *   1D plans: ||T v||^2 from T's structure (orthonormal core plus boundary columns and
 *   ghost rows): the sums of ht_gcv_scan plus up to four weighted sums of sigma_i ghat_i
 *   with fixed vectors; allocates nothing.
 *   2D plans: ||T0 V T1^T||^2 from the same structure of both axes: the 1D form of every
 *   interior row plus the axis-0 boundary terms, built from the rows' functionals and the
 *   weighted column sums of V (a row pass, a column pass and a combination per grid
 *   value, images in chunks that fit the plan's workspace); batch <= max_batch and K at
 *   most the grid size reserved for the plan (128 unless ht_plan_reserve_exact_gcv
 *   reserved more); allocates nothing.  Calls on one plan must be ordered on one stream
 *   (they share its workspace).
 *   The periodic and reflective comparators are unitary: eq. gcv is eq. gcv2 (1D plans
 *   run ht_gcv_scan).  HT_ERR_UNSUPPORTED for HT_KIND_F3.                               */
ht_status ht_gcv_scan_exact(const ht_plan* plan, const void* coeff, const void* d, const double* s,
                            int64_t eig_batch, int layout, const double* mu_grid, int32_t K,
                            int grid_per_item, double* G, int32_t* k_best, double* mu_best,
                            int64_t batch, hipStream_t stream);

/* ht_gcv_scan_exact_static -- ht_gcv_scan_exact with its 2D workspace in a fixed 64 MiB
 * device array of the library instead of the plan's workspace: for callers that cannot
 * allocate or rely on a per-plan reservation (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and error behaviour;
 * K may be up to 1024 regardless of ht_plan_reserve_exact_gcv, but one image's row-pass
 * outputs and partials (about n0 K 22 doubles plus 44 K ceil((n1-2)/64) doubles), plus
 * K batch doubles when G is NULL, must fit the 2^23 doubles: otherwise
 * HT_ERR_INVALID_ARG before any launch.  Allocates nothing (hipMalloc is never called; the
 * array's device address is looked up once per device, at ht_plan_create).  Every call on
 * one GPU shares that GPU's array, so calls that overlap on one GPU (different streams or
 * threads) race: order them on one stream.  1D plans and the comparators delegate to
 * ht_gcv_scan_exact, which needs no workspace.  The plan's device must be current.     */
ht_status ht_gcv_scan_exact_static(const ht_plan* plan, const void* coeff, const void* d, const double* s,
                                   int64_t eig_batch, int layout, const double* mu_grid, int32_t K,
                                   int grid_per_item, double* G, int32_t* k_best, double* mu_best,
                                   int64_t batch, hipStream_t stream);

/* ht_plan_reserve_exact_gcv -- size the workspace of ht_gcv_scan_exact on a 2D plan for
 * grids of up to max_k values (1..1024): row-pass outputs for a chunk of images (at most
 * 256 MiB, at least one image: n0 max_k 22 doubles per image), column-pass partials for
 * the same chunk and max_k doubles of G per image.  ht_plan_create reserves max_k = 128;
 * a call with a larger K than reserved returns HT_ERR_INVALID_ARG.  Set-up call:
 * synchronises the device; no-op for 1D plans, the comparators and a max_k already
 * reserved.                                                                           */
ht_status ht_plan_reserve_exact_gcv(ht_plan* plan, int32_t max_k);

/* ---------------------------------------------------------------------------------
 * Ragged batches: many 1D signals of uneven length n_b, each with its own PSF mask,
 * boundary degree and mu grid, restored end to end (eigenvalues, inverse transform, GCV
 * choice of mu over the signal's grid, filter, forward transform; Sections 2-4) by
 * persistent fused kernels, one per FFT size class, that take signals from a
 * longest-first queue.  Symmetric PSFs only (real transforms: AR, C, DST2, DST3).
 * Every call is asynchronous, allocates nothing and may be captured in a HIP graph.
 * --------------------------------------------------------------------------------- */
typedef struct ht_batch ht_batch;

/* Describe a batch (host arrays of length count): signal lengths n[b] in [5, 8192],
 * degree[b] / psf_symmetric[b] resolved per `family` as for ht_plan_create, and the
 * shape of each PSF mask (psf_len[b], psf_center[b]; 2m+1 <= n-2).  Builds the tables of
 * every distinct (n, kind) once.  Signals are concatenated in item order (offsets are
 * the prefix sums of n), masks likewise (prefix sums of psf_len).  A signal's size class
 * is the smallest FFT length (a power of two >= 512) its core transform needs: N + 2 for
 * a half-length real core (core real-DFT length even: N for T_C, N + 1 for the sine
 * cores), N + (N+1)/2 - 1 for the half-output cosine core (N odd), 2N - 1 for the
 * chirp-z core, whichever is shortest (N = n - 2).                                    */
ht_status ht_batch_create(int64_t count, const int64_t* n, const int* degree,
                          const int* psf_symmetric, int family, const int64_t* psf_len,
                          const int64_t* psf_center, ht_batch** out);
ht_status ht_batch_destroy(ht_batch* batch);
/* sum of n[b] (length of the signal and restored arrays), or -1 */
int64_t ht_batch_total_length(const ht_batch* batch);
/* sum of psf_len[b] (length of the PSF array), or -1 */
int64_t ht_batch_psf_total(const ht_batch* batch);
/* number of signals, or -1 */
int64_t ht_batch_count(const ht_batch* batch);

/* ht_batch_restore -- for every signal b: d, s on its grid, ghat = T^{-1} g,
 * G_b(mu_{b,k}) for k < K (eq. mugcv), k_b = first argmin, f = T Phi D^{-1} ghat at
 * mu_{b,k_b} (eq. freg).
 *   signal [total_length], psf [psf_total], mu_grid [count][K] (one grid per signal,
 *   mu > 0), restored [total_length] (must not overlap signal), G [count][K] or NULL,
 *   k_best int32 [count] (-1 if some G is not finite; the restoration is then NaN),
 *   mu_best [count].  1 <= K <= 256.  The sums of G are float64 in a fixed order.   */
ht_status ht_batch_restore(const ht_batch* batch, const double* signal, const double* psf,
                           int norm, const double* mu_grid, int32_t K, double* restored,
                           double* G, int32_t* k_best, double* mu_best, hipStream_t stream);

/* Schedule knobs (set by the autotuner) of size class `size_class` (0..5: FFT lengths
 * 512, 1024, 2048, 4096, 8192, 2 x 8192): the number of persistent workgroups (<= 0:
 * unchanged; capped at the class size, and at 1024 for class 5) and the kernel variant
 * (-1: unchanged; 0: 8 points per thread, 1: 16 points per thread, classes 3..5 only).
 * The values in effect are returned through the non-NULL pointers.  Results do not depend
 * on the schedule.                                                                   */
ht_status ht_batch_schedule(ht_batch* batch, int size_class, int workgroups, int variant,
                            int* cur_workgroups, int* cur_variant);
/* Tuning aid: restrict ht_batch_restore to the size classes whose bit is set in `mask`
 * (bit c = class c; default all six).  Signals of the other classes are left untouched.
 * Used to time one class at a time; a batch used for results keeps the full mask.     */
ht_status ht_batch_class_mask(ht_batch* batch, unsigned mask);
/* number of signals in a size class, or -1 */
int ht_batch_class_count(const ht_batch* batch, int size_class);

/* ---------------------------------------------------------------------------------
 * Learned mu: a small network predicts log10(mu) from statistics of the transform
 * coefficients and the blur spectrum; the GCV functional certifies the prediction and
 * the full scan is the fallback.  Not in the paper: an accelerator of its GCV step.
 * --------------------------------------------------------------------------------- */

/* ht_batch_features -- for every signal: ghat = T^{-1} g (written to coeff [total_length],
 * ordered as the coefficient vectors of ht_transform_inv) and 72 features
 * (features [count][72], float32): the means of log10(|ghat_j|^2 + 1e-20) over 64 equal
 * bands of the normalised core frequency j/(n-2) (band b holds j with
 * floor(64 j / (n-2)) = b; the two polynomial entries are excluded), then the means of
 * log10(|d_j|^2 + 1e-20) over 8 such bands of the blur eigenvalues (the floor keeps the
 * logarithms well conditioned where the spectrum vanishes; the logarithms are float32).
 * spectrum [total_length] (nullable) receives the blur eigenvalues d in coefficient
 * order, for ht_batch_restore_learned.  Needs n >= 66.                                 */
ht_status ht_batch_features(const ht_batch* batch, const double* signal, const double* psf,
                            double* coeff, float* features, double* spectrum,
                            hipStream_t stream);

/* ht_batch_restore_learned -- coeff_restored holds the coefficients from
 * ht_batch_features on entry and the restorations on exit; spectrum (nullable) is the
 * eigenvalue output of that same call (recomputed from psf when NULL).  For every signal
 * the grid index k^ nearest to pred_log10_mu[b] is certified: G is evaluated on
 * [k^-h, k^+h] (h = cert_half in [1, K-1], clipped to the grid); with k_m its first
 * minimum there, the certificate holds if G(k^) <= 1.05 G(k_m) and k_m is not an
 * interior edge of the bracket, and then mu = mu_{k_m}; otherwise the full grid is
 * scanned (fallback[b] = 1) and mu is the scan's choice.  G [count][K] (nullable)
 * receives the evaluated values only.                                                  */
ht_status ht_batch_restore_learned(const ht_batch* batch, double* coeff_restored,
                                   const double* psf, const double* spectrum, int norm,
                                   const double* mu_grid, int32_t K,
                                   const float* pred_log10_mu, int32_t cert_half,
                                   double* G, int32_t* k_best, double* mu_best,
                                   int32_t* fallback, hipStream_t stream);

/* The network of the learned-mu predictor as device pointers: weights w[l] bfloat16
 * (uint16_t bit patterns) row-major [in][out] for the layers 72 -> 256 -> 256 -> 256 -> 1,
 * biases b[l] float32 [out], feature standardisation mean / std float32 [72].           */
typedef struct {
    const uint16_t* w[4];
    const float* b[4];
    const float* mean;
    const float* std;
} ht_mlp_weights;

/* ht_batch_restore_fused -- the learned-mu restoration in one pass per signal: inverse
 * transform, eigenvalues, the 72 features of ht_batch_features, the network's prediction
 * of log10 mu (exact GELU, bfloat16 rounding of the standardised features and of every
 * hidden activation, float32 accumulation: the rounding points of ht_gemm_bf16 with
 * act = 1 and Cb), then the certificate and fallback of ht_batch_restore_learned, the
 * filter and the forward transform.  restored [total_length] must not overlap signal;
 * pred [count] and features [count][72] (float32) are optional outputs.  Needs n >= 66. */
ht_status ht_batch_restore_fused(const ht_batch* batch, const double* signal, const double* psf,
                                 int norm, const double* mu_grid, int32_t K,
                                 const ht_mlp_weights* net, int32_t cert_half, double* restored,
                                 int32_t* k_best, double* mu_best, int32_t* fallback, float* pred,
                                 float* features, hipStream_t stream);

/* Network kernels (row-major matrices; bfloat16 stored as uint16_t bit patterns):
 * ht_gemm_bf16: C = act(A B + bias), A(i,k) = A[i sa_i + k sa_k], B(k,j) = B[k sb_k + j sb_j]
 *   (bfloat16), float32 accumulation on the matrix cores (operands contiguous along the
 *   contraction, or B contiguous along j, in 16-byte vectors when the strides and sizes
 *   are multiples of 8); act 0 = none, 1 = GELU
 *   0.5 x (1 + erf(x / sqrt 2)); Z (pre-activation), C (activation; rounded to bfloat16
 *   when Cb is also given, so that C and Cb hold the same values) and Cb may each be NULL;
 *   all outputs use leading dimension ldc.
 * ht_to_bf16: dst = bf16((src - mean[col]) / std[col]) (mean, std both NULL: plain).
 * ht_from_bf16: dst = float32 value of the bfloat16 src.
 * ht_gelu_backward: dz = dh * GELU'(z), dzb (nullable) its bfloat16 copy.
 * ht_colsum: out[j] = sum_i X[i][j] (* weight[i] if weight != NULL), fixed order.
 * ht_mse_grad: dy = 2 (y - t) / rows, sq = (y - t)^2.
 * ht_outer: dh[i][j] = dy[i] * w[j].
 * ht_adam: Adam on float32 parameters (bias-corrected, step >= 1); pb (nullable) gets
 *   the bfloat16 copy of the updated parameters.                                      */
ht_status ht_gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sa_i, int64_t sa_k,
                       const uint16_t* B, int64_t sb_k, int64_t sb_j, const float* bias, int act,
                       float* Z, float* C, int64_t ldc, uint16_t* Cb, hipStream_t stream);
ht_status ht_to_bf16(const float* src, uint16_t* dst, int64_t rows, int cols, const float* mean,
                     const float* stdv, hipStream_t stream);
ht_status ht_from_bf16(const uint16_t* src, float* dst, int64_t count, hipStream_t stream);
ht_status ht_gelu_backward(const float* z, const float* dh, float* dz, uint16_t* dzb,
                           int64_t count, hipStream_t stream);
ht_status ht_colsum(const float* X, int64_t rows, int cols, const float* weight, float* out,
                    hipStream_t stream);
ht_status ht_mse_grad(const float* y, const float* t, float* dy, float* sq, int64_t rows,
                      hipStream_t stream);
ht_status ht_outer(const float* dy, const float* w, float* dh, int64_t rows, int cols,
                   hipStream_t stream);
/* ht_transpose_bf16: dst[c][r] = src[r][c] for a [rows][cols] bfloat16 matrix (dst must not
 * overlap src).                                                                       */
ht_status ht_transpose_bf16(const uint16_t* src, uint16_t* dst, int rows, int cols, hipStream_t stream);
ht_status ht_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr,
                  float beta1, float beta2, float eps, int64_t step, uint16_t* pb,
                  hipStream_t stream);

/* ---------------------------------------------------------------------------------
 * The learned-mu predictor as a library object (the network above with its weights,
 * Adam state, feature standardisation and activation buffers).  Created once; every
 * other call launches kernels only (no allocation), asynchronously on the stream.  Calls
 * on one network must be ordered on one stream (they share its buffers).  Not in the
 * paper: an accelerator of the GCV choice of mu of Section 4 (eq. mugcv), trained on
 * problems the method labels itself.
 * Parameters are one float32 vector of ht_mlp_param_count() = 150529 entries:
 * W1 [72][256], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256], W4 [256][1],
 * b4 [1]; W row-major [in][out].
 * --------------------------------------------------------------------------------- */
typedef struct ht_mlp ht_mlp;

int64_t ht_mlp_param_count(void);

/* ht_mlp_create -- allocate a network for minibatches / prediction chunks of up to
 * max_rows rows (1 <= max_rows <= 2^24) on the current device: parameters and Adam
 * moments zero, standardisation mean 0 / std 1.  HT_ERR_OOM if the allocation fails.   */
ht_status ht_mlp_create(int64_t max_rows, ht_mlp** out);
ht_status ht_mlp_destroy(ht_mlp* mlp);

/* ht_mlp_set_params -- copy params (device float32 [150529]) into the network and refresh
 * its bfloat16 copies.                                                                  */
ht_status ht_mlp_set_params(ht_mlp* mlp, const float* params, hipStream_t stream);

/* ht_mlp_get -- copy one of the network's vectors into out (device float32): the
 * parameters, the gradients of the last backward pass, the Adam moments ([150529] each),
 * or the standardisation mean / std ([72]).                                             */
typedef enum {
    HT_MLP_PARAMS_VEC = 0, HT_MLP_GRADS_VEC = 1, HT_MLP_ADAM_M_VEC = 2, HT_MLP_ADAM_V_VEC = 3,
    HT_MLP_MEAN_VEC = 4, HT_MLP_STD_VEC = 5
} ht_mlp_vector;
ht_status ht_mlp_get(const ht_mlp* mlp, int which, float* out, hipStream_t stream);

/* ht_mlp_set_state -- restore Adam moments (adam_m, adam_v: device [150529], both or
 * neither), the Adam step count, and the standardisation (mean, std: device [72], both or
 * neither).                                                                            */
ht_status ht_mlp_set_state(ht_mlp* mlp, const float* adam_m, const float* adam_v, int64_t steps,
                           const float* mean, const float* std, hipStream_t stream);
/* Adam steps taken so far, or -1 for a null network. */
int64_t ht_mlp_steps(const ht_mlp* mlp);

/* ht_mlp_fit_standardisation -- per-feature mean and population standard deviation
 * (floored at 1e-6) of features (device float32 [rows][72]), float64 sums in a fixed
 * order; the network standardises its inputs with them from then on.                  */
ht_status ht_mlp_fit_standardisation(ht_mlp* mlp, const float* features, int64_t rows,
                                     hipStream_t stream);

/* ht_mlp_forward -- pred[r] (float32, device, nullable: the network keeps its own copy
 * for ht_mlp_backward) = the network at the standardised features[r] (device float32
 * [rows][72]): standardised inputs and every hidden activation rounded to bfloat16, exact
 * GELU, float32 accumulation.  1 <= rows <= max_rows.                                  */
ht_status ht_mlp_forward(ht_mlp* mlp, const float* features, int64_t rows, float* pred,
                         hipStream_t stream);

/* ht_mlp_predict -- pred[r] (device float32 [rows], required) = the network at features[r]
 * as ht_mlp_forward computes it, for any rows >= 0 (chunks of max_rows); keeps no
 * activations for a backward pass (ht_mlp_backward is refused until the next
 * ht_mlp_forward), so it writes only what the next layer reads.                         */
ht_status ht_mlp_predict(ht_mlp* mlp, const float* features, int64_t rows, float* pred, hipStream_t stream);

/* ht_mlp_backward -- gradients of the mean squared error mean_r (pred_r - target_r)^2 of
 * the last ht_mlp_forward (same rows) with respect to every parameter, kept in the
 * network (read with ht_mlp_get); the pre-activation gradients are rounded to bfloat16
 * before the products that consume them.  loss (device float32 [1], nullable) receives the
 * mean squared error (float64 sum in a fixed order).                                    */
ht_status ht_mlp_backward(ht_mlp* mlp, const float* target, int64_t rows, float* loss,
                          hipStream_t stream);

/* ht_mlp_adam_step -- one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias corrected by
 * the network's step count, which this call increments on the host: a captured graph
 * would replay one fixed step) on every parameter with the current gradients, then the
 * bfloat16 copies.  lr > 0.                                                             */
ht_status ht_mlp_adam_step(ht_mlp* mlp, float lr, hipStream_t stream);

/* ht_mlp_train_step -- one minibatch step: rows r of the minibatch are features[idx[r]]
 * and target[idx[r]] (features device float32 [*][72], target device float32 [*], idx
 * device int32 [rows], every index valid for the caller's arrays), gathered on the
 * device; then forward, backward and an Adam step as above.  loss as for ht_mlp_backward.
 * 1 <= rows <= max_rows.                                                                */
ht_status ht_mlp_train_step(ht_mlp* mlp, const float* features, const float* target, const int32_t* idx,
                            int64_t rows, float lr, float* loss, hipStream_t stream);

/* ht_mlp_weights_of -- the network as ht_mlp_weights (device pointers into the network,
 * valid until it is destroyed) for ht_batch_restore_fused.                             */
ht_status ht_mlp_weights_of(const ht_mlp* mlp, ht_mlp_weights* out);

/* ht_log10_labels -- labels[i] = float32(log10(mu[i])) (mu device float64 [count], e.g.
 * the mu_best of ht_batch_restore: the GCV-optimal mu that labels a training problem).  */
ht_status ht_log10_labels(const double* mu, float* labels, int64_t count, hipStream_t stream);

/* ht_lambda_predict -- predicted log10 mu for every signal of a ragged batch:
 * ht_batch_features (coeff [total_length], features [count][72], spectrum nullable) then
 * the network on the features in chunks of max_rows rows; pred device float32 [count].
 * The result feeds ht_batch_restore_learned.                                           */
ht_status ht_lambda_predict(const ht_batch* batch, ht_mlp* mlp, const double* signal, const double* psf,
                            double* coeff, float* features, double* spectrum, float* pred,
                            hipStream_t stream);

const char* ht_status_str(ht_status status);
const char* ht_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HT_H */
