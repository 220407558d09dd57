// Ragged batches: thousands of 1D signals of uneven length, each with its own PSF, boundary
// degree and mu grid, restored by one persistent fused kernel per FFT size class (the
// kernel is in batch_kernel.h).  Host side: tables of every distinct (n, kind), the
// longest-first queues per size class, the schedule, the entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "batch_kernel.h"
#include "plan_build.h"

namespace ht {
__global__ void k_reset_counters(int* c) {
    if (threadIdx.x < NCLASS * NSEG) c[threadIdx.x] = 0;
}
}  // namespace ht

using namespace ht;

struct ht_batch {
    int64_t count = 0;
    int device = 0;
    const double2* tw = nullptr;
    void* arena = nullptr;          // axis tables
    Axis* d_axes = nullptr;
    RSig* d_sigs = nullptr;
    int* d_counters = nullptr;      // [NCLASS][NSEG] queue heads
    int* d_seg = nullptr;           // [NCLASS][NSEG + 1] segment offsets within each class
    double* d_scratch = nullptr;    // split class: MAX_N doubles per persistent workgroup
    int64_t total_n = 0, total_psf = 0;
    int class_start[NCLASS] = {0};
    int class_count[NCLASS] = {0};
    int grid[NCLASS] = {0};         // persistent workgroups per class (schedule)
    int variant[NCLASS] = {0};      // 0: 8 points per thread, 1: 16 (FFT lengths >= 4096 only)
    unsigned class_mask = (1u << NCLASS) - 1;  // size classes ht_batch_restore runs
    int64_t min_n = 0;
};

namespace {

constexpr int SPLIT_MAX_GRID = 1024;  // persistent workgroups of the split class (scratch rows)

int class_logp(int c) { return c == 5 ? 13 : MIN_LOGP + c; }
bool is_split(int c) { return c == 5; }
bool has_variant(int c) { return class_logp(c) >= 12; }

int full_grid(int cls, int variant, int device) { return batch_full_grid(cls, variant, device); }

void launch_any(const RaggedArgs& a, int mode, int c, int variant, int start, int cnt, int grid, hipStream_t stream) {
    if (mode == MODE_FEATURES)
        batch_launch_features(a, c, variant, start, cnt, grid, stream);
    else if (mode == MODE_LEARNED)
        batch_launch_learned(a, c, variant, start, cnt, grid, stream);
    else if (mode == MODE_LEARNED_RC)
        batch_launch_learned_rc(a, c, variant, start, cnt, grid, stream);
    else if (mode == MODE_FUSED)
        batch_launch_fused(a, c, variant, start, cnt, grid, stream);
    else
        batch_launch_scan(a, c, variant, start, cnt, grid, stream);
}

ht_status run_classes(const ht_batch* bt, const RaggedArgs& a_in, int mode, hipStream_t stream) {
    RaggedArgs a = a_in;
    a.seg = bt->d_seg;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, stream, bt->d_counters);
    ht_status st = check_hip(hipGetLastError(), "batch counter reset");
    if (st != HT_OK) return st;
    // largest class first: its signals dominate the run time
    for (int c = NCLASS - 1; c >= 0; --c) {
        const int cnt = bt->class_count[c];
        if (cnt == 0 || !(bt->class_mask & (1u << c))) continue;
        launch_any(a, mode, c, bt->variant[c], bt->class_start[c], cnt, bt->grid[c], stream);
        st = check_hip(hipGetLastError(), "batch launch");
        if (st != HT_OK) return st;
    }
    return HT_OK;
}

}  // namespace

extern "C" ht_status ht_batch_create(int64_t count, const int64_t* n, const int* degree, const int* psf_symmetric,
                                     int family, const int64_t* psf_len, const int64_t* psf_center, ht_batch** out) {
    if (!out) return fail(HT_ERR_INVALID_ARG, "ht_batch_create: null output");
    *out = nullptr;
    if (count < 1 || count > (1LL << 24)) return fail(HT_ERR_INVALID_ARG, "ht_batch_create: count must be in [1, 2^24]");
    if (!n || !degree || !psf_symmetric || !psf_len || !psf_center)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_create: null argument");
    std::vector<int> kind(count);
    for (int64_t b = 0; b < count; ++b) {
        if (n[b] < 5 || n[b] > MAX_N) return fail(HT_ERR_INVALID_ARG, "ht_batch_create: n must be in [5, 8192]");
        ht_status st;
        kind[b] = resolve_kind(degree[b], psf_symmetric[b], family, &st);
        if (st != HT_OK) return st;
        if (kind[b] == HT_KIND_F || kind[b] == HT_KIND_P || kind[b] == HT_KIND_R || kind[b] == HT_KIND_F3)
            return fail(HT_ERR_UNSUPPORTED,
                        "ht_batch_create: ragged batches take the boundary transforms of real kinds (AR, C, DST)");
        const int64_t len = psf_len[b], c = psf_center[b];
        if (len < 1 || c < 0 || c >= len) return fail(HT_ERR_INVALID_ARG, "ht_batch_create: bad PSF length or center");
        const int64_t m = std::max(c, len - 1 - c);
        if (2 * m + 1 > n[b] - 2) return fail(HT_ERR_PSF_TOO_WIDE, "ht_batch_create: PSF half-width m needs 2m+1 <= n-2");
    }
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(HT_ERR_HIP, "ht_batch_create: no HIP device");
    ht_status st;
    const double2* tw = device_twiddles(device, &st);
    if (!tw) return st;

    // distinct (n, kind) pairs share one set of tables
    std::map<std::pair<int, int>, int> ids;
    std::vector<std::pair<int, int>> keys;
    std::vector<int> axis_of(count);
    for (int64_t b = 0; b < count; ++b) {
        const auto key = std::make_pair(static_cast<int>(n[b]), kind[b]);
        auto it = ids.find(key);
        if (it == ids.end()) {
            it = ids.emplace(key, static_cast<int>(keys.size())).first;
            keys.push_back(key);
        }
        axis_of[b] = it->second;
    }
    const int64_t nax = static_cast<int64_t>(keys.size());
    std::vector<HostAxis> hs(nax);
    std::vector<ht_status> status(nax, HT_OK);
    {
        std::atomic<int64_t> next(0);
        const int nthr = std::max(1, std::min<int>(static_cast<int>(std::thread::hardware_concurrency()), 32));
        std::vector<std::thread> pool;
        for (int t = 0; t < nthr; ++t)
            pool.emplace_back([&]() {
                for (int64_t a = next++; a < nax; a = next++) status[a] = build_axis(keys[a].first, keys[a].second, hs[a], true);
            });
        for (auto& th : pool) th.join();
    }
    for (int64_t a = 0; a < nax; ++a)
        if (status[a] != HT_OK) return fail(status[a], "ht_batch_create: building the tables of a signal length failed");
    ht_batch* bt = new (std::nothrow) ht_batch();
    if (!bt) return fail(HT_ERR_OOM, "ht_batch_create: host allocation failed");
    bt->count = count;
    bt->device = device;
    bt->tw = tw;
    std::vector<Axis> axes(nax);
    st = upload_axes(hs.data(), nax, &bt->arena, axes.data());
    if (st != HT_OK) {
        delete bt;
        return st;
    }
    for (auto& ax : axes) ax.tw = tw;
    // signal descriptors grouped by size class, longest first within a class
    std::vector<int64_t> off(count), poff(count);
    int64_t acc = 0, pacc = 0;
    for (int64_t b = 0; b < count; ++b) {
        off[b] = acc;
        poff[b] = pacc;
        acc += n[b];
        pacc += psf_len[b];
    }
    bt->total_n = acc;
    bt->total_psf = pacc;
    bt->min_n = *std::min_element(n, n + count);
    std::vector<RSig> sigs(count);
    for (int64_t b = 0; b < count; ++b)
        sigs[b] = RSig{off[b], poff[b], static_cast<int32_t>(psf_len[b]), static_cast<int32_t>(psf_center[b]),
                       axis_of[b], static_cast<int32_t>(b)};
    std::stable_sort(sigs.begin(), sigs.end(), [&](const RSig& x, const RSig& y) {
        const int cx = class_of(axes[x.axis]), cy = class_of(axes[y.axis]);
        if (cx != cy) return cx < cy;
        return axes[x.axis].n > axes[y.axis].n;
    });
    for (int64_t i = 0; i < count; ++i) bt->class_count[class_of(axes[sigs[i].axis])]++;
    for (int c = 1; c < NCLASS; ++c) bt->class_start[c] = bt->class_start[c - 1] + bt->class_count[c - 1];
    for (int c = 0; c < NCLASS; ++c) {
        bt->variant[c] = 0;  // 8 points per thread: the faster variant on MI355X (autotuner)
        bt->grid[c] = std::max(1, std::min(bt->class_count[c], full_grid(c, bt->variant[c], device)));
    }
    bt->grid[5] = std::min(bt->grid[5], SPLIT_MAX_GRID);
    // per class, NSEG contiguous segments of about equal total length.  Only the classes of
    // 4096 points and more (tables of 100-400 KB per length and direction): there the L2
    // copies save HBM traffic (measured: 44-51 % less fetched by the feature and certified
    // passes of those classes, 2-3 % less time); the small classes' short queues lose more
    // to the segments' imbalance than they gain, and keep one queue (segment 0).
    std::vector<int> seg(NCLASS * (NSEG + 1), 0);
    for (int c = 0; c < NCLASS; ++c) {
        const int c0 = bt->class_start[c], cc = bt->class_count[c];
        if (class_logp(c) < 12) {
            for (int s = 1; s <= NSEG; ++s) seg[c * (NSEG + 1) + s] = cc;
            continue;
        }
        double total = 0.0;
        for (int i = 0; i < cc; ++i) total += static_cast<double>(axes[sigs[c0 + i].axis].n);
        double run = 0.0;
        int s = 1;
        for (int i = 0; i < cc && s < NSEG; ++i) {
            run += static_cast<double>(axes[sigs[c0 + i].axis].n);
            while (s < NSEG && run >= total * s / NSEG) seg[c * (NSEG + 1) + s++] = i + 1;
        }
        while (s <= NSEG) seg[c * (NSEG + 1) + s++] = cc;
    }
    bool ok = hipMalloc(&bt->d_axes, sizeof(Axis) * nax) == hipSuccess &&
              hipMalloc(&bt->d_sigs, sizeof(RSig) * count) == hipSuccess &&
              hipMalloc(&bt->d_counters, sizeof(int) * NCLASS * NSEG) == hipSuccess &&
              hipMalloc(&bt->d_seg, sizeof(int) * seg.size()) == hipSuccess;
    if (ok && bt->class_count[5] > 0)  // the split class
        ok = hipMalloc(&bt->d_scratch, sizeof(double) * MAX_N * SPLIT_MAX_GRID) == hipSuccess;
    ok = ok && hipMemcpy(bt->d_axes, axes.data(), sizeof(Axis) * nax, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(bt->d_sigs, sigs.data(), sizeof(RSig) * count, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(bt->d_seg, seg.data(), sizeof(int) * seg.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        ht_batch_destroy(bt);
        return fail(HT_ERR_OOM, "ht_batch_create: device allocation failed");
    }
    *out = bt;
    return HT_OK;
}

extern "C" ht_status ht_batch_destroy(ht_batch* bt) {
    if (!bt) return HT_OK;
    if (bt->arena) (void)hipFree(bt->arena);
    if (bt->d_axes) (void)hipFree(bt->d_axes);
    if (bt->d_sigs) (void)hipFree(bt->d_sigs);
    if (bt->d_counters) (void)hipFree(bt->d_counters);
    if (bt->d_seg) (void)hipFree(bt->d_seg);
    if (bt->d_scratch) (void)hipFree(bt->d_scratch);
    delete bt;
    return HT_OK;
}

extern "C" int64_t ht_batch_total_length(const ht_batch* bt) { return bt ? bt->total_n : -1; }
extern "C" int64_t ht_batch_psf_total(const ht_batch* bt) { return bt ? bt->total_psf : -1; }
extern "C" int64_t ht_batch_count(const ht_batch* bt) { return bt ? bt->count : -1; }

extern "C" ht_status ht_batch_restore_fused(const ht_batch* bt, const double* signal, const double* psf, int norm,
                                            const double* mu_grid, int32_t K, const ht_mlp_weights* net,
                                            int32_t cert_half, double* restored, int32_t* k_best, double* mu_best,
                                            int32_t* fallback, float* pred, float* features, hipStream_t stream) {
    if (!bt) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: null batch");
    if (bt->count == 0) return HT_OK;
    if (!signal || !psf || !mu_grid || !net || !restored || !k_best || !mu_best || !fallback)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: null argument");
    for (int l = 0; l < 4; ++l)
        if (!net->w[l] || !net->b[l]) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: null network weight");
    if (!net->mean || !net->std) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: null standardisation");
    if (signal == restored) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: signal and restored must not overlap");
    if (norm != HT_NORM_IDENTITY && norm != HT_NORM_SECOND_DIFF)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: bad norm");
    if (K < 1 || K > BATCH_MAX_K) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: K must be in [1, 256]");
    if (cert_half < 1 || cert_half >= K)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_fused: cert_half must be in [1, K-1]");
    if (bt->min_n < NFEAT_G + 2) return fail(HT_ERR_UNSUPPORTED, "ht_batch_restore_fused: needs n >= 66 (64 bands)");
    RaggedArgs a{bt->d_axes, bt->d_sigs, bt->d_counters, signal, psf, mu_grid, K, norm, restored, nullptr, k_best,
                 mu_best, bt->d_scratch, nullptr, fallback, features, cert_half, nullptr,
                 {net->w[0], net->w[1], net->w[2], net->w[3]}, {net->b[0], net->b[1], net->b[2], net->b[3]},
                 net->mean, net->std, pred};
    return run_classes(bt, a, MODE_FUSED, stream);
}

extern "C" ht_status ht_batch_schedule(ht_batch* bt, int size_class, int workgroups, int variant,
                                       int* cur_workgroups, int* cur_variant) {
    if (!bt || size_class < 0 || size_class >= NCLASS) return fail(HT_ERR_INVALID_ARG, "ht_batch_schedule: bad argument");
    if (variant >= 0) {
        if (variant > 1 || (variant == 1 && !has_variant(size_class)))
            return fail(HT_ERR_INVALID_ARG, "ht_batch_schedule: variant not available for this size class");
        bt->variant[size_class] = variant;
    }
    if (workgroups > 0) {
        int cap = std::max(1, bt->class_count[size_class]);
        if (is_split(size_class)) cap = std::min(cap, SPLIT_MAX_GRID);
        bt->grid[size_class] = std::max(1, std::min(workgroups, cap));
    }
    if (cur_workgroups) *cur_workgroups = bt->grid[size_class];
    if (cur_variant) *cur_variant = bt->variant[size_class];
    return HT_OK;
}

extern "C" ht_status ht_batch_class_mask(ht_batch* bt, unsigned mask) {
    if (!bt || mask == 0 || mask >= (1u << NCLASS)) return fail(HT_ERR_INVALID_ARG, "ht_batch_class_mask: bad argument");
    bt->class_mask = mask;
    return HT_OK;
}

extern "C" int ht_batch_class_count(const ht_batch* bt, int size_class) {
    if (!bt || size_class < 0 || size_class >= NCLASS) return -1;
    return bt->class_count[size_class];
}

extern "C" ht_status ht_batch_restore(const ht_batch* bt, const double* signal, const double* psf, int norm,
                                      const double* mu_grid, int32_t K, double* restored, double* G,
                                      int32_t* k_best, double* mu_best, hipStream_t stream) {
    if (!bt) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore: null batch");
    if (!signal || !psf || !mu_grid || !restored || !k_best || !mu_best)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore: null argument");
    if (norm != HT_NORM_IDENTITY && norm != HT_NORM_SECOND_DIFF) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore: bad norm");
    if (K < 1 || K > BATCH_MAX_K) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore: K must be in [1, 256]");
    if (signal == restored) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore: signal and restored must not overlap");
    RaggedArgs a{bt->d_axes, bt->d_sigs, bt->d_counters, signal, psf, mu_grid, K, norm, restored, G, k_best, mu_best,
                 bt->d_scratch, nullptr, nullptr, nullptr};
    return run_classes(bt, a, MODE_SCAN, stream);
}

extern "C" ht_status ht_batch_features(const ht_batch* bt, const double* signal, const double* psf, double* coeff,
                                       float* features, double* spectrum, hipStream_t stream) {
    if (!bt) return fail(HT_ERR_INVALID_ARG, "ht_batch_features: null batch");
    if (!signal || !psf || !coeff || !features) return fail(HT_ERR_INVALID_ARG, "ht_batch_features: null argument");
    if (signal == coeff) return fail(HT_ERR_INVALID_ARG, "ht_batch_features: signal and coeff must not overlap");
    if (bt->min_n < NFEAT_G + 2) return fail(HT_ERR_UNSUPPORTED, "ht_batch_features: needs n >= 66 (64 bands)");
    RaggedArgs a{bt->d_axes, bt->d_sigs, bt->d_counters, signal, psf, nullptr, 1, HT_NORM_SECOND_DIFF, coeff, nullptr,
                 nullptr, nullptr, bt->d_scratch, nullptr, nullptr, features, 0, spectrum};
    return run_classes(bt, a, MODE_FEATURES, stream);
}

extern "C" ht_status ht_batch_restore_learned(const ht_batch* bt, double* coeff_restored, const double* psf,
                                              const double* spectrum, int norm, const double* mu_grid, int32_t K,
                                              const float* pred_log10_mu, int32_t cert_half, double* G,
                                              int32_t* k_best, double* mu_best, int32_t* fallback,
                                              hipStream_t stream) {
    if (!bt) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_learned: null batch");
    if (!coeff_restored || !psf || !mu_grid || !pred_log10_mu || !k_best || !mu_best || !fallback)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_learned: null argument");
    if (norm != HT_NORM_IDENTITY && norm != HT_NORM_SECOND_DIFF)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_learned: bad norm");
    if (K < 1 || K > BATCH_MAX_K) return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_learned: K must be in [1, 256]");
    if (cert_half < 1 || cert_half >= K)
        return fail(HT_ERR_INVALID_ARG, "ht_batch_restore_learned: cert_half must be in [1, K-1]");
    RaggedArgs a{bt->d_axes, bt->d_sigs, bt->d_counters, nullptr, psf, mu_grid, K, norm, coeff_restored, G, k_best,
                 mu_best, bt->d_scratch, pred_log10_mu, fallback, nullptr, cert_half, const_cast<double*>(spectrum)};
    return run_classes(bt, a, spectrum ? MODE_LEARNED : MODE_LEARNED_RC, stream);
}
