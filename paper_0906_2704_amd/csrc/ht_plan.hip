// Plan creation: every table the kernels read, computed once on the host in long double
// with exactly reduced angles and uploaded to the device.
//
//   q / p       the preserved-polynomial column: p_i = (1 - (i-1)/(n-1)) normalised to
//               unit norm (eq. ART); q = q~/||q~||, q~_{i+1} = (b - x_i)^2 on the
//               extended grid of eqs. ints/points (T_C) or intn/pointn (T_F)
//   minv        inverse of the 2x2 capacitance system of Theorem th:inv in the form it
//               takes once c_a, c_b are recognised as rows of the core (C: first/last rows
//               of C^T; F: rows N and 1 of F^H):
//                 C: [[q1-q2, -q_{n-1}], [-q_{n-1}, q1-q2]] [x1, xn] = [y1-y2, yn-y_{n-1}]
//                 F: [[q1-q_{n-1}, -q2], [-q2, q1-q_{n-1}]] [x1, xn] = [y1-y_{n-1}, yn-y2]
//   chirp       pre/post factors and filter spectra of the chirp-z form of each core
//   DST family  bubbles, K = Q * bubbles and (E^T K)^{-1}
//   trig        cos / sin (pi r / den) for the eigenvalue grid
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ht_internal.h"
#include "plan_build.h"

namespace ht {

static thread_local std::string g_last_error;

ht_status fail(ht_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

ht_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return HT_OK;
    return fail(HT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

using ld = long double;
static const ld PI_L = 3.141592653589793238462643383279502884L;

// exp(2 pi i r / period), r reduced exactly
static cd cis_exact(int64_t r, int64_t period, ld scale = 1.0L) {
    r %= period;
    if (r < 0) r += period;
    const ld a = 2.0L * PI_L * static_cast<ld>(r) / static_cast<ld>(period);
    return cd(static_cast<double>(scale * cosl(a)), static_cast<double>(scale * sinl(a)));
}

// ---------------------------------------------------------------- global twiddles

const double2* device_twiddles(int device, ht_status* st) {
    static std::mutex mu;
    static std::map<int, double2*> tables;
    std::lock_guard<std::mutex> lock(mu);
    auto it = tables.find(device);
    if (it != tables.end()) {
        *st = HT_OK;
        return it->second;
    }
    std::vector<double2> h(TWN);
    for (int m = 0; m < TWN; ++m) {
        const cd w = cis_exact(-m, TWN);
        h[m] = make_double2(w.real(), w.imag());
    }
    double2* dptr = nullptr;
    if (hipMalloc(&dptr, sizeof(double2) * TWN) != hipSuccess) {
        *st = fail(HT_ERR_OOM, "device twiddle table allocation failed");
        return nullptr;
    }
    if (hipMemcpy(dptr, h.data(), sizeof(double2) * TWN, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dptr);
        *st = fail(HT_ERR_HIP, "device twiddle table upload failed");
        return nullptr;
    }
    tables[device] = dptr;
    *st = HT_OK;
    return dptr;
}

// ------------------------------------------------------------------- host FFT (pow2)

// In-place radix-2 FFT of length M (power of two), forward sign -1, float64 arithmetic
// with long-double twiddles.
static void host_fft(std::vector<cd>& x, int sign) {
    const size_t M = x.size();
    for (size_t i = 1, j = 0; i < M; ++i) {
        size_t bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    std::vector<cd> w(M / 2);
    for (size_t k = 0; k < M / 2; ++k) w[k] = cis_exact(sign * static_cast<int64_t>(k), static_cast<int64_t>(M));
    for (size_t len = 2; len <= M; len <<= 1) {
        const size_t step = M / len;
        for (size_t i = 0; i < M; i += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                const cd u = x[i + k];
                const cd v = x[i + k + len / 2] * w[k * step];
                x[i + k] = u + v;
                x[i + k + len / 2] = u - v;
            }
        }
    }
}

// Chirp-z form of the core transforms (0-based j, k < N):
//   sum_j x_j w^{jk} = c_k sum_j (c_j x_j) conj(c_{k-j}),  c_m = w^{m^2/2}.
// DST-I  (sine core, both directions): w = e^{i pi/(N+1)}, Q_kj = sqrt(2/(N+1)) Im(...)
//        with the index shift (j+1)(k+1) = jk + j + k + 1 folded into pre / post.
// DCT-II (C analysis): X_k = w_k Re(e^{i pi k/(2N)} sum_j x_j e^{i pi jk/N}).
// DCT-III (C synthesis): u_j = Re(sum_k (w_k e^{i pi k/(2N)} x_k) e^{i pi jk/N}).
// DFT (F analysis, e^{-2 pi i jk/N}/sqrt N) and inverse DFT (F synthesis).
static void make_chirp(int kind, bool synthesis, int N, int M, HostChirp& hc) {
    hc.pre.assign(N, cd());
    hc.post.assign(N, cd());
    std::vector<cd> b(N);
    int64_t Pang;
    if (kind == HT_KIND_C) {
        Pang = 4LL * N;
        const ld w0 = sqrtl(1.0L / N), w1 = sqrtl(2.0L / N);
        for (int64_t m = 0; m < N; ++m) {
            const ld wk = m == 0 ? w0 : w1;
            if (!synthesis) {
                hc.pre[m] = cis_exact(m * m, Pang);
                hc.post[m] = cis_exact(m * m + m, Pang, wk);
            } else {
                hc.pre[m] = cis_exact(m * m + m, Pang, wk);
                hc.post[m] = cis_exact(m * m, Pang);
            }
            b[m] = cis_exact(-m * m, Pang);
        }
        hc.mode = MODE_RE;
    } else if (kind == HT_KIND_F) {
        Pang = 2LL * N;
        const int sg = synthesis ? 1 : -1;
        const ld sc = 1.0L / sqrtl(static_cast<ld>(N));
        for (int64_t m = 0; m < N; ++m) {
            hc.pre[m] = cis_exact(sg * m * m, Pang);
            hc.post[m] = cis_exact(sg * m * m, Pang, sc);
            b[m] = cis_exact(-sg * m * m, Pang);
        }
        hc.mode = synthesis ? MODE_RE : MODE_CPLX;
    } else {  // sine core
        Pang = 4LL * (N + 1);
        const ld sc = sqrtl(2.0L / (N + 1));
        for (int64_t m = 0; m < N; ++m) {
            hc.pre[m] = cis_exact(m * m + 2 * m, Pang);
            hc.post[m] = cis_exact(m * m + 2 * m + 2, Pang, sc);
            b[m] = cis_exact(-m * m, Pang);
        }
        hc.mode = MODE_IM;
    }
    std::vector<cd> bc(M, cd());
    for (int m = 0; m < N; ++m) bc[m] = b[m];
    for (int m = 1; m < N; ++m) bc[M - m] = b[m];
    host_fft(bc, -1);
    const double inv = 1.0 / M;
    for (auto& v : bc) v *= inv;
    hc.B.swap(bc);
}

// Chirp-z tables of the plain complex DFT of length L, Y_k = sum_j x_j e^{sign 2 pi i jk/L}
// (unscaled), for an input of nin leading entries of which the first nout outputs are
// kept: pre_j = post_j = e^{sign i pi j^2/L}, b_m = e^{-sign i pi m^2/L} for -nin < m < nout,
// stored circularly in M >= nin + nout - 1 points so that no wrapped term reaches a kept
// output.
static void make_dft_chirp(int L, int sign, int M, int nin, int nout, HostChirp& hc) {
    hc.pre.assign(nin, cd());
    hc.post.assign(nout, cd());
    std::vector<cd> bc(M, cd());
    for (int64_t m = 0; m < std::max(nin, nout); ++m) {
        const cd c = cis_exact(sign * m * m, 2LL * L);
        if (m < nin) hc.pre[m] = c;
        if (m < nout) hc.post[m] = c;
        const cd b = cis_exact(-sign * m * m, 2LL * L);
        if (m < nout) bc[m] = b;
        if (m > 0 && m < nin) bc[M - m] = b;
    }
    host_fft(bc, -1);
    const double inv = 1.0 / M;
    for (auto& v : bc) v *= inv;
    hc.B.swap(bc);
    hc.mode = MODE_CPLX;
}

// Half-length real cores.  Both core transforms are real DFTs of length L (N for the
// cosine core, N + 1 for the sine core) with pre- and post-processing; a real DFT needs
// only its outputs k <= L/2.
//  * Even L (half = 1, H = L/2): a complex DFT of length H of the packed pairs.  The
//    cosine core (Makhoul's reordering v_p = x_{2p}, v_{N-1-p} = x_{2p+1}) turns the
//    DCT-II into X_k = Re(e^{-i pi k/(2N)} V_k) with V the real DFT of v, computed as the
//    complex DFT of u_m = v_{2m} + i v_{2m+1}; the DCT-III is the same steps reversed.  The
//    sine core: with y_t = sin(pi t/L)(x_t + x_{L-t}) + (x_t - x_{L-t})/2 (x_0 = x_L = 0)
//    and Y its real DFT (e^{+}), S_{2k} = Im Y_k and S_{2k+1} = S_{2k-1} + Re Y_k
//    (S_1 = Re Y_0 / 2).  FFT length: the smallest power of two >= N + 2 (>= 2H - 1, and
//    room in LDS for the eigenvalue staging).
//  * Odd L, cosine core only (half = 2, H = (N + 1)/2): the same real DFT taken as a
//    chirp-z transform of length N that keeps only the H outputs the post-processing reads
//    (DCT-II), or reads only the H inputs that are not conjugate mirrors (DCT-III, the real
//    part of a DFT of its first H terms with the k = 0 term not doubled).  FFT length: the
//    smallest power of two >= N + H - 1 instead of >= 2N - 1.  The sine core keeps the
//    full chirp-z core for odd L: its odd outputs are a running sum over about L/2 DFT
//    outputs, whose rounding errors add up to 10-20 times the error of the direct core
//    (float64 emulation against an exact sum), more than the restorations' 1e-12 relative
//    accuracy leaves room for when the filter gain is large.  (The even-L sine form has the
//    same running sum; it is kept, with its measured errors in the tests.)
static ht_status make_half(HostAxis& h) {
    Axis& a = h.ax;
    const int N = a.N;
    const bool cosine = a.kind == HT_KIND_C;
    const int L = cosine ? N : N + 1;
    if (L < 4) return HT_OK;
    const bool odd = L % 2 != 0;
    if (odd && !cosine) return HT_OK;
    const int H = odd ? (N + 1) / 2 : L / 2;
    const int need = odd ? N + H - 1 : N + 2;
    int M = 512;
    while (M < need) M <<= 1;
    if (M >= h.M) return HT_OK;  // no gain
    a.half = odd ? 2 : 1;
    a.H = H;
    a.hw[0] = static_cast<double>(cosine ? sqrtl(1.0L / N) : sqrtl(2.0L / L));
    a.hw[1] = static_cast<double>(cosine ? sqrtl(2.0L / N) : 0.0L);
    h.M = M;
    a.S = 1;
    a.logP = 0;
    while ((1 << a.logP) < M) ++a.logP;
    if (odd) {  // analysis: N inputs, H outputs; synthesis: H inputs, N outputs
        make_dft_chirp(N, -1, M, N, H, h.ana);
        make_dft_chirp(N, 1, M, H, N, h.syn);
        h.htw.assign(H, cd());  // e^{-i pi k/(2N)}, k < H
        for (int k = 0; k < H; ++k) h.htw[k] = cis_exact(-k, 4LL * N);
        return HT_OK;
    }
    make_dft_chirp(H, cosine ? -1 : 1, M, H, H, h.ana);
    make_dft_chirp(H, 1, M, H, H, h.syn);
    h.htw.assign(2 * static_cast<size_t>(H + 1), cd());
    for (int k = 0; k <= H; ++k) {
        if (cosine) {
            h.htw[k] = cis_exact(-k, N);
            h.htw[H + 1 + k] = cis_exact(-k, 4LL * N);
        } else {
            h.htw[k] = cis_exact(k, L);
            h.htw[H + 1 + k] = cd(cis_exact(k, 2LL * L).imag(), 0.0);
        }
    }
    return HT_OK;
}

// Host replica of the chirp-z core (used at plan creation only): the core transform of a
// real vector, as the device core returns it (real part, imaginary part for the sine
// core, or the complex value for the DFT analysis).
static std::vector<cd> host_core_c(const HostChirp& hc, const std::vector<double>& x, int M) {
    const int N = static_cast<int>(x.size());
    std::vector<cd> a(M, cd());
    for (int j = 0; j < N; ++j) a[j] = x[j] * hc.pre[j];
    host_fft(a, -1);
    for (int k = 0; k < M; ++k) a[k] *= hc.B[k];
    host_fft(a, 1);
    std::vector<cd> y(N);
    for (int k = 0; k < N; ++k) {
        const cd v = a[k] * hc.post[k];
        y[k] = hc.mode == MODE_IM ? cd(v.imag(), 0.0) : hc.mode == MODE_RE ? cd(v.real(), 0.0) : v;
    }
    return y;
}

static std::vector<double> host_core(const HostChirp& hc, const std::vector<double>& x, int M) {
    const std::vector<cd> y = host_core_c(hc, x, M);
    std::vector<double> r(y.size());
    for (size_t k = 0; k < y.size(); ++k) r[k] = y[k].real();
    return r;
}

// ----------------------------------------------------------------------- axis tables

int resolve_kind(int degree, int sym, int family, ht_status* st) {
    *st = HT_OK;
    if (family == HT_FAMILY_PAPER_DST3 && degree == 3) {
        if (!sym) return HT_KIND_F3;
        family = HT_FAMILY_DST;
    }
    if (family == HT_FAMILY_PAPER || family == HT_FAMILY_PAPER_DST3) {
        if (degree == 1) {
            if (!sym) *st = fail(HT_ERR_UNSUPPORTED, "degree 1 (antireflective) needs a symmetric PSF");
            return HT_KIND_AR;
        }
        if (degree == 2) return sym ? HT_KIND_C : HT_KIND_F;
        *st = fail(HT_ERR_UNSUPPORTED, "HT_FAMILY_PAPER supports degrees 1 and 2");
        return 0;
    }
    if (family == HT_FAMILY_DST) {
        if (!sym) *st = fail(HT_ERR_UNSUPPORTED, "HT_FAMILY_DST needs a symmetric PSF");
        if (degree == 1) return HT_KIND_AR;
        if (degree == 2) return HT_KIND_DST2;
        if (degree == 3) return HT_KIND_DST3;
        *st = fail(HT_ERR_UNSUPPORTED, "HT_FAMILY_DST supports degrees 1..3");
        return 0;
    }
    if (family == HT_FAMILY_PERIODIC || family == HT_FAMILY_REFLECTIVE) {
        if (degree != 0) {
            *st = fail(HT_ERR_UNSUPPORTED, "the periodic / reflective comparators have degree 0");
            return 0;
        }
        if (family == HT_FAMILY_REFLECTIVE && !sym) {
            *st = fail(HT_ERR_UNSUPPORTED, "the reflective comparator needs a symmetric PSF");
            return 0;
        }
        return family == HT_FAMILY_PERIODIC ? HT_KIND_P : HT_KIND_R;
    }
    *st = fail(HT_ERR_INVALID_ARG, "unknown family");
    return 0;
}

static ld to_ld(int64_t num, int64_t den) { return static_cast<ld>(num) / static_cast<ld>(den); }

// FFT length M >= 2N - 1 of a chirp-z core of order N, its split and LDS size.
static ht_status size_core(int N, HostAxis& h) {
    Axis& a = h.ax;
    int M = 512;
    while (M < 2 * N - 1) M <<= 1;
    h.M = M;
    a.S = M >= SPLIT_M ? 2 : 1;
    const int P = M / a.S;
    a.logP = 0;
    while ((1 << a.logP) < P) ++a.logP;
    if (a.logP < MIN_LOGP || a.logP > MAX_LOGP || M > TWN)
        return fail(HT_ERR_INVALID_ARG, "internal: unsupported FFT size");
    return HT_OK;
}

// The comparators of Section 2.1: the whole signal is the core (order n), A_P = F^H diag F
// (the exponential core of T_F at order n) and A_R = C^T diag C (the cosine core of T_C at
// order n); eigenvalue grid pi r / n.
static ht_status build_comparator_axis(int n, int kind, HostAxis& h) {
    Axis& a = h.ax;
    a.n = n;
    a.N = n;
    a.kind = kind;
    a.rank = 0;
    ht_status st = size_core(n, h);
    if (st != HT_OK) return st;
    h.q.assign(n, 0.0);
    a.q1 = 0.0;
    for (int i = 0; i < 4; ++i) a.minv[i] = a.Gm[i] = 0.0;
    const int core = kind == HT_KIND_P ? HT_KIND_F : HT_KIND_C;
    make_chirp(core, false, n, h.M, h.ana);
    make_chirp(core, true, n, h.M, h.syn);
    a.den = n;
    h.tcos.resize(2 * a.den);
    h.tsin.resize(2 * a.den);
    for (int r = 0; r < 2 * a.den; ++r) {
        const cd w = cis_exact(r, 2LL * a.den);
        h.tcos[r] = w.real();
        h.tsin[r] = w.imag();
    }
    return HT_OK;
}

static ht_status build_f3_tables(HostAxis& h);

ht_status build_axis(int n, int kind_in, HostAxis& h, bool half_cores) {
    if (kind_in == HT_KIND_P || kind_in == HT_KIND_R) return build_comparator_axis(n, kind_in, h);
    // F3 is T_F plus a rank-2 modification: every T_F table, then its own
    const int kind = kind_in == HT_KIND_F3 ? HT_KIND_F : kind_in;
    const int N = n - 2;
    Axis& a = h.ax;
    a.n = n;
    a.N = N;
    a.kind = kind;
    ht_status st = size_core(N, h);
    if (st != HT_OK) return st;
    const int M = h.M;
    a.rank = kind == HT_KIND_DST2 ? 1 : kind == HT_KIND_DST3 ? 2 : 0;

    // polynomial column
    std::vector<ld> qv(n);
    if (kind == HT_KIND_C || kind == HT_KIND_F) {
        // b - x_i on the extended grid, in units of pi: C: x_i = (2i-1)/(2N), b = (2N+1)/(2N);
        // F: x_i = 2(i-1)/N, b = 2.  q~_{i+1} = (b - x_i)^2.
        for (int i = 0; i < n; ++i) {
            ld diff = kind == HT_KIND_C ? to_ld(2LL * N + 1 - (2LL * i - 1), 2LL * N)
                                        : 2.0L - to_ld(2LL * (i - 1), N);
            qv[i] = diff * diff;
        }
    } else {
        for (int i = 0; i < n; ++i) qv[i] = 1.0L - to_ld(i, n - 1);  // 1 - (i-1)/(n-1), 1-based
    }
    ld nrm = 0.0L;
    for (ld v : qv) nrm += v * v;
    nrm = sqrtl(nrm);
    h.q.resize(n);
    for (int i = 0; i < n; ++i) h.q[i] = static_cast<double>(qv[i] / nrm);
    a.q1 = h.q[0];

    // 2x2 boundary system (closed form of the capacitance matrix)
    a.minv[0] = a.minv[1] = a.minv[2] = a.minv[3] = 0.0;
    if (kind == HT_KIND_C || kind == HT_KIND_F) {
        const ld q1 = qv[0] / nrm, q2 = qv[1] / nrm, qm = qv[n - 2] / nrm;
        const ld diag = kind == HT_KIND_C ? q1 - q2 : q1 - qm;
        const ld off = kind == HT_KIND_C ? -qm : -q2;
        const ld det = diag * diag - off * off;
        if (fabsl(det) < 1e-300L) return fail(HT_ERR_SINGULAR, "boundary 2x2 system is singular");
        a.minv[0] = static_cast<double>(diag / det);
        a.minv[1] = static_cast<double>(-off / det);
        a.minv[2] = static_cast<double>(-off / det);
        a.minv[3] = static_cast<double>(diag / det);
    }

    // chirp tables
    make_chirp(kind, false, N, M, h.ana);
    make_chirp(kind, true, N, M, h.syn);

    // DST family correction
    a.Gm[0] = a.Gm[1] = a.Gm[2] = a.Gm[3] = 0.0;
    if (a.rank > 0) {
        h.bub.assign(static_cast<size_t>(a.rank) * N, 0.0);
        h.U.assign(static_cast<size_t>(a.rank) * N, 0.0);
        std::vector<std::vector<double>> K(a.rank);
        for (int c = 0; c < a.rank; ++c) {
            // x(pi - x) and (x - pi/2) x (pi - x) at x = i pi/(n-1), i = 1..N (units of pi)
            std::vector<ld> v(N);
            ld s2 = 0.0L;
            for (int i = 1; i <= N; ++i) {
                const ld x = to_ld(i, n - 1);
                ld val = x * (1.0L - x);
                if (c == 1) val *= (x - 0.5L);
                v[i - 1] = val;
                s2 += val * val;
            }
            const ld sn = sqrtl(s2);
            std::vector<double> bv(N);
            for (int i = 0; i < N; ++i) bv[i] = static_cast<double>(v[i] / sn);
            std::memcpy(&h.bub[static_cast<size_t>(c) * N], bv.data(), sizeof(double) * N);
            K[c] = host_core(h.ana, bv, M);
            for (int i = 0; i < N; ++i) h.U[static_cast<size_t>(c) * N + i] = K[c][i] - (i == c ? 1.0 : 0.0);
        }
        if (a.rank == 1) {
            if (std::fabs(K[0][0]) < 1e-300) return fail(HT_ERR_SINGULAR, "DST correction is singular");
            a.Gm[0] = 1.0 / K[0][0];
        } else {
            // E^T K = [[K0[0], K1[0]], [K0[1], K1[1]]]
            const double e00 = K[0][0], e01 = K[1][0], e10 = K[0][1], e11 = K[1][1];
            const double det = e00 * e11 - e01 * e10;
            if (std::fabs(det) < 1e-300) return fail(HT_ERR_SINGULAR, "DST correction is singular");
            a.Gm[0] = e11 / det;
            a.Gm[1] = -e01 / det;
            a.Gm[2] = -e10 / det;
            a.Gm[3] = e00 / det;
        }
    }

    // eigenvalue grid trig tables
    a.den = (kind == HT_KIND_C || kind == HT_KIND_F) ? N : n - 1;
    h.tcos.resize(2 * a.den);
    h.tsin.resize(2 * a.den);
    for (int r = 0; r < 2 * a.den; ++r) {
        const cd w = cis_exact(r, 2LL * a.den);  // exp(i pi r / den)
        h.tcos[r] = w.real();
        h.tsin[r] = w.imag();
    }
    if (kind_in == HT_KIND_F3) {
        a.kind = HT_KIND_F3;
        return build_f3_tables(h);
    }
    // the DST correction above used the full core (host_core); only then the half tables
    if (half_cores && (kind == HT_KIND_C || kind == HT_KIND_AR || kind == HT_KIND_DST2 || kind == HT_KIND_DST3))
        return make_half(h);
    return HT_OK;
}

// T_F^{-1} y for a real vector y on the host (the kernel's steps: the 2x2 boundary
// solve, the interior correction, the DFT analysis core).
static std::vector<cd> host_inverse_f(const HostAxis& h, const std::vector<double>& y) {
    const Axis& a = h.ax;
    const int n = a.n, N = a.N;
    const double r1 = y[0] - y[n - 2], r2 = y[n - 1] - y[1];
    const double x1 = a.minv[0] * r1 + a.minv[1] * r2, xn = a.minv[2] * r1 + a.minv[3] * r2;
    std::vector<double> r(N);
    for (int j = 0; j < N; ++j) r[j] = y[j + 1] - h.q[j + 1] * x1 - h.q[N - j] * xn;
    const std::vector<cd> core = host_core_c(h.ana, r, h.M);
    std::vector<cd> x(n);
    x[0] = cd(x1, 0.0);
    x[n - 1] = cd(xn, 0.0);
    for (int j = 0; j < N; ++j) x[j + 1] = core[j];
    return x;
}

// Tables of the degree-3 transform for any PSF (columns 2 and n-2 of T_F replaced by the
// cosine column and the cubic x (x - pi)(x - 2 pi) on the extended grid of T_F).
static ht_status build_f3_tables(HostAxis& h) {
    Axis& a = h.ax;
    const int n = a.n, N = a.N;
    if (N < 3) return fail(HT_ERR_UNSUPPORTED, "degree 3 for a nonsymmetric PSF needs n >= 5");
    h.f3b.assign(2 * static_cast<size_t>(n), 0.0);
    std::vector<ld> cub(n);
    ld nrm = 0.0L;
    for (int r = 0; r < n; ++r) {
        // x_r / pi = 2 (r - 1) / N for 0-based r (the grid point of row r + 1)
        const ld t = to_ld(2LL * (r - 1), N);
        cub[r] = t * (t - 1.0L) * (t - 2.0L);
        nrm += cub[r] * cub[r];
        const cd w = cis_exact(static_cast<int64_t>(r - 1), N, sqrtl(2.0L / N));  // sqrt(2/N) e^{i x_r}
        h.f3b[r] = w.real();
    }
    nrm = sqrtl(nrm);
    std::vector<double> cubic(n);
    for (int r = 0; r < n; ++r) {
        cubic[r] = static_cast<double>(cub[r] / nrm);
        h.f3b[n + r] = cubic[r];
    }
    h.f3v = host_inverse_f(h, cubic);
    // V_E = [[1/sqrt2, v_2], [1/sqrt2, v_{n-2}]]
    const cd s2(1.0 / std::sqrt(2.0), 0.0);
    const cd v2 = h.f3v[2], vm = h.f3v[n - 2];
    const cd det = s2 * vm - v2 * s2;
    if (std::abs(det) < 1e-300) return fail(HT_ERR_SINGULAR, "degree-3 correction is singular");
    const cd vi[4] = {vm / det, -v2 / det, -s2 / det, s2 / det};
    for (int k = 0; k < 4; ++k) a.f3vi[k] = make_double2(vi[k].real(), vi[k].imag());
    return HT_OK;
}

// Tables of the exact GCV (eq. gcv) of a 1D plan: the columns R_c (interior parts of the
// boundary columns, bubble minus the sine column it replaces), M_c = S^H R_c by the host
// core, their Gram matrix, the ghost rows a, b of the cosine / Fourier cores and the corner
// entries of T.
ht_status build_exact_gcv(const HostAxis& h, ht_plan* p, int axis) {
    const Axis& ax = h.ax;
    const int n = ax.n, N = ax.N, kind = ax.kind;
    XgcvParams xp{};
    std::vector<std::vector<double>> R;
    std::vector<std::vector<cd>> Mc;
    std::vector<double> qi(N), jqi(N);
    for (int k = 0; k < N; ++k) {
        qi[k] = h.q[k + 1];
        jqi[k] = h.q[n - 2 - k];
    }
    R.push_back(qi);
    R.push_back(jqi);
    Mc.push_back(host_core_c(h.ana, qi, h.M));
    Mc.push_back(host_core_c(h.ana, jqi, h.M));
    xp.cidx[0] = 0;
    xp.cidx[1] = n - 1;
    for (int c = 0; c < ax.rank; ++c) {
        // bubble c replaces sine column c+1: R = bub - s, S^H R = K - e_c = U[c]
        std::vector<double> r(N);
        const ld sc = sqrtl(2.0L / (N + 1));
        for (int k = 0; k < N; ++k) {
            const cd w = cis_exact(static_cast<int64_t>(c + 1) * (k + 1), 2LL * (N + 1), sc);  // sqrt(2/(N+1)) e^{i pi (c+1)(k+1)/(N+1)}
            r[k] = h.bub[static_cast<size_t>(c) * N + k] - w.imag();
        }
        R.push_back(r);
        std::vector<cd> m(N);
        for (int k = 0; k < N; ++k) m[k] = cd(h.U[static_cast<size_t>(c) * N + k], 0.0);
        Mc.push_back(m);
        xp.cidx[2 + c] = c + 1;
    }
    xp.nc = static_cast<int>(R.size());
    xp.rows = (kind == HT_KIND_C || kind == HT_KIND_F) ? 1 : 0;
    xp.nv = xp.nc + 2 * xp.rows;  // 2 (AR), 3 (DST2), 4 (C, F, DST3)
    if (xp.nv > 4) return fail(HT_ERR_INVALID_ARG, "internal: too many exact GCV vectors");
    for (int i = 0; i < xp.nc; ++i)
        for (int j = 0; j < xp.nc; ++j) {
            ld acc = 0.0L;
            for (int k = 0; k < N; ++k) acc += static_cast<ld>(R[i][k]) * R[j][k];
            xp.gam[i][j] = static_cast<double>(acc);
        }
    xp.t00 = h.q[0];
    xp.t0n = h.q[n - 1];
    xp.tn0 = h.q[n - 1];
    xp.tnn = h.q[0];
    std::vector<double2> host(static_cast<size_t>(xp.nv) * N);
    for (int c = 0; c < xp.nc; ++c)
        for (int k = 0; k < N; ++k) host[static_cast<size_t>(c) * N + k] = make_double2(Mc[c][k].real(), -Mc[c][k].imag());
    if (xp.rows) {
        double2* av = &host[static_cast<size_t>(xp.nc) * N];
        double2* bv = &host[static_cast<size_t>(xp.nc + 1) * N];
        for (int m = 0; m < N; ++m) {
            if (kind == HT_KIND_C) {
                // column m of the DCT-III core at the ghost points x = -pi/(2N), (2N+1) pi/(2N)
                const ld wm = sqrtl((m == 0 ? 1.0L : 2.0L) / N);
                const cd e = cis_exact(m, 4LL * N, wm);
                av[m] = make_double2(e.real(), 0.0);
                bv[m] = make_double2((m & 1) ? -e.real() : e.real(), 0.0);
            } else {
                // column m of the inverse DFT core at x = -2 pi/N and x = 2 pi
                const cd e = cis_exact(-static_cast<int64_t>(m), N, 1.0L / sqrtl(static_cast<ld>(N)));
                av[m] = make_double2(e.real(), e.imag());
                bv[m] = make_double2(static_cast<double>(1.0L / sqrtl(static_cast<ld>(N))), 0.0);
            }
        }
    }
    void* mem = nullptr;
    if (hipMalloc(&mem, sizeof(double2) * host.size()) != hipSuccess) return fail(HT_ERR_OOM, "exact GCV table allocation failed");
    if (hipMemcpy(mem, host.data(), sizeof(double2) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(mem);
        return fail(HT_ERR_HIP, "exact GCV table upload failed");
    }
    xp.vec = static_cast<const double2*>(mem);
    p->xg[axis] = xp;
    p->xg_mem[axis] = mem;
    return HT_OK;
}

// Upload the host tables of `nax` axes into one device arena and fill in the device
// pointers of each Axis.
ht_status upload_axes(const HostAxis* hs, int64_t nax, void** arena_out, Axis* axes_out) {
    size_t bytes = 0;
    auto reserve = [&](size_t nbytes) {
        const size_t off = bytes;
        bytes += (nbytes + 255) & ~static_cast<size_t>(255);
        return off;
    };
    struct Offs { size_t q, bub, U, tcos, tsin, apre, apost, aB, spre, spost, sB, f3v, f3b, htw; };
    std::vector<Offs> o(nax);
    for (int64_t a = 0; a < nax; ++a) {
        const HostAxis& h = hs[a];
        const size_t N = h.ax.N;
        o[a].f3v = reserve(sizeof(double2) * (h.f3v.size() + 1));
        o[a].f3b = reserve(sizeof(double) * (h.f3b.size() + 1));
        o[a].htw = reserve(sizeof(double2) * (h.htw.size() + 1));
        o[a].q = reserve(sizeof(double) * h.q.size());
        o[a].bub = reserve(sizeof(double) * (h.bub.size() + 1));
        o[a].U = reserve(sizeof(double) * (h.U.size() + 1));
        o[a].tcos = reserve(sizeof(double) * h.tcos.size());
        o[a].tsin = reserve(sizeof(double) * h.tsin.size());
        o[a].apre = reserve(sizeof(double2) * h.ana.pre.size());
        o[a].apost = reserve(sizeof(double2) * h.ana.post.size());
        o[a].aB = reserve(sizeof(double2) * h.M);
        o[a].spre = reserve(sizeof(double2) * h.syn.pre.size());
        o[a].spost = reserve(sizeof(double2) * h.syn.post.size());
        o[a].sB = reserve(sizeof(double2) * h.M);
        (void)N;
    }
    std::vector<char> host;
    try {
        host.assign(bytes, 0);
    } catch (...) {
        return fail(HT_ERR_OOM, "host staging allocation failed");
    }
    auto put = [&](size_t off, const void* src, size_t nb) {
        if (nb) std::memcpy(host.data() + off, src, nb);
    };
    auto putc = [&](size_t off, const std::vector<cd>& v) {
        double2* dst = reinterpret_cast<double2*>(host.data() + off);
        for (size_t i = 0; i < v.size(); ++i) dst[i] = make_double2(v[i].real(), v[i].imag());
    };
    // filter spectra stored split-major: half s holds B[S u + s], u < M / S, contiguously
    auto putc_split = [&](size_t off, const std::vector<cd>& v, int S) {
        double2* dst = reinterpret_cast<double2*>(host.data() + off);
        const size_t P = v.size() / S;
        for (int sidx = 0; sidx < S; ++sidx)
            for (size_t u = 0; u < P; ++u) {
                const cd w = v[S * u + sidx];
                dst[sidx * P + u] = make_double2(w.real(), w.imag());
            }
    };
    for (int64_t a = 0; a < nax; ++a) {
        const HostAxis& h = hs[a];
        put(o[a].q, h.q.data(), sizeof(double) * h.q.size());
        putc(o[a].f3v, h.f3v);
        putc(o[a].htw, h.htw);
        put(o[a].f3b, h.f3b.data(), sizeof(double) * h.f3b.size());
        put(o[a].bub, h.bub.data(), sizeof(double) * h.bub.size());
        put(o[a].U, h.U.data(), sizeof(double) * h.U.size());
        put(o[a].tcos, h.tcos.data(), sizeof(double) * h.tcos.size());
        put(o[a].tsin, h.tsin.data(), sizeof(double) * h.tsin.size());
        putc(o[a].apre, h.ana.pre);
        putc(o[a].apost, h.ana.post);
        putc_split(o[a].aB, h.ana.B, h.ax.S);
        putc(o[a].spre, h.syn.pre);
        putc(o[a].spost, h.syn.post);
        putc_split(o[a].sB, h.syn.B, h.ax.S);
    }
    char* dev = nullptr;
    if (hipMalloc(&dev, bytes) != hipSuccess) return fail(HT_ERR_OOM, "table allocation failed");
    if (hipMemcpy(dev, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dev);
        return fail(HT_ERR_HIP, "table upload failed");
    }
    *arena_out = dev;
    for (int64_t a = 0; a < nax; ++a) {
        Axis ax = hs[a].ax;
        ax.q = reinterpret_cast<const double*>(dev + o[a].q);
        ax.f3v = reinterpret_cast<const double2*>(dev + o[a].f3v);
        ax.f3b = reinterpret_cast<const double*>(dev + o[a].f3b);
        ax.htw = reinterpret_cast<const double2*>(dev + o[a].htw);
        ax.bub = reinterpret_cast<const double*>(dev + o[a].bub);
        ax.U = reinterpret_cast<const double*>(dev + o[a].U);
        ax.tcos = reinterpret_cast<const double*>(dev + o[a].tcos);
        ax.tsin = reinterpret_cast<const double*>(dev + o[a].tsin);
        ax.ana = Chirp{reinterpret_cast<const double2*>(dev + o[a].apre), reinterpret_cast<const double2*>(dev + o[a].apost),
                       reinterpret_cast<const double2*>(dev + o[a].aB), hs[a].ana.mode};
        ax.syn = Chirp{reinterpret_cast<const double2*>(dev + o[a].spre), reinterpret_cast<const double2*>(dev + o[a].spost),
                       reinterpret_cast<const double2*>(dev + o[a].sB), hs[a].syn.mode};
        ax.tw = nullptr;
        axes_out[a] = ax;
    }
    return HT_OK;
}

// ---------------------------------------------------------------- float32 cores

void plan_release_f32(ht_plan* p) {
    if (p->arena32) (void)hipFree(p->arena32);
    p->arena32 = nullptr;
    p->f32 = 0;
    for (int a = 0; a < 2; ++a) {
        p->ax[a].ana32 = Chirp32{};
        p->ax[a].syn32 = Chirp32{};
        p->ax[a].tw32 = nullptr;
    }
}

// float32 copies (rounded from the exact-angle float64 values) of the plan's chirp tables
// and of the twiddle table, for HT_PRECISION_F32.
ht_status plan_build_f32(ht_plan* p) {
    std::vector<HostAxis> hs(p->ndim);
    for (int a = 0; a < p->ndim; ++a) {
        ht_status st = build_axis(p->ax[a].n, p->ax[a].kind, hs[a]);
        if (st != HT_OK) return st;
    }
    size_t bytes = 0;
    auto reserve = [&](size_t n2) {
        const size_t off = bytes;
        bytes += (sizeof(float2) * n2 + 255) & ~static_cast<size_t>(255);
        return off;
    };
    const size_t otw = reserve(TWN);
    struct Offs { size_t apre, apost, aB, spre, spost, sB; } o[2];
    for (int a = 0; a < p->ndim; ++a) {
        const size_t N = hs[a].ax.N, M = hs[a].M;
        o[a] = {reserve(N), reserve(N), reserve(M), reserve(N), reserve(N), reserve(M)};
    }
    std::vector<float2> host(bytes / sizeof(float2));
    auto at = [&](size_t off) { return host.data() + off / sizeof(float2); };
    for (int m = 0; m < TWN; ++m) {
        const cd w = cis_exact(-m, TWN);
        at(otw)[m] = make_float2(static_cast<float>(w.real()), static_cast<float>(w.imag()));
    }
    auto putc = [&](size_t off, const std::vector<cd>& v) {
        for (size_t i = 0; i < v.size(); ++i)
            at(off)[i] = make_float2(static_cast<float>(v[i].real()), static_cast<float>(v[i].imag()));
    };
    auto putc_split = [&](size_t off, const std::vector<cd>& v, int S) {  // as the float64 tables
        const size_t P = v.size() / S;
        for (int sidx = 0; sidx < S; ++sidx)
            for (size_t u = 0; u < P; ++u) {
                const cd w = v[S * u + sidx];
                at(off)[sidx * P + u] = make_float2(static_cast<float>(w.real()), static_cast<float>(w.imag()));
            }
    };
    for (int a = 0; a < p->ndim; ++a) {
        putc(o[a].apre, hs[a].ana.pre);
        putc(o[a].apost, hs[a].ana.post);
        putc_split(o[a].aB, hs[a].ana.B, hs[a].ax.S);
        putc(o[a].spre, hs[a].syn.pre);
        putc(o[a].spost, hs[a].syn.post);
        putc_split(o[a].sB, hs[a].syn.B, hs[a].ax.S);
    }
    char* dev = nullptr;
    if (hipMalloc(&dev, bytes) != hipSuccess) return fail(HT_ERR_OOM, "float32 table allocation failed");
    if (hipMemcpy(dev, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dev);
        return fail(HT_ERR_HIP, "float32 table upload failed");
    }
    plan_release_f32(p);
    p->arena32 = dev;
    p->f32 = 1;
    auto ptr = [&](size_t off) { return reinterpret_cast<const float2*>(dev + off); };
    for (int a = 0; a < p->ndim; ++a) {
        p->ax[a].ana32 = Chirp32{ptr(o[a].apre), ptr(o[a].apost), ptr(o[a].aB), p->ax[a].ana.mode};
        p->ax[a].syn32 = Chirp32{ptr(o[a].spre), ptr(o[a].spost), ptr(o[a].sB), p->ax[a].syn.mode};
        p->ax[a].tw32 = ptr(otw);
    }
    return HT_OK;
}

}  // namespace ht

using namespace ht;

extern "C" ht_status ht_plan_create(int ndim, const int64_t* n, int degree, int psf_symmetric, int family,
                                    int64_t max_batch, ht_plan** out) {
    if (!out || !n) return fail(HT_ERR_INVALID_ARG, "ht_plan_create: null argument");
    *out = nullptr;
    if (ndim != 1 && ndim != 2) return fail(HT_ERR_INVALID_ARG, "ht_plan_create: ndim must be 1 or 2");
    for (int a = 0; a < ndim; ++a)
        if (n[a] < 5 || n[a] > MAX_N) return fail(HT_ERR_INVALID_ARG, "ht_plan_create: n must be in [5, 8192]");
    if (ndim == 2 && (max_batch < 1 || max_batch > 4096))
        return fail(HT_ERR_INVALID_ARG, "ht_plan_create: max_batch must be in [1, 4096] for 2D plans");
    ht_status st;
    const int kind = resolve_kind(degree, psf_symmetric, family, &st);
    if (st != HT_OK) return st;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(HT_ERR_HIP, "ht_plan_create: no HIP device");
    const double2* tw = device_twiddles(device, &st);
    if (tw && (st = static_scratch_init(device, nullptr)) != HT_OK) return st;
    if (!tw) return st;
    HostAxis hs[2];
    for (int a = 0; a < ndim; ++a) {
        st = build_axis(static_cast<int>(n[a]), kind, hs[a]);
        if (st != HT_OK) return st;
    }
    ht_plan* p = new (std::nothrow) ht_plan();
    if (!p) return fail(HT_ERR_OOM, "ht_plan_create: host allocation failed");
    p->ndim = ndim;
    p->device = device;
    p->tw = tw;
    p->cplx = (kind == HT_KIND_F || kind == HT_KIND_P || kind == HT_KIND_F3) ? 1 : 0;
    p->max_batch = max_batch < 1 ? 1 : max_batch;
    st = upload_axes(hs, ndim, &p->arena, p->ax);
    if (st != HT_OK) {
        delete p;
        return st;
    }
    for (int a = 0; a < ndim; ++a) p->ax[a].tw = tw;
    if (kind != HT_KIND_P && kind != HT_KIND_R && kind != HT_KIND_F3) {  // P, R: eq. gcv2 is exact
        for (int a = 0; a < ndim; ++a) {
            st = build_exact_gcv(hs[a], p, a);
            if (st != HT_OK) {
                ht_plan_destroy(p);
                return st;
            }
        }
    }
    if (ndim == 2) {
        const int64_t img = n[0] * n[1];
        if (hipMalloc(&p->work, sizeof(double2) * img * max_batch) != hipSuccess) {
            ht_plan_destroy(p);
            return fail(HT_ERR_OOM, "ht_plan_create: 2D workspace allocation failed");
        }
        p->gcv_part_elems = 2LL * 512 * 1024 * max_batch;
        if (hipMalloc(&p->gcv_part, sizeof(double) * p->gcv_part_elems) != hipSuccess) {
            ht_plan_destroy(p);
            return fail(HT_ERR_OOM, "ht_plan_create: GCV workspace allocation failed");
        }
        if (p->xg_mem[0]) {  // exact GCV for images: workspace for grids of up to 128 values
            st = reserve_exact_gcv_2d(p, XG2_DEFAULT_K);
            if (st != HT_OK) {
                ht_plan_destroy(p);
                return st;
            }
        }
    }
    *out = p;
    return HT_OK;
}

extern "C" ht_status ht_plan_destroy(ht_plan* p) {
    if (!p) return HT_OK;
    if (p->arena) (void)hipFree(p->arena);
    if (p->work) (void)hipFree(p->work);
    if (p->gcv_part) (void)hipFree(p->gcv_part);
    if (p->xg2_mem) (void)hipFree(p->xg2_mem);
    for (void* m : p->xg_mem)
        if (m) (void)hipFree(m);
    gemm_release(p->gemm);
    plan_release_f32(p);
    delete p;
    return HT_OK;
}

extern "C" int ht_plan_kind(const ht_plan* p, int axis) {
    if (!p || axis < 0 || axis >= p->ndim) return -1;
    return p->ax[axis].kind;
}

extern "C" int ht_plan_is_complex(const ht_plan* p) { return p ? p->cplx : 0; }

extern "C" const char* ht_status_str(ht_status s) {
    switch (s) {
        case HT_OK: return "HT_OK";
        case HT_ERR_INVALID_ARG: return "HT_ERR_INVALID_ARG";
        case HT_ERR_UNSUPPORTED: return "HT_ERR_UNSUPPORTED";
        case HT_ERR_PSF_TOO_WIDE: return "HT_ERR_PSF_TOO_WIDE";
        case HT_ERR_SINGULAR: return "HT_ERR_SINGULAR";
        case HT_ERR_NONFINITE: return "HT_ERR_NONFINITE";
        case HT_ERR_HIP: return "HT_ERR_HIP";
        case HT_ERR_OOM: return "HT_ERR_OOM";
    }
    return "HT_ERR_UNKNOWN";
}

extern "C" const char* ht_last_error(void) { return g_last_error.c_str(); }
