// Host-side construction of the per-axis tables (shared by plans and ragged batches).
#pragma once

#include <complex>
#include <vector>

#include "ht_internal.h"

namespace ht {

using cd = std::complex<double>;

struct HostChirp {
    std::vector<cd> pre, post, B;
    int mode = MODE_RE;
};

struct HostAxis {
    Axis ax{};
    std::vector<double> q, bub, U, tcos, tsin;
    std::vector<cd> f3v;       // kind F3 only
    std::vector<double> f3b;   // kind F3 only
    std::vector<cd> htw;       // half-length cores only
    HostChirp ana, syn;
    int M = 0;
};

// Transform kind realising (degree, symmetric PSF, family); sets *st on failure.
int resolve_kind(int degree, int sym, int family, ht_status* st);
// All host tables of one 1D transform of length n.  half_cores: use the half-length real
// cores where the kind and length allow (ragged batches only).
ht_status build_axis(int n, int kind, HostAxis& h, bool half_cores = false);
// Upload `nax` axes into one device arena; fills device pointers into axes_out.
ht_status upload_axes(const HostAxis* hs, int64_t nax, void** arena_out, Axis* axes_out);

}  // namespace ht
