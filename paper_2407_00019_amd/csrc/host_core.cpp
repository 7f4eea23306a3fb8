// Host-only parts of libspmvat (no HIP): the server's offset allocator,
// D_mat from the row moments (Eq. (4)) and the auto-tuner's table and
// on-line decision (section 2.2).
#include "host_core.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <limits>
#include <new>

#define SPMV_API extern "C" __attribute__((visibility("default")))

using namespace spmvat;

// ------------------------------------------------------------- arena

spmv_arena::spmv_arena(size_t bytes) : cap(bytes / kGrain * kGrain), free_bytes(cap) {
    if (cap) free_[0] = cap;
}

size_t spmv_arena::round(size_t bytes) {
    const size_t b = std::max<size_t>(bytes, 1);
    if (b > std::numeric_limits<size_t>::max() - (kGrain - 1)) return 0;
    return (b + kGrain - 1) / kGrain * kGrain;
}

int64_t spmv_arena::alloc(size_t bytes) {
    const size_t need = round(bytes);
    if (need == 0 || need > free_bytes) return -1;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= need) {
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > need) free_[off + need] = sz - need;
            free_bytes -= need;
            return (int64_t)off;
        }
    }
    return -1;
}

bool spmv_arena::release(int64_t off, size_t bytes) {
    size_t sz = round(bytes);
    if (off < 0 || sz == 0 || (size_t)off > cap || sz > cap - (size_t)off) return false;
    const size_t o = (size_t)off;
    auto next = free_.lower_bound(o);
    if (next != free_.end() && next->first < o + sz) return false;                      // overlaps the next free block
    if (next != free_.begin() && std::prev(next)->first + std::prev(next)->second > o) return false;  // or the one before
    free_bytes += sz;
    if (next != free_.end() && o + sz == next->first) {
        sz += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == o) {
            prev->second += sz;
            return true;
        }
    }
    free_[o] = sz;
    return true;
}

size_t spmv_arena::largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
}

SPMV_API spmv_arena* spmv_arena_create(size_t bytes) { return new (std::nothrow) spmv_arena(bytes); }
SPMV_API int64_t spmv_arena_alloc(spmv_arena* a, size_t bytes) { return a ? a->alloc(bytes) : -1; }
SPMV_API void spmv_arena_free(spmv_arena* a, int64_t off, size_t bytes) {
    if (a) a->release(off, bytes);
}
SPMV_API size_t spmv_arena_free_bytes(const spmv_arena* a) { return a ? a->free_bytes : 0; }
SPMV_API size_t spmv_arena_largest(const spmv_arena* a) { return a ? a->largest() : 0; }
SPMV_API void spmv_arena_destroy(spmv_arena* a) { delete a; }

// ------------------------------------------------------------- D_mat

namespace spmvat {

void dmat_from_moments(int32_t n, uint64_t s1, uint64_t s2, spmv_stats* st) {
    // num = n*s2 - s1^2 (= n^2 sigma^2) is exact in 128 bits
    const unsigned __int128 num = (unsigned __int128)(uint64_t)n * s2 - (unsigned __int128)s1 * s1;
    const uint64_t hi = (uint64_t)(num >> 64), lo = (uint64_t)num;
    double numd;
    if (hi == 0) {
        numd = (double)lo;   // the conversion rounds to nearest even
    } else {
        // nearest binary64 of the 128-bit integer: the top 64 significant bits
        // carry the rounding, the bits below them only stick
        const int lz = __builtin_clzll(hi);
        const int sh = 64 - lz;
        uint64_t top = (hi << lz) | (lz ? (lo >> (64 - lz)) : 0);
        const uint64_t rest = lz ? (lo << lz) : lo;
        top |= (rest != 0) ? 1u : 0u;
        numd = std::ldexp((double)top, sh);   // one rounding of 64 -> 53 bits
    }
    const double r = std::sqrt(numd);
    st->mu = (double)s1 / (double)n;
    st->sigma = r / (double)n;
    st->d_mat = s1 == 0 ? 0.0 : r / (double)s1;
}

}  // namespace spmvat

// ----------------------------------------------------------- auto-tuning

SPMV_API spmv_status at_table_build(const double* d, const double* r, const int32_t* feasible, int32_t m,
                                    double c, at_table* out) {
    if (!out || m < 0 || (m > 0 && (!d || !r))) return SPMV_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->c = c;
    // D* = the smallest D_mat among feasible points whose R_ell falls below c
    double dstar = std::numeric_limits<double>::infinity();
    for (int32_t i = 0; i < m; ++i) {
        if (feasible && !feasible[i]) continue;
        if (!(r[i] >= c) && d[i] < dstar) dstar = d[i];
    }
    out->d_star = dstar;
    return SPMV_OK;
}

namespace {

int dbucket(double d) {
    static const double edges[AT_DBUCKETS - 1] = {0.0625, 0.125, 0.25, 0.5, 1.0, 2.0, 4.0};
    int b = 0;
    while (b < AT_DBUCKETS - 1 && d >= edges[b]) ++b;
    return b;
}

// Algorithmic bytes of one SpMV in a format (x and y counted once, ELL
// padding included) and of the transformation into it.
double spmv_bytes(const spmv_stats& st, spmv_dtype dt, spmv_format f) {
    const double n = st.n, nnz = (double)st.nnz, vb = vbytes_of(dt), xb = xbytes_of(dt);
    switch (f) {
        case SPMV_CRS: return (vb + 4) * nnz + 4 * (n + 1) + 2 * xb * n;
        case SPMV_COO_ROW: return (vb + 8) * nnz + 2 * xb * n;
        case SPMV_ELL_ROW: return (vb + 4) * n * (double)st.max_row + 2 * xb * n;
        default: return 0;
    }
}
double trans_bytes(const spmv_stats& st, spmv_dtype dt, spmv_format f) {
    const double n = st.n, nnz = (double)st.nnz, vb = vbytes_of(dt);
    switch (f) {
        case SPMV_COO_ROW: return 4 * (n + 1) + 4 * nnz;
        case SPMV_ELL_ROW: return (vb + 4) * nnz + 4 * (n + 1) + (vb + 4) * n * (double)st.max_row;
        default: return 0;
    }
}

// ELL-Row footprint check of spmv_buffer_sizes, from statistics.
bool ell_row_fits(const spmv_stats& st, spmv_dtype dt, size_t limit) {
    const unsigned __int128 slots =
        (unsigned __int128)(uint64_t)(st.max_row < 0 ? 0 : st.max_row) * (uint64_t)(st.n < 0 ? 0 : st.n);
    if (slots > (unsigned __int128)(SIZE_MAX / 16)) return false;
    return (size_t)slots * (size_t)(vbytes_of(dt) + 4) <= limit;
}

}  // namespace

SPMV_API spmv_status at_choose_format_stats(const spmv_stats* st, spmv_dtype dt, size_t limit,
                                            const at_table* t, int64_t k_repeats, spmv_format* fmt,
                                            int* variant, at_decision* why) {
    if (!st || !t || !fmt || !variant || !valid_dtype(dt) || st->n < 1) return SPMV_E_ARG;
    at_decision d{};
    d.d_mat = st->d_mat;
    d.feasible_ell = ell_row_fits(*st, dt, limit) ? 1 : 0;
    if (k_repeats <= 0 || !t->calibrated) {
        // the paper's on-line phase: ELL when D_mat < D*
        d.rule = 0;
        if (d.feasible_ell && st->d_mat < t->d_star) { *fmt = SPMV_ELL_ROW; *variant = 0; }
        else { *fmt = SPMV_CRS; *variant = 1; }
    } else {
        // least estimated transformation + k SpMVs among the transformed
        // formats; it replaces CRS only by more than the model's error
        d.rule = 1;
        const int b = dbucket(st->d_mat);
        const int loc = st->bandwidth <= AT_LOCAL_BAND ? 0 : 1;
        const double k = (double)k_repeats;
        auto est = [&](double bytes, double bps, int launches) {
            return bps > 0 ? bytes / bps + launches * t->launch_s : std::numeric_limits<double>::infinity();
        };
        const double tc0 = est(spmv_bytes(*st, dt, SPMV_CRS), t->spmv_bps[loc][SPMV_CRS][0][b], 1);
        const double tc1 = est(spmv_bytes(*st, dt, SPMV_CRS), t->spmv_bps[loc][SPMV_CRS][1][b], 1);
        spmv_format bf = SPMV_CRS;
        int bv = tc1 < tc0 ? 1 : 0;
        const double tcrs = std::min(tc0, tc1);
        double best = std::numeric_limits<double>::infinity(), bt = tcrs, btr = 0;
        spmv_format cf = SPMV_CRS;
        const spmv_format cands[2] = {SPMV_COO_ROW, SPMV_ELL_ROW};
        for (spmv_format f : cands) {
            if (f == SPMV_ELL_ROW && !d.feasible_ell) continue;
            const double ts = est(spmv_bytes(*st, dt, f), t->spmv_bps[loc][f][0][b], f == SPMV_COO_ROW ? 2 : 1);
            const double tr = est(trans_bytes(*st, dt, f), t->trans_bps[loc][f][b], 1);
            const double cost = tr + k * ts;
            if (cost < best) { best = cost; cf = f; bt = ts; btr = tr; }
        }
        const double margin = t->k_margin > 0 ? t->k_margin : AT_K_MARGIN;
        if (cf != SPMV_CRS && margin * best < k * tcrs) { bf = cf; bv = 0; }
        else { bt = tcrs; btr = 0; }
        *fmt = bf; *variant = bv;
        d.t_crs_hat = tcrs; d.t_fmt_hat = bt; d.t_trans_hat = btr;
        if (bf != SPMV_CRS && bt < tcrs) d.k_break_even = (btr / tcrs) / (1.0 - bt / tcrs);
    }
    if (why) *why = d;
    return SPMV_OK;
}
