// Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
// oracle, the input generators and the host-only part of the library (the
// server's offset allocator, D_mat from the row moments, the auto-tuner's
// decision).  Built and run by tests/test_sanitize_host.py; any sanitizer
// report aborts the run, and each check below that fails prints a line and
// makes the exit status non-zero.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <random>
#include <vector>

#include "../../include/spmvat.h"
#include "../../paper_2407_00019_amd/csrc/host_core.h"

extern "C" {
// oracle/oracle.c
int orc_validate_crs(int32_t n, int64_t nnz, const int32_t* irp, const int32_t* icol);
void orc_row_moments(int32_t n, const int32_t* irp, int64_t* s1, int64_t* s2, int32_t* lmax, int32_t* lmin);
int32_t orc_bandwidth(int32_t n, const int32_t* irp, const int32_t* icol);
void orc_dmat(int32_t n, int64_t s1, int64_t s2, double* mu, double* sigma, double* d);
void orc_expand_ptr(int32_t n, const int32_t* ptr, int32_t* idx);
int orc_csr_to_ccs(int32_t n, const int32_t* irp, const int32_t* icol, const void* val, int vbytes, int32_t* ccp,
                   int32_t* irow_t, void* val_t);
int32_t orc_max_len(int32_t n, const int32_t* ptr);
void orc_to_ell(int32_t n, const int32_t* ptr, const int32_t* idx, const void* val, int vbytes, int32_t width,
                void* ell_val, int32_t* ell_idx);
void orc_spmv_crs(int32_t n, const int32_t* irp, const int32_t* icol, const double* val, const double* x, double* y);
void orc_spmv_coo_row(int32_t n, int64_t nnz, const int32_t* irow, const int32_t* icol, const double* val,
                      const double* x, double* y);
void orc_spmv_ell_row(int32_t n, int32_t width, const double* ev, const int32_t* ec, const double* x, double* y);
void orc_spmv_coo_col(int32_t n, int64_t nnz, const int32_t* jcol, const int32_t* irow_t, const double* val_t,
                      const double* x, double* y);
void orc_spmv_ell_col(int32_t n, int32_t width, const double* ev, const int32_t* er, const double* x, double* y);
void orc_round_values(int dtype, int64_t m, const double* in, void* out);
void orc_widen_values(int dtype, int64_t m, const void* in, double* out);
// gen/spmvgen.c
void gen_uniform(int64_t m, double lo, double hi, uint64_t seed, uint64_t stream, double* out);
void gen_normal(int64_t m, uint64_t seed, uint64_t stream, double* out);
int64_t gen_lap2d(int32_t nx, int32_t ny, double diag, double off, int32_t* irp, int32_t* icol, double* val);
int64_t gen_stencil27(int32_t nx, int32_t ny, int32_t nz, int integer_values, uint64_t seed, int32_t* irp,
                      int32_t* icol, double* val);
void gen_lognormal_lengths(int32_t n, double mean, double s, int32_t lmin, int32_t lmax, uint64_t seed, int32_t* len);
int64_t gen_lengths_to_irp(int32_t n, const int32_t* len, int32_t* irp);
void gen_random_cols(int32_t n, int32_t ncols, const int32_t* irp, uint64_t seed, int32_t* icol);
void gen_window_cols(int32_t n, int32_t w, const int32_t* irp, uint64_t seed, int32_t* icol);
int64_t gen_banded(int32_t n, int32_t b, uint64_t seed, int32_t* irp, int32_t* icol, double* val);
void gen_unif_stream(int64_t m, uint64_t seed, uint64_t stream, double* out);
}

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                        \
    do {                                                        \
        if (!(cond)) {                                          \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);    \
            std::printf(__VA_ARGS__);                           \
            std::printf("\n");                                  \
            ++g_fail;                                           \
        }                                                       \
    } while (0)

struct Crs {
    int32_t n = 0;
    std::vector<int32_t> irp, icol;
    std::vector<double> val;
    int64_t nnz() const { return irp.empty() ? 0 : irp[n]; }
};

// Exactly sized arrays: the sanitizer flags any write past them.
Crs from_lengths(std::vector<int32_t> len, int32_t ncols_window, bool window, uint64_t seed) {
    Crs m;
    m.n = (int32_t)len.size();
    m.irp.assign(m.n + 1, 0);
    const int64_t nnz = gen_lengths_to_irp(m.n, len.data(), m.irp.data());
    m.icol.assign(nnz, 0);
    m.val.assign(nnz, 0.0);
    if (window) gen_window_cols(m.n, ncols_window, m.irp.data(), seed, m.icol.data());
    else gen_random_cols(m.n, m.n, m.irp.data(), seed, m.icol.data());
    std::mt19937_64 r(seed);
    for (auto& v : m.val) v = (double)((int)(r() % 7) - 3);   // small integers: every sum is exact
    return m;
}

std::vector<Crs> matrices() {
    std::vector<Crs> out;
    {   // 5-point Laplacian
        Crs m;
        const int nx = 9, ny = 7;
        m.n = nx * ny;
        const int64_t nnz = gen_lap2d(nx, ny, 4.0, -1.0, nullptr, nullptr, nullptr);
        m.irp.assign(m.n + 1, 0); m.icol.assign(nnz, 0); m.val.assign(nnz, 0.0);
        gen_lap2d(nx, ny, 4.0, -1.0, m.irp.data(), m.icol.data(), m.val.data());
        out.push_back(m);
    }
    {   // 27-point stencil with integer values
        Crs m;
        m.n = 5 * 4 * 3;
        const int64_t nnz = gen_stencil27(5, 4, 3, 1, 11, nullptr, nullptr, nullptr);
        m.irp.assign(m.n + 1, 0); m.icol.assign(nnz, 0); m.val.assign(nnz, 0.0);
        gen_stencil27(5, 4, 3, 1, 11, m.irp.data(), m.icol.data(), m.val.data());
        out.push_back(m);
    }
    {   // banded
        Crs m;
        m.n = 40;
        const int64_t nnz = gen_banded(40, 3, 5, nullptr, nullptr, nullptr);
        m.irp.assign(m.n + 1, 0); m.icol.assign(nnz, 0); m.val.assign(nnz, 0.0);
        gen_banded(40, 3, 5, m.irp.data(), m.icol.data(), m.val.data());
        for (auto& v : m.val) v = std::floor(8 * v);
        out.push_back(m);
    }
    {   // lognormal row lengths, random and windowed columns, empty rows
        const int32_t n = 300;
        std::vector<int32_t> len(n);
        gen_lognormal_lengths(n, 6.0, 1.2, 0, 40, 3, len.data());
        out.push_back(from_lengths(len, 0, false, 21));
        for (auto& l : len) l = std::min(l, 26);   // the clipped window [i - 25, i + 25] holds at least 26 columns
        out.push_back(from_lengths(len, 25, true, 22));
    }
    out.push_back(from_lengths({0}, 0, false, 1));            // one empty row
    out.push_back(from_lengths({1}, 0, false, 2));            // one entry
    out.push_back(from_lengths({0, 0, 0, 0}, 0, false, 3));   // no entries at all
    {   // duplicates and unsorted rows (accepted by the method)
        Crs m;
        m.n = 4;
        m.irp = {0, 3, 3, 6, 8};
        m.icol = {2, 0, 2, 3, 3, 1, 0, 0};
        m.val = {1, 2, 3, 4, 5, 6, 7, 8};
        out.push_back(m);
    }
    return out;
}

void check_matrix(const Crs& m, int idx) {
    const int32_t n = m.n;
    const int64_t nnz = m.nnz();
    CHECK(orc_validate_crs(n, nnz, m.irp.data(), m.icol.data()) == 0, "matrix %d invalid", idx);
    int64_t s1, s2;
    int32_t lmax, lmin;
    orc_row_moments(n, m.irp.data(), &s1, &s2, &lmax, &lmin);
    CHECK(s1 == nnz, "matrix %d: s1", idx);
    (void)orc_bandwidth(n, m.irp.data(), m.icol.data());

    // D_mat: the library's host code against the oracle, bit for bit
    double mu, sg, d;
    orc_dmat(n, s1, s2, &mu, &sg, &d);
    spmv_stats st{};
    spmvat::dmat_from_moments(n, (uint64_t)s1, (uint64_t)s2, &st);
    CHECK(st.mu == mu && st.sigma == sg && st.d_mat == d, "matrix %d: D_mat %.17g vs %.17g", idx, st.d_mat, d);

    // every transformation into exactly sized arrays
    std::vector<int32_t> irow(nnz), ccp(n + 1), irow_t(nnz), jcol(nnz);
    std::vector<double> val_t(nnz);
    orc_expand_ptr(n, m.irp.data(), irow.data());
    CHECK(orc_csr_to_ccs(n, m.irp.data(), m.icol.data(), m.val.data(), 8, ccp.data(), irow_t.data(),
                         val_t.data()) == 0, "matrix %d: CCS", idx);
    CHECK(ccp[0] == 0 && ccp[n] == nnz, "matrix %d: ccp ends", idx);
    orc_expand_ptr(n, ccp.data(), jcol.data());
    const int32_t wr = orc_max_len(n, m.irp.data()), wc = orc_max_len(n, ccp.data());
    std::vector<double> evr((size_t)wr * n), evc((size_t)wc * n);
    std::vector<int32_t> ecr((size_t)wr * n), erc((size_t)wc * n);
    orc_to_ell(n, m.irp.data(), m.icol.data(), m.val.data(), 8, wr, evr.data(), ecr.data());
    orc_to_ell(n, ccp.data(), irow_t.data(), val_t.data(), 8, wc, evc.data(), erc.data());

    // with small integer values and x every SpMV is exact: all formats agree
    std::vector<double> x(n), y0(n), y(n);
    gen_uniform(n, -4.0, 4.0, 7, 1, x.data());
    for (auto& v : x) v = std::floor(v);
    orc_spmv_crs(n, m.irp.data(), m.icol.data(), m.val.data(), x.data(), y0.data());
    orc_spmv_coo_row(n, nnz, irow.data(), m.icol.data(), m.val.data(), x.data(), y.data());
    CHECK(y == y0, "matrix %d: COO-Row SpMV", idx);
    orc_spmv_ell_row(n, wr, evr.data(), ecr.data(), x.data(), y.data());
    CHECK(y == y0, "matrix %d: ELL-Row SpMV", idx);
    orc_spmv_coo_col(n, nnz, jcol.data(), irow_t.data(), val_t.data(), x.data(), y.data());
    CHECK(y == y0, "matrix %d: COO-Column SpMV", idx);
    orc_spmv_ell_col(n, wc, evc.data(), erc.data(), x.data(), y.data());
    CHECK(y == y0, "matrix %d: ELL-Column SpMV", idx);

    // reduced-precision storage of the values, and back
    std::vector<double> wide(nnz);
    std::vector<uint32_t> b32(nnz);
    std::vector<uint16_t> b16(nnz);
    orc_round_values(1, nnz, m.val.data(), b32.data());
    orc_widen_values(1, nnz, b32.data(), wide.data());
    CHECK(wide == m.val, "matrix %d: binary32 round trip", idx);
    for (int dt = 2; dt <= 3; ++dt) {
        orc_round_values(dt, nnz, m.val.data(), b16.data());
        orc_widen_values(dt, nnz, b16.data(), wide.data());
        CHECK(wide == m.val, "matrix %d: 16-bit round trip (%d)", idx, dt);
    }
}

void check_rounding() {
    // values across every binade of the three formats, subnormals and overflow
    const int64_t m = 4096;
    std::vector<double> v(m), u(m), w(m);
    gen_normal(m, 9, 2, v.data());
    gen_unif_stream(m, 9, 3, u.data());
    for (int64_t i = 0; i < m; ++i) v[i] = std::ldexp(v[i], (int)(u[i] * 300.0) - 150);
    std::vector<uint32_t> b32(m);
    std::vector<uint16_t> b16(m);
    orc_round_values(1, m, v.data(), b32.data());
    orc_widen_values(1, m, b32.data(), w.data());
    for (int64_t i = 0; i < m; ++i) {
        const float f = (float)v[i];   // the host's conversion rounds to nearest even
        CHECK((double)f == w[i], "binary32 of %.17g: %.17g vs %.9g", v[i], w[i], (double)f);
    }
    for (int dt = 2; dt <= 3; ++dt) {
        orc_round_values(dt, m, v.data(), b16.data());
        orc_widen_values(dt, m, b16.data(), w.data());
        for (int64_t i = 0; i < m; ++i)
            CHECK(std::isinf(w[i]) || std::fabs(w[i] - v[i]) <= std::fabs(v[i]) * (dt == 2 ? 0x1p-8 : 0x1p-11) + 0x1p-24,
                  "16-bit (%d) of %.17g: %.17g", dt, v[i], w[i]);
    }
}

void check_dmat_extremes() {
    // n - 1 rows of length a and one of length b: moments large enough that
    // n s2 - s1^2 needs all 128 bits
    std::mt19937_64 r(5);
    for (int t = 0; t < 20000; ++t) {
        const int32_t n = (int32_t)(1 + r() % 0x7fffffffu);
        const uint64_t a = r() % (1ull << (r() % 31)), b = r() % (1ull << 31);
        const unsigned __int128 S1 = (unsigned __int128)(uint64_t)(n - 1) * a + b;
        const unsigned __int128 S2 = (unsigned __int128)(uint64_t)(n - 1) * a * a + (unsigned __int128)b * b;
        if (S1 >> 63 || S2 >> 63) continue;   // the moments are int64 in the interface
        double mu, sg, d;
        orc_dmat(n, (int64_t)S1, (int64_t)S2, &mu, &sg, &d);
        spmv_stats st{};
        spmvat::dmat_from_moments(n, (uint64_t)S1, (uint64_t)S2, &st);
        CHECK(st.mu == mu && st.sigma == sg && st.d_mat == d, "D_mat n=%d a=%llu b=%llu: %.17g vs %.17g", n,
              (unsigned long long)a, (unsigned long long)b, st.d_mat, d);
    }
}

void check_arena() {
    const size_t cap = 1 << 20;
    spmv_arena* A = spmv_arena_create(cap + 100);   // the capacity is rounded down to the grain
    CHECK(spmv_arena_free_bytes(A) == cap, "arena capacity");
    CHECK(spmv_arena_alloc(A, SIZE_MAX) == -1, "SIZE_MAX allocation");
    CHECK(spmv_arena_alloc(A, SIZE_MAX - 100) == -1, "near-SIZE_MAX allocation");
    CHECK(spmv_arena_alloc(A, cap + 1) == -1, "oversized allocation");
    // random alloc / free against a model of the live blocks
    std::map<int64_t, size_t> live;
    std::mt19937_64 r(3);
    for (int t = 0; t < 20000; ++t) {
        if (!live.empty() && r() % 2) {
            auto it = live.begin();
            std::advance(it, (long)(r() % live.size()));
            spmv_arena_free(A, it->first, it->second);
            spmv_arena_free(A, it->first, it->second);   // a second free of the same block is ignored
            live.erase(it);
        } else {
            const size_t b = 1 + r() % 20000;
            const int64_t o = spmv_arena_alloc(A, b);
            if (o >= 0) {
                const size_t rb = (b + 255) / 256 * 256;
                auto nx = live.lower_bound(o);
                CHECK(nx == live.end() || (size_t)o + rb <= (size_t)nx->first, "overlap with a later block");
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    CHECK((size_t)pv->first + (pv->second + 255) / 256 * 256 <= (size_t)o, "overlap with an earlier block");
                }
                live[o] = b;
            }
        }
        size_t used = 0;
        for (auto& kv : live) used += (kv.second + 255) / 256 * 256;
        CHECK(spmv_arena_free_bytes(A) + used == cap, "free bytes at step %d", t);
    }
    spmv_arena_free(A, -256, 256);                    // outside the arena: ignored
    spmv_arena_free(A, (int64_t)cap, 256);
    spmv_arena_free(A, 0, SIZE_MAX);
    for (auto& kv : live) spmv_arena_free(A, kv.first, kv.second);
    CHECK(spmv_arena_free_bytes(A) == cap && spmv_arena_largest(A) == cap, "arena coalesced at the end");
    spmv_arena_destroy(A);
    spmv_arena_destroy(nullptr);
}

void check_decisions() {
    std::mt19937_64 r(17);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const double inf = std::numeric_limits<double>::infinity();
    for (int t = 0; t < 20000; ++t) {
        spmv_stats st{};
        st.n = (int32_t)(1 + r() % (t % 3 == 0 ? 0x7fffffffu : 100000u));
        st.max_row = (int32_t)(r() % (t % 5 == 0 ? 0x7fffffffu : 5000u));
        st.nnz = (int64_t)(U(r) * st.n * (double)st.max_row);
        st.d_mat = t % 7 == 0 ? std::nan("") : U(r) * 4.0;
        st.bandwidth = (int32_t)(r() % 0x7fffffffu);
        at_table tab{};
        tab.c = 1.0;
        tab.d_star = t % 11 == 0 ? inf : U(r) * 2.0;
        tab.calibrated = (int32_t)(r() % 2);
        for (auto& a : tab.spmv_bps) for (auto& b : a) for (auto& c : b) for (auto& v : c) v = t % 13 == 0 ? 0.0 : 1e12 * U(r);
        for (auto& a : tab.trans_bps) for (auto& b : a) for (auto& v : b) v = 1e12 * U(r);
        tab.launch_s = 1e-5 * U(r);
        tab.k_margin = t % 2 ? 0.0 : 1.0 + U(r);
        const spmv_dtype dt = (spmv_dtype)(r() % 4);
        const size_t limit = (size_t)(r() % (1ull << 40));
        const int64_t k = t % 4 == 0 ? 0 : (int64_t)(r() % 1000);
        spmv_format f;
        int var;
        at_decision why{};
        CHECK(at_choose_format_stats(&st, dt, limit, &tab, k, &f, &var, &why) == SPMV_OK, "decision status");
        CHECK(f == SPMV_CRS || f == SPMV_COO_ROW || f == SPMV_ELL_ROW, "format %d", (int)f);
        CHECK(f != SPMV_ELL_ROW || why.feasible_ell, "ELL-Row chosen while it does not fit");
        if (why.rule == 0)
            CHECK((f == SPMV_ELL_ROW) == (why.feasible_ell && st.d_mat < tab.d_star), "the paper's rule");
        CHECK(f == SPMV_CRS || !(why.k_break_even < 0), "break-even count %g", why.k_break_even);
    }
    // argument checks
    spmv_stats st{};
    at_table tab{};
    spmv_format f;
    int var;
    CHECK(at_choose_format_stats(&st, SPMV_F64, 0, &tab, 0, &f, &var, nullptr) == SPMV_E_ARG, "n = 0 refused");
    st.n = 1;
    CHECK(at_choose_format_stats(&st, (spmv_dtype)7, 0, &tab, 0, &f, &var, nullptr) == SPMV_E_ARG, "bad dtype refused");
    CHECK(at_choose_format_stats(nullptr, SPMV_F64, 0, &tab, 0, &f, &var, nullptr) == SPMV_E_ARG, "null stats refused");
    // D* of a table
    const double d[5] = {0.0, 0.1, 0.2, 0.3, std::nan("")};
    const double rr[5] = {2.0, 1.5, 0.9, 0.5, 0.1};
    const int32_t feas[5] = {1, 1, 0, 1, 1};
    CHECK(at_table_build(d, rr, feas, 5, 1.0, &tab) == SPMV_OK && tab.d_star == 0.3, "D* %g", tab.d_star);
    CHECK(at_table_build(d, rr, nullptr, 5, 1.0, &tab) == SPMV_OK && tab.d_star == 0.2, "D* without feasibility");
    CHECK(at_table_build(nullptr, nullptr, nullptr, 0, 1.0, &tab) == SPMV_OK && std::isinf(tab.d_star), "empty table");
    CHECK(at_table_build(d, rr, nullptr, -1, 1.0, &tab) == SPMV_E_ARG, "negative count refused");
}

}  // namespace

int main() {
    int idx = 0;
    for (const Crs& m : matrices()) check_matrix(m, idx++);
    check_rounding();
    check_dmat_extremes();
    check_arena();
    check_decisions();
    std::printf("%s: %d matrices, %d failures\n", g_fail ? "FAILED" : "ok", idx, g_fail);
    return g_fail ? 1 : 0;
}
