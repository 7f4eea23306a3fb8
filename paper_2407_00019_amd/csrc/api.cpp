// C ABI of libspmvat (include/spmvat.h): plans, transformations, SpMV
// dispatch and the auto-tuner's host-side decisions (section 2.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/spmvat.h"
#include "host_core.h"
#include "kernels.h"
#include "plan_internal.h"

using namespace spmvat;

#define SPMV_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr size_t kAlign = 256;

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

spmv_status hip_fail(const spmv_plan* p, hipError_t e) {
    if (p) const_cast<spmv_plan*>(p)->err = hipGetErrorString(e);
    return SPMV_E_HIP;
}

#define HIP_TRY(p, call)                                       \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail((p), e_);        \
    } while (0)

// Plan workspace layout: [RowStats | row-statistics partials | COO carries].
inline size_t stats_bytes() {
    return round_up(sizeof(RowStats), kAlign) + round_up(row_stats_partial_count() * sizeof(RowStats), kAlign);
}
inline size_t plan_ws_bytes(int64_t nnz) { return stats_bytes() + round_up(coo_carry_bytes(nnz), kAlign); }
inline RowStats* plan_rowstats(const spmv_plan* p) { return reinterpret_cast<RowStats*>(p->work); }
inline RowStats* plan_partials(const spmv_plan* p) {
    return reinterpret_cast<RowStats*>(p->work + round_up(sizeof(RowStats), kAlign));
}
inline void* plan_carries(const spmv_plan* p) { return p->work + stats_bytes(); }

size_t crs_bytes(const spmv_plan* p) {
    return (size_t)(p->n + 1) * 4 + (size_t)p->nnz * (4 + (size_t)vbytes_of(p->dt));
}

// CRS -> CCS algorithm (spmv_ccs_algorithm).  Chosen by the matrix's
// structure unless the plan names one: limited bandwidth (a row tile's
// window of 64-column blocks fits the kernels' LDS) takes the banded
// two-level counting sort, everything else the radix sort by column.  The
// sort and bucketed routes stay selectable.
bool ccs_banded_ok(int32_t n, int32_t bw, int32_t max_row) { return wccs_geom(n, bw, max_row).usable; }
bool ccs_bucketed_ok(int32_t n) { return n <= (1 << kCcsRowBits); }

int ccs_route(int32_t n, int32_t bw, int32_t max_row, int alg) {
    if (alg != SPMV_CCS_AUTO) return alg;
    if (ccs_banded_ok(n, bw, max_row)) return SPMV_CCS_BANDED;
    return SPMV_CCS_RADIX;
}

// CCS workspace layout: bucketed -- count table, its chunk sums, summary,
// level-1 keys and values; else -- counts/cursors, scan sums and maxima,
// long-column lists and their extents, summary, the windowed route's flags,
// then one region holding either the windowed route's bitmaps and count
// table or the sort route's keys and merge scratch.
struct CcsWs {
    size_t cursor, bsum, mid, lng, ext, sum, info, keys, tmp;   // sort and windowed routes
    size_t wtable, bstart, wflag, wkey, wval;                 // windowed route (overlays keys)
    size_t table, csum, bkey, bval;                           // bucketed route
    size_t xcol, xrow, xval, ycol, yrow, yval;                // radix route (with table, csum, sum)
    size_t total;
};
CcsWs ccs_ws(int32_t n, int64_t nnz, int vb, int32_t bw, int32_t max_row, int alg) {
    CcsWs w{};
    size_t o = 0;
    const int route = ccs_route(n, bw, max_row, alg);
    if (route == SPMV_CCS_RADIX) {
        const RadixGeom g = radix_geom(n, nnz);
        const size_t e4 = round_up((size_t)std::max<int64_t>(nnz, 1) * 4, kAlign);
        const size_t ev = round_up((size_t)std::max<int64_t>(nnz, 1) * vb, kAlign);
        w.xcol = o; o += e4;
        w.xrow = o; o += e4;
        w.xval = o; o += ev;
        w.ycol = o; o += e4;
        w.yrow = o; o += e4;
        w.yval = o; o += ev;
        w.table = o; o += round_up((size_t)std::max<int64_t>(g.table, 1) * 4, kAlign);
        w.csum = o;  o += round_up((size_t)std::max<int64_t>(g.chunks, 1) * 4, kAlign);
        w.sum = o;   o += round_up(sizeof(ColSummary), kAlign);
        w.total = o;
        return w;
    }
    if (route == SPMV_CCS_BUCKETED) {
        const CcsGeom g = ccs_geom(n);
        w.table = o; o += round_up((size_t)g.table * 4, kAlign);
        w.csum = o;  o += round_up((size_t)g.chunks * 4, kAlign);
        w.sum = o;   o += round_up(sizeof(ColSummary), kAlign);
        w.bkey = o;  o += round_up((size_t)nnz * 4, kAlign);
        w.bval = o;  o += round_up((size_t)nnz * vb, kAlign);
        w.total = o;
        return w;
    }
    w.cursor = o; o += round_up((size_t)n * 4, kAlign);
    w.bsum = o;   o += round_up(col_scan_bsum_count(n) * 8, kAlign);
    const size_t nmid = std::min<size_t>((size_t)n, (size_t)(nnz / (kSortSmall + 1)) + 1);
    const size_t nlong = std::min<size_t>((size_t)n, (size_t)(nnz / (kSortMid + 1)) + 1);
    w.mid = o;    o += round_up(nmid * 4, kAlign);
    w.lng = o;    o += round_up(nlong * 4, kAlign);
    w.ext = o;    o += round_up(nlong * 8, kAlign);
    w.sum = o;    o += round_up(sizeof(ColSummary), kAlign);
    w.info = o;   o += round_up(sizeof(WccsInfo), kAlign);
    w.keys = o;
    const size_t sort_bytes = round_up((size_t)nnz * 8, kAlign) + round_up((size_t)std::min<int64_t>(n, nnz) * 8, kAlign);
    w.tmp = o + round_up((size_t)nnz * 8, kAlign);
    size_t win_bytes = 0;
    if (route == SPMV_CCS_BANDED) {
        const WccsGeom g = wccs_geom(n, bw, max_row);
        size_t q = o;
        w.wtable = q; q += round_up((size_t)g.table * 4, kAlign);
        w.bstart = q; q += round_up(((size_t)g.nb + 1) * 4, kAlign);
        w.wflag = q;  q += round_up((size_t)g.stretches * 4, kAlign);
        w.wkey = q;   q += round_up((size_t)nnz * 4, kAlign);
        w.wval = q;   q += round_up((size_t)nnz * vb, kAlign);
        win_bytes = q - o;
    }
    o += std::max(sort_bytes, win_bytes);
    w.total = o;
    return w;
}

// Pinned host records for the small results a call reads back (the row
// statistics of spmv_plan_create, the summaries of csr_to_ccs): taken for
// the call and returned after it, so their number is the most calls that
// ever ran at once, whatever threads made them.  A copy into pinned memory
// is one DMA with no staging, so a call's read-backs queue behind its
// kernels and one synchronisation ends them all.
struct HostRec {
    alignas(64) unsigned char bytes[64];
};
static_assert(sizeof(RowStats) <= sizeof(HostRec), "row statistics fit a record");
static_assert(sizeof(ColSummary) + sizeof(WccsInfo) <= sizeof(HostRec), "CCS summaries fit a record");

std::mutex g_pinned_mu;
std::vector<HostRec*> g_pinned_free;

HostRec* pinned_take() {
    {
        std::lock_guard<std::mutex> g(g_pinned_mu);
        if (!g_pinned_free.empty()) {
            HostRec* r = g_pinned_free.back();
            g_pinned_free.pop_back();
            return r;
        }
    }
    HostRec* r = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&r), sizeof(HostRec), hipHostMallocCoherent) != hipSuccess)
        return nullptr;
    return r;
}

void pinned_give(HostRec* r) {
    std::lock_guard<std::mutex> g(g_pinned_mu);
    g_pinned_free.push_back(r);
}

// A record held for one call: returned on every way out of it, after the
// stream has passed any copy still bound for it.
struct HeldRec {
    HostRec* r = pinned_take();
    hipStream_t s;
    bool pending = false;
    explicit HeldRec(hipStream_t st) : s(st) {}
    HeldRec(const HeldRec&) = delete;
    HeldRec& operator=(const HeldRec&) = delete;
    ~HeldRec() {
        if (!r) return;
        if (pending) (void)hipStreamSynchronize(s);
        pinned_give(r);
    }
    // copies bytes from the device into the record at offset `at`
    hipError_t fetch(size_t at, const void* src, size_t bytes) {
        pending = true;
        return hipMemcpyAsync(r->bytes + at, src, bytes, hipMemcpyDeviceToHost, s);
    }
    hipError_t wait() {
        const hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess) pending = false;
        return e;
    }
    template <typename T> T get(size_t at) const {
        T v;
        std::memcpy(&v, r->bytes + at, sizeof(T));
        return v;
    }
};

bool check_buffers(const spmv_buffers* out, int count, const spmv_sizes& need) {
    if (!out) return false;
    for (int k = 0; k < count; ++k) {
        if (need.bytes[k] == 0) continue;
        if (!out->ptr[k] || !aligned16(out->ptr[k]) || out->bytes[k] < need.bytes[k]) return false;
    }
    return true;
}

}  // namespace

// ------------------------------------------------------------------ plan

SPMV_API size_t spmv_plan_workspace_bytes(int32_t n, int64_t nnz) {
    (void)n;
    return plan_ws_bytes(nnz < 0 ? 0 : nnz);
}

namespace spmvat {

spmv_status plan_begin(spmv_plan* p, int32_t n, int64_t nnz, const int32_t* irp, const int32_t* icol,
                       const void* val, spmv_dtype val_type, void* plan_work, size_t plan_work_bytes,
                       RowStats* host_stats, hipStream_t s) {
    if (n < 1 || nnz < 0 || nnz > SPMV_MAX_NNZ || !valid_dtype(val_type)) return SPMV_E_ARG;
    if (!irp || !plan_work || (nnz > 0 && (!icol || !val))) return SPMV_E_ARG;
    if (!aligned16(irp) || !aligned16(icol) || !aligned16(val) || !aligned16(plan_work)) return SPMV_E_ARG;
    if (plan_work_bytes < plan_ws_bytes(nnz)) return SPMV_E_ARG;
    p->n = n; p->nnz = nnz; p->dt = val_type;
    p->irp = irp; p->icol = icol; p->val = val;
    p->work = static_cast<char*>(plan_work); p->work_bytes = plan_work_bytes;
    // the final statistics kernel writes the result straight into the pinned
    // host buffer: no copy command after it
    const hipError_t e = launch_row_stats(n, nnz, irp, icol, plan_partials(p), plan_rowstats(p), host_stats, s);
    return e == hipSuccess ? SPMV_OK : hip_fail(p, e);
}

spmv_status plan_finish(spmv_plan* p, const RowStats& rs) {
    if (rs.flags != 0) return SPMV_E_MATRIX;
    const int32_t n = p->n;
    spmv_stats& st = p->st;
    st.n = n; st.nnz = p->nnz;
    st.sum_len = (int64_t)rs.s1; st.sum_len2 = (int64_t)rs.s2;
    st.max_row = rs.max_len; st.min_row = (int32_t)rs.min_len; st.max_col = -1; st.bandwidth = rs.max_band;
    dmat_from_moments(n, rs.s1, rs.s2, &st);   // Eq. (4)
    p->limit = 8 * crs_bytes(p);
    return SPMV_OK;
}

}  // namespace spmvat

SPMV_API spmv_status spmv_plan_create(spmv_plan** plan, int32_t n, int64_t nnz, const int32_t* irp,
                                      const int32_t* icol, const void* val, spmv_dtype val_type,
                                      void* plan_work, size_t plan_work_bytes, void* stream) {
    if (!plan) return SPMV_E_ARG;
    *plan = nullptr;
    // sizes first: a rejected matrix touches neither the host heap nor HIP
    if (n < 1 || nnz < 0 || nnz > SPMV_MAX_NNZ || !valid_dtype(val_type)) return SPMV_E_ARG;
    spmv_plan* p = new (std::nothrow) spmv_plan();
    if (!p) return SPMV_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // a pinned record receives the statistics straight from the kernel
    HostRec* rec = pinned_take();
    if (!rec) {
        delete p;
        return SPMV_E_HIP;
    }
    RowStats* pinned = reinterpret_cast<RowStats*>(rec->bytes);
    spmv_status st = plan_begin(p, n, nnz, irp, icol, val, val_type, plan_work, plan_work_bytes, pinned, s);
    if (st == SPMV_OK && hipStreamSynchronize(s) != hipSuccess) st = SPMV_E_HIP;
    if (st == SPMV_OK) st = plan_finish(p, *pinned);
    // the record goes back only once nothing on the stream can still write it
    if (st == SPMV_E_HIP) (void)hipStreamSynchronize(s);
    pinned_give(rec);
    if (st != SPMV_OK) { delete p; return st; }
    *plan = p;
    return SPMV_OK;
}

SPMV_API spmv_status spmv_plan_stats(const spmv_plan* p, spmv_stats* out) {
    if (!p || !out) return SPMV_E_ARG;
    *out = p->st;
    return SPMV_OK;
}

SPMV_API spmv_status spmv_plan_value_type(const spmv_plan* p, spmv_dtype* out) {
    if (!p || !out) return SPMV_E_ARG;
    *out = p->dt;
    return SPMV_OK;
}

SPMV_API spmv_status spmv_plan_set_limit(spmv_plan* p, size_t max_format_bytes) {
    if (!p) return SPMV_E_ARG;
    p->limit = max_format_bytes;
    return SPMV_OK;
}

SPMV_API spmv_status spmv_plan_set_ccs_algorithm(spmv_plan* p, spmv_ccs_algorithm alg) {
    if (!p) return SPMV_E_ARG;
    switch (alg) {
        case SPMV_CCS_AUTO:
        case SPMV_CCS_SORT:
        case SPMV_CCS_RADIX:
            break;
        case SPMV_CCS_BUCKETED:
            if (!ccs_bucketed_ok(p->n)) return SPMV_E_ARG;
            break;
        case SPMV_CCS_BANDED:
            if (!ccs_banded_ok(p->n, p->st.bandwidth, p->st.max_row)) return SPMV_E_ARG;
            break;
        default:
            return SPMV_E_ARG;
    }
    p->ccs_alg = alg;
    return SPMV_OK;
}

SPMV_API void spmv_plan_destroy(spmv_plan* p) { delete p; }

SPMV_API const char* spmv_status_string(spmv_status s) {
    switch (s) {
        case SPMV_OK: return "ok";
        case SPMV_E_ARG: return "invalid argument";
        case SPMV_E_MATRIX: return "matrix breaks the CRS contract";
        case SPMV_E_TOO_LARGE: return "format exceeds the memory limit";
        case SPMV_E_NOT_READY: return "format not built";
        case SPMV_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

SPMV_API const char* spmv_plan_last_error(const spmv_plan* p) { return p ? p->err.c_str() : ""; }

// ------------------------------------------------------------------ sizes

SPMV_API spmv_status spmv_buffer_sizes(const spmv_plan* p, spmv_format f, spmv_sizes* out) {
    if (!p || !out) return SPMV_E_ARG;
    std::memset(out, 0, sizeof(*out));
    const size_t nnz = (size_t)p->nnz, n = (size_t)p->n, vb = (size_t)vbytes_of(p->dt);
    switch (f) {
        case SPMV_COO_ROW:
            out->bytes[0] = nnz * 4;
            return SPMV_OK;
        case SPMV_CCS:
            out->bytes[0] = (n + 1) * 4;
            out->bytes[1] = nnz * 4;
            out->bytes[2] = nnz * vb;
            out->workspace = ccs_ws(p->n, p->nnz, vbytes_of(p->dt), p->st.bandwidth, p->st.max_row, p->ccs_alg).total;
            return SPMV_OK;
        case SPMV_COO_COL:
            out->bytes[0] = nnz * 4;
            return SPMV_OK;
        case SPMV_ELL_ROW:
        case SPMV_ELL_COL: {
            int32_t w = f == SPMV_ELL_ROW ? p->st.max_row : p->st.max_col;
            if (w < 0) return SPMV_E_NOT_READY;
            out->width = w;
            const unsigned __int128 slots = (unsigned __int128)w * n;
            if (slots > (unsigned __int128)(SIZE_MAX / 16)) return SPMV_E_TOO_LARGE;
            out->bytes[0] = (size_t)slots * vb;
            out->bytes[1] = (size_t)slots * 4;
            if (out->bytes[0] + out->bytes[1] > p->limit) return SPMV_E_TOO_LARGE;
            return SPMV_OK;
        }
        default:
            return SPMV_E_ARG;
    }
}

// ------------------------------------------------------- transformations

SPMV_API spmv_status csr_to_coo(spmv_plan* p, int column_wise, const spmv_buffers* out, void* work,
                                size_t work_bytes, void* stream) {
    (void)work; (void)work_bytes;
    if (!p) return SPMV_E_ARG;
    if (!column_wise && p->crs_consumed) return SPMV_E_NOT_READY;
    spmv_sizes need;
    spmv_status st = spmv_buffer_sizes(p, column_wise ? SPMV_COO_COL : SPMV_COO_ROW, &need);
    if (st != SPMV_OK) return st;
    if (column_wise && !p->has_ccs) return SPMV_E_NOT_READY;
    if (!check_buffers(out, 1, need)) return SPMV_E_ARG;
    if (need.bytes[0] > p->limit) return SPMV_E_TOO_LARGE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t* dst = static_cast<int32_t*>(out->ptr[0]);
    if (p->nnz > 0) HIP_TRY(p, launch_expand_ptr(p->n, column_wise ? p->ccp : p->irp, dst, s));
    if (column_wise) { p->jcol = dst; p->has_coo_col = true; }
    else { p->irow = dst; p->has_coo_row = true; }
    return SPMV_OK;
}

SPMV_API spmv_status csr_to_ccs(spmv_plan* p, const spmv_buffers* out, void* work, size_t work_bytes,
                                void* stream) {
    if (!p) return SPMV_E_ARG;
    if (p->crs_consumed) return SPMV_E_NOT_READY;
    spmv_sizes need;
    spmv_status st = spmv_buffer_sizes(p, SPMV_CCS, &need);
    if (st != SPMV_OK) return st;
    if (!check_buffers(out, 3, need)) return SPMV_E_ARG;
    if (need.bytes[0] + need.bytes[1] + need.bytes[2] > p->limit) return SPMV_E_TOO_LARGE;
    if (!work || !aligned16(work) || work_bytes < need.workspace) return SPMV_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int vb = vbytes_of(p->dt);
    const int32_t bw = p->st.bandwidth, mr = p->st.max_row;
    const int route = ccs_route(p->n, bw, mr, p->ccs_alg);
    const CcsWs w = ccs_ws(p->n, p->nnz, vb, bw, mr, p->ccs_alg);
    char* base = static_cast<char*>(work);
    int32_t* ccp = static_cast<int32_t*>(out->ptr[0]);
    int32_t* irow_t = static_cast<int32_t*>(out->ptr[1]);
    void* val_t = out->ptr[2];
    ColSummary* dsum = reinterpret_cast<ColSummary*>(base + w.sum);
    ColSummary cs{};
    // the summaries come back through one pinned record: [ColSummary | WccsInfo]
    HeldRec rec(s);
    if (!rec.r) return SPMV_E_HIP;
    constexpr size_t kAtInfo = sizeof(ColSummary);
    auto built = [&]() {
        p->ccp = ccp; p->irow_t = irow_t; p->val_t = val_t; p->has_ccs = true;
        p->st.max_col = cs.max_len;
        p->jcol = nullptr; p->has_coo_col = false;   // a rebuilt CCS invalidates the formats built on it
        p->ellc_w = -1; p->ellc_val = nullptr; p->ellc_row = nullptr;
        return SPMV_OK;
    };

    if (route == SPMV_CCS_RADIX) {
        // passes of a stable counting sort by 8-bit column digits, least
        // significant first; the column pointer from the sorted columns; one
        // sync at the end for the longest column
        const RadixGeom g = radix_geom(p->n, p->nnz);
        RadixWs rw{};
        rw.xcol = reinterpret_cast<int32_t*>(base + w.xcol);
        rw.xrow = reinterpret_cast<int32_t*>(base + w.xrow);
        rw.xval = base + w.xval;
        rw.ycol = reinterpret_cast<int32_t*>(base + w.ycol);
        rw.yrow = reinterpret_cast<int32_t*>(base + w.yrow);
        rw.yval = base + w.yval;
        rw.table = reinterpret_cast<int32_t*>(base + w.table);
        rw.csum = reinterpret_cast<int32_t*>(base + w.csum);
        if (p->nnz == 0) HIP_TRY(p, launch_fill_zero(ccp, ((int64_t)p->n + 1) * 4, s));
        HIP_TRY(p, launch_ccs_radix(g, p->n, p->nnz, p->irp, p->icol, p->val, vb, rw, ccp, irow_t, val_t, dsum, s));
        HIP_TRY(p, rec.fetch(0, dsum, sizeof(cs)));
        HIP_TRY(p, rec.wait());
        cs = rec.get<ColSummary>(0);
        if ((int64_t)cs.total != p->nnz) {
            p->err = "column pointer does not end at nnz";
            return SPMV_E_HIP;
        }
        return built();
    }
    if (route == SPMV_CCS_BUCKETED) {
        // level 1 (count table, its scan, ordered distribution to column
        // blocks) and level 2 (ordered placement inside each block); one sync
        // at the end for the longest column
        const CcsGeom g = ccs_geom(p->n);
        HIP_TRY(p, launch_ccs_bucketed(g, p->n, p->nnz, p->irp, p->icol, p->val, vb,
                                       reinterpret_cast<int32_t*>(base + w.table),
                                       reinterpret_cast<int32_t*>(base + w.csum),
                                       reinterpret_cast<uint32_t*>(base + w.bkey), base + w.bval, ccp, irow_t, val_t,
                                       dsum, s));
        HIP_TRY(p, rec.fetch(0, dsum, sizeof(cs)));
        HIP_TRY(p, rec.wait());
        cs = rec.get<ColSummary>(0);
        if ((int64_t)cs.total != p->nnz) {
            p->err = "column-block counts do not add up to nnz";
            return SPMV_E_HIP;
        }
        return built();
    }
    int32_t* cursor = reinterpret_cast<int32_t*>(base + w.cursor);
    int32_t* bsum = reinterpret_cast<int32_t*>(base + w.bsum);
    int32_t* mid = reinterpret_cast<int32_t*>(base + w.mid);
    int32_t* lng = reinterpret_cast<int32_t*>(base + w.lng);
    int32_t* ext = reinterpret_cast<int32_t*>(base + w.ext);
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(base + w.keys);
    unsigned long long* tmp = reinterpret_cast<unsigned long long*>(base + w.tmp);

    if (p->nnz > 0 && route == SPMV_CCS_BANDED) {
        // (1) per-(tile, wave) counts over the window blocks, per-block walk
        // -> block lengths, scan -> block starts, (2) ordered distribution to
        // the blocks, per-block placement; one sync at the end
        const WccsGeom g = wccs_geom(p->n, bw, mr);
        int32_t* table = reinterpret_cast<int32_t*>(base + w.wtable);
        int32_t* bstart = reinterpret_cast<int32_t*>(base + w.bstart);
        WccsInfo* dinfo = reinterpret_cast<WccsInfo*>(base + w.info);
        WccsInfo wi{};
        HIP_TRY(p, launch_wccs_front(g, p->n, bw, p->irp, p->icol, table, cursor,
                                     reinterpret_cast<int32_t*>(base + w.wflag), dinfo, s));
        HIP_TRY(p, launch_wccs_scan(g, cursor, bstart, bsum, dsum, s));
        HIP_TRY(p, launch_wccs_back(g, p->n, bw, vb, p->irp, p->icol, p->val, table, bstart,
                                    reinterpret_cast<uint32_t*>(base + w.wkey), base + w.wval, ccp, irow_t, val_t,
                                    dinfo, s));
        HIP_TRY(p, rec.fetch(0, dsum, sizeof(cs)));
        HIP_TRY(p, rec.fetch(kAtInfo, dinfo, sizeof(wi)));
        HIP_TRY(p, rec.wait());
        cs = rec.get<ColSummary>(0);
        wi = rec.get<WccsInfo>(kAtInfo);
        if (wi.flags & kWccsOutside) {
            p->err = "a column index lies outside the bandwidth measured when the plan was made";
            return SPMV_E_MATRIX;
        }
        if ((int64_t)cs.total != p->nnz) {
            p->err = "column counts do not add up to nnz";
            return SPMV_E_HIP;
        }
        cs.max_len = wi.kmax;
        return built();
    }
    // (1) column counts, (2) exclusive scan -> ccp and cursors
    HIP_TRY(p, hipMemsetAsync(cursor, 0, (size_t)p->n * 4, s));
    if (p->nnz > 0) HIP_TRY(p, launch_col_count(p->n, p->st.bandwidth, p->irp, p->icol, cursor, s));
    HIP_TRY(p, launch_col_scan(p->n, cursor, ccp, cursor, bsum, mid, lng, dsum, s));
    HIP_TRY(p, rec.fetch(0, dsum, sizeof(cs)));
    HIP_TRY(p, rec.wait());
    cs = rec.get<ColSummary>(0);
    if ((int64_t)cs.total != p->nnz) {
        p->err = "column counts do not add up to nnz";
        return SPMV_E_HIP;
    }
    if (p->nnz > 0) {
        // (3) scatter of packed (position, row) keys, (4) per-column sort + emit
        HIP_TRY(p, launch_ccs_scatter(p->n, p->st.bandwidth, p->irp, p->icol, cursor, keys, s));
        HIP_TRY(p, launch_ccs_sort_small(p->n, ccp, keys, p->val, vb, irow_t, val_t, s));
        HIP_TRY(p, launch_ccs_sort_mid(cs.n_mid, mid, ccp, keys, p->val, vb, irow_t, val_t, s));
        if (cs.n_long > 0) {
            // every long column's (start, end) in one copy
            std::vector<int32_t> se((size_t)cs.n_long * 2);
            HIP_TRY(p, launch_col_extents(cs.n_long, lng, ccp, ext, s));
            HIP_TRY(p, hipMemcpyAsync(se.data(), ext, se.size() * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(p, hipStreamSynchronize(s));
            for (int32_t i = 0; i < cs.n_long; ++i) {
                const int32_t start = se[2 * (size_t)i], len = se[2 * (size_t)i + 1] - start;
                // the merge passes need len keys of scratch; longer columns (only
                // possible with duplicate entries) rank without scratch
                const size_t cap = (size_t)std::min<int64_t>(p->n, p->nnz);
                HIP_TRY(p, launch_ccs_sort_long(start, len, keys, (size_t)len <= cap ? tmp : nullptr, p->val, vb,
                                                irow_t, val_t, s));
            }
        }
    }
    return built();
}

// Temporary CCS arrays at the front of the in-place workspace, then the
// workspace of csr_to_ccs.
namespace {
struct InplaceWs {
    size_t ccp, irow, val, ccs_work, ccs_work_bytes, total;
};
InplaceWs inplace_ws(const spmv_plan* p) {
    InplaceWs w{};
    spmv_sizes sz{};
    (void)spmv_buffer_sizes(p, SPMV_CCS, &sz);
    size_t o = 0;
    w.ccp = o;  o += round_up(sz.bytes[0], kAlign);
    w.irow = o; o += round_up(std::max<size_t>(sz.bytes[1], 1), kAlign);
    w.val = o;  o += round_up(std::max<size_t>(sz.bytes[2], 1), kAlign);
    w.ccs_work = o;
    w.ccs_work_bytes = sz.workspace;
    o += round_up(sz.workspace, kAlign);
    w.total = o;
    return w;
}
}  // namespace

SPMV_API spmv_status spmv_ccs_inplace_workspace_bytes(const spmv_plan* p, size_t* bytes) {
    if (!p || !bytes) return SPMV_E_ARG;
    *bytes = inplace_ws(p).total;
    return SPMV_OK;
}

SPMV_API spmv_status csr_to_ccs_inplace(spmv_plan* p, int32_t* irp, int32_t* icol, void* val, void* work,
                                        size_t work_bytes, void* stream) {
    if (!p) return SPMV_E_ARG;
    if (p->crs_consumed) return SPMV_E_NOT_READY;
    // the caller hands back, writable, the very arrays the plan borrowed
    if (irp != p->irp || icol != p->icol || val != p->val) return SPMV_E_ARG;
    const InplaceWs w = inplace_ws(p);
    if (!work || !aligned16(work) || work_bytes < w.total) return SPMV_E_ARG;
    spmv_sizes need{};
    spmv_status st = spmv_buffer_sizes(p, SPMV_CCS, &need);
    if (st != SPMV_OK) return st;
    char* base = static_cast<char*>(work);
    spmv_buffers tmp{};
    for (int k = 0; k < 3; ++k) tmp.bytes[k] = std::max<size_t>(need.bytes[k], 16);
    tmp.ptr[0] = base + w.ccp;
    tmp.ptr[1] = base + w.irow;
    tmp.ptr[2] = base + w.val;
    // the limit guards the extra arrays of a transformation; here they are
    // temporary and the result takes the CRS arrays' place
    const size_t limit = p->limit;
    p->limit = SIZE_MAX;
    st = csr_to_ccs(p, &tmp, base + w.ccs_work, w.ccs_work_bytes, stream);
    p->limit = limit;
    if (st != SPMV_OK) return st;
    // the copy-back of Phase I: column pointers over IRP, rows over ICOL,
    // values over VAL (the same sizes: n + 1, nnz, nnz)
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(p, hipMemcpyAsync(irp, tmp.ptr[0], need.bytes[0], hipMemcpyDeviceToDevice, s));
    if (p->nnz > 0) {
        HIP_TRY(p, hipMemcpyAsync(icol, tmp.ptr[1], need.bytes[1], hipMemcpyDeviceToDevice, s));
        HIP_TRY(p, hipMemcpyAsync(val, tmp.ptr[2], need.bytes[2], hipMemcpyDeviceToDevice, s));
    }
    p->ccp = irp; p->irow_t = icol; p->val_t = val;
    p->crs_consumed = true;
    p->has_coo_row = false; p->irow = nullptr;   // COO-Row used the CRS ICOL and VAL
    return SPMV_OK;
}

SPMV_API spmv_status csr_to_ell(spmv_plan* p, int column_wise, const spmv_buffers* out, void* work,
                                size_t work_bytes, void* stream) {
    (void)work; (void)work_bytes;
    if (!p) return SPMV_E_ARG;
    if (column_wise && !p->has_ccs) return SPMV_E_NOT_READY;
    if (!column_wise && p->crs_consumed) return SPMV_E_NOT_READY;
    spmv_sizes need;
    spmv_status st = spmv_buffer_sizes(p, column_wise ? SPMV_ELL_COL : SPMV_ELL_ROW, &need);
    if (st != SPMV_OK) return st;
    if (!check_buffers(out, 2, need)) return SPMV_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int vb = vbytes_of(p->dt);
    if (column_wise) {
        HIP_TRY(p, launch_ell_pack(p->n, need.width, p->ccp, p->irow_t, p->val_t, vb, out->ptr[0],
                                   static_cast<int32_t*>(out->ptr[1]), s));
        p->ellc_w = need.width; p->ellc_val = out->ptr[0]; p->ellc_row = static_cast<int32_t*>(out->ptr[1]);
    } else {
        HIP_TRY(p, launch_ell_pack(p->n, need.width, p->irp, p->icol, p->val, vb, out->ptr[0],
                                   static_cast<int32_t*>(out->ptr[1]), s));
        p->ell_w = need.width; p->ell_val = out->ptr[0]; p->ell_col = static_cast<int32_t*>(out->ptr[1]);
    }
    return SPMV_OK;
}

// ------------------------------------------------------------------ SpMV

namespace {

// Column SpMV kernel of a variant: 1 one global atomic per entry, 2 y
// privatised in LDS by pages; 0 takes 2 when the bandwidth lets every
// workgroup's row window fit the page table.
int col_variant(const spmv_plan* p, int variant) {
    if (variant != 0) return variant;
    return col_paged_fits(p->n, p->st.bandwidth) ? 2 : 1;
}

}  // namespace

spmv_status spmvat::plan_exec(const spmv_plan* p, spmv_format f, int variant, const void* x, void* y,
                              double alpha, hipStream_t s) {
    if (!p || !x || !y || !aligned16(x) || !aligned16(y)) return SPMV_E_ARG;
    if (alpha != 1.0 && f != SPMV_CRS && f != SPMV_ELL_ROW) return SPMV_E_ARG;
    const int dt = (int)p->dt;
    const int64_t ybytes = (int64_t)p->n * xbytes_of(p->dt);
    switch (f) {
        case SPMV_CRS: {
            if (variant < 0 || variant > 8) return SPMV_E_ARG;
            if (p->crs_consumed) return SPMV_E_NOT_READY;
            const bool stream = variant == 8 || variant == 1;
            if (variant == 0) HIP_TRY(p, launch_spmv_crs_scalar(dt, p->n, p->irp, p->icol, p->val, x, y, alpha, s));
            else if (stream) HIP_TRY(p, launch_spmv_crs_stream(dt, p->n, p->nnz, p->irp, p->icol, p->val, x, y, alpha, s));
            else {
                const int w = 1 << (variant - 1);
                HIP_TRY(p, launch_spmv_crs_vector(dt, w, p->n, p->irp, p->icol, p->val, x, y, alpha, s));
            }
            return SPMV_OK;
        }
        case SPMV_COO_ROW:
            if (variant != 0) return SPMV_E_ARG;
            if (!p->has_coo_row || p->crs_consumed) return SPMV_E_NOT_READY;
            if (p->st.min_row == 0 || p->nnz == 0) HIP_TRY(p, launch_fill_zero(y, ybytes, s));
            HIP_TRY(p, launch_spmv_coo_row(dt, p->n, p->nnz, p->irow, p->icol, p->val, x, y, plan_carries(p), s));
            return SPMV_OK;
        case SPMV_ELL_ROW:
            if (variant != 0) return SPMV_E_ARG;
            if (p->ell_w < 0) return SPMV_E_NOT_READY;
            HIP_TRY(p, launch_spmv_ell_row(dt, p->n, p->ell_w, p->ell_val, p->ell_col, x, y, alpha, s));
            return SPMV_OK;
        case SPMV_ELL_COL:
            if (variant < 0 || variant > 2) return SPMV_E_ARG;
            if (p->ellc_w < 0) return SPMV_E_NOT_READY;
            if (col_variant(p, variant) == 2)
                HIP_TRY(p, launch_spmv_ell_col_paged(dt, p->n, p->ellc_w, p->st.bandwidth, p->ellc_val, p->ellc_row,
                                                     x, y, s));
            else
                HIP_TRY(p, launch_spmv_ell_col(dt, p->n, p->ellc_w, p->ellc_val, p->ellc_row, x, y, s));
            return SPMV_OK;
        case SPMV_COO_COL:
            if (variant < 0 || variant > 2) return SPMV_E_ARG;
            if (!p->has_coo_col || !p->has_ccs) return SPMV_E_NOT_READY;
            if (col_variant(p, variant) == 2) {
                HIP_TRY(p, launch_spmv_coo_col_paged(dt, p->n, p->nnz, p->st.bandwidth, p->jcol, p->irow_t, p->val_t,
                                                     x, y, s));
                return SPMV_OK;
            }
            HIP_TRY(p, launch_fill_zero(y, ybytes, s));
            if (p->nnz > 0)
                HIP_TRY(p, launch_spmv_coo_col(dt, p->nnz, p->jcol, p->irow_t, p->val_t, x, y, s));
            return SPMV_OK;
        case SPMV_CCS:
            return SPMV_E_ARG;   // CCS is an intermediate form; SpMV uses COO_COL or ELL_COL
        default:
            return SPMV_E_ARG;
    }
}

SPMV_API spmv_status spmv_exec(const spmv_plan* p, spmv_format f, int variant, const void* x, void* y,
                               void* stream) {
    return plan_exec(p, f, variant, x, y, 1.0, static_cast<hipStream_t>(stream));
}

SPMV_API spmv_status spmv_exec_coo_row_noalloc(int32_t n, int64_t nnz, const int32_t* irow, const int32_t* icol,
                                               const void* val, spmv_dtype val_type, const void* x, void* y,
                                               void* stream) {
    if (n < 1 || nnz < 0 || !valid_dtype(val_type)) return SPMV_E_ARG;
    if (nnz > SPMV_COO_ROW_NOALLOC_MAX_NNZ) return SPMV_E_TOO_LARGE;
    if (!x || !y || !aligned16(x) || !aligned16(y)) return SPMV_E_ARG;
    if (nnz > 0 && (!irow || !icol || !val || !aligned16(irow) || !aligned16(icol) || !aligned16(val)))
        return SPMV_E_ARG;
    const hipError_t e = launch_spmv_coo_row_static((int)val_type, n, nnz, irow, icol, val, x, y,
                                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SPMV_OK : SPMV_E_HIP;
}

// ----------------------------------------------------------- conversion

SPMV_API spmv_status spmv_convert_values(const double* in, void* out, int64_t m, spmv_dtype to, void* stream) {
    if (m < 0 || (to != SPMV_F32 && to != SPMV_BF16 && to != SPMV_F16)) return SPMV_E_ARG;
    if (m == 0) return SPMV_OK;
    if (!in || !out || !aligned16(in) || !aligned16(out)) return SPMV_E_ARG;
    hipError_t e = launch_convert((int)to, m, in, out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SPMV_OK : SPMV_E_HIP;
}

// ----------------------------------------------------------- auto-tuning

SPMV_API spmv_status at_choose_format(const spmv_plan* p, const at_table* t, int64_t k_repeats, spmv_format* fmt,
                                      int* variant, at_decision* why) {
    if (!p) return SPMV_E_ARG;
    return at_choose_format_stats(&p->st, p->dt, p->limit, t, k_repeats, fmt, variant, why);
}
