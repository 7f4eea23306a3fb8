// Column-format SpMV (Fig. 1: the entries of column j add val * x(j) into
// y(row)) with y privatised in LDS page by page, for matrices of limited
// bandwidth: the GPU form of the figures' private copies of Y, restricted
// to the rows a workgroup actually touches.
//
// A workgroup owns 256 consecutive columns (ELL-Column) or 8192 consecutive
// entries (COO-Column).  Every row its entries add into lies in the window
// [first column - bw, last column + bw], bw = max |i - j|.  The window is
// cut into pages of 64 rows.  The workgroup
//   1. marks the pages its entries touch (only the first lane of each run
//      of equal pages in a wave stores the mark),
//   2. numbers the marked pages with a scan: page k gets partial-sum slot k,
//   3. adds each product into its row's LDS partial sum (LDS atomics),
//   4. adds every non-zero partial sum into y with one global atomic.
// On a stencil a workgroup's entries fall into a few narrow bands of rows,
// each row collecting several of them, so the global atomics that bound
// the per-entry kernels drop by that factor.  Entries on pages past the LDS
// capacity, and whole workgroups whose window is too wide, add straight
// into y.  y is cleared first; the order of the additions depends on
// scheduling, as with the per-entry kernels.
#include "common.h"
#include "kernels.h"

namespace spmvat {

namespace {

constexpr int kPgBits = 6;
constexpr int kPgRows = 1 << kPgBits;        // rows per page
constexpr int kPgWindow = 1024;              // pages of a window: 65,536 rows
constexpr int kPgAccBytes = 20480;           // LDS partial sums: 40 binary64 or 80 binary32 pages
constexpr int kEcCache = 32;                 // ELL-Column: widths whose rows stay in registers
constexpr int kCcChunk = 8192;               // COO-Column: entries per workgroup
constexpr int kCcPer = kCcChunk / kBlock;    // 32 per thread
constexpr int kPgPer = kPgWindow / kBlock;   // window pages per thread in the numbering scan
static_assert(kPgWindow % kBlock == 0, "the numbering scan gives each thread whole pages");

template <typename X>
struct PgSmem {
    static constexpr int kCap = kPgAccBytes / (int)sizeof(X) / kPgRows;   // pages that get a partial sum
    X acc[kCap * kPgRows];
    int slot[kPgWindow];        // per window page: 1 when marked, then its slot or -1
    int page_of[kCap];          // window page of each slot
    int wsum[kBlock / kWave];
};

template <typename X>
__device__ __forceinline__ void add_global(X* p, X v) { unsafeAtomicAdd(p, v); }

// Workgroup-scope relaxed add on an LDS address: a ds_add instruction.
template <typename X>
__device__ __forceinline__ void add_lds(X* p, X v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Marks window page pg (< 0: nothing).  Every lane of the wave calls it; a
// lane stores only when the lane below it holds another page.
__device__ __forceinline__ void mark_page(int* slot, int pg) {
    const int lane = threadIdx.x & (kWave - 1);
    const int below = __shfl_up(pg, 1, kWave);
    if (pg >= 0 && (lane == 0 || below != pg))
        __hip_atomic_store(&slot[pg], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Turns the marks of slot[0 .. nwin) into partial-sum slots in page order
// (-1 for unmarked pages and for marked pages past the capacity), fills
// page_of and returns the number of slots used.  Starts and ends with a
// barrier.
template <typename X>
__device__ __forceinline__ int number_pages(PgSmem<X>& sm, int nwin) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    __syncthreads();
    int m[kPgPer];
    int c = 0;
#pragma unroll
    for (int e = 0; e < kPgPer; ++e) {
        const int pg = tid * kPgPer + e;
        m[e] = pg < nwin ? sm.slot[pg] : 0;
        c += m[e];
    }
    int incl = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int u = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += u;
    }
    if (lane == kWave - 1) sm.wsum[w] = incl;
    __syncthreads();
    int s = incl - c, total = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) {
        s += k < w ? sm.wsum[k] : 0;
        total += sm.wsum[k];
    }
#pragma unroll
    for (int e = 0; e < kPgPer; ++e) {
        const int pg = tid * kPgPer + e;
        if (pg >= nwin) continue;
        int v = -1;
        if (m[e]) {
            if (s < PgSmem<X>::kCap) {
                v = s;
                sm.page_of[s] = pg;
            }
            ++s;
        }
        sm.slot[pg] = v;
    }
    __syncthreads();
    return min(total, PgSmem<X>::kCap);
}

template <typename X>
__device__ __forceinline__ void clear_acc(PgSmem<X>& sm, int used) {
    for (int t = threadIdx.x; t < used * kPgRows; t += kBlock) sm.acc[t] = (X)0;
    __syncthreads();
}

// Window page of row r, or -1 when r lies outside the window.
__device__ __forceinline__ int page_in(int r, int lo, int nwin) {
    const int d = r - lo;
    return (r >= 0 && d >= 0 && (d >> kPgBits) < nwin) ? (d >> kPgBits) : -1;
}

// Adds v into row r: its LDS partial sum when its page has a slot, else y.
template <typename X>
__device__ __forceinline__ void add_row(PgSmem<X>& sm, int lo, int nwin, int r, X v, X* y) {
    const int pg = page_in(r, lo, nwin);
    const int s = pg >= 0 ? sm.slot[pg] : -1;
    if (s >= 0) add_lds(&sm.acc[s * kPgRows + ((r - lo) & (kPgRows - 1))], v);
    else add_global(&y[r], v);
}

// One global atomic per row whose partial sum is not zero (a row that got
// no product keeps +0.0, and adding +0.0 would change nothing).  Starts
// with a barrier.
template <typename X>
__device__ __forceinline__ void flush(PgSmem<X>& sm, int used, int lo, X* y) {
    __syncthreads();
    for (int t = threadIdx.x; t < used * kPgRows; t += kBlock) {
        const X a = sm.acc[t];
        if (a != (X)0) add_global(&y[lo + sm.page_of[t >> kPgBits] * kPgRows + (t & (kPgRows - 1))], a);
    }
}

// Rows [lo, hi) of a workgroup's window; lo is aligned to a page.
__device__ __forceinline__ void window(int n, int64_t first, int64_t last, int bw, int& lo, int& nwin) {
    const int64_t a = max((int64_t)0, first - bw) & ~(int64_t)(kPgRows - 1);
    const int64_t b = min((int64_t)n, last + 1 + bw);
    lo = (int)a;
    nwin = (int)((b - a + kPgRows - 1) >> kPgBits);
}

}  // namespace

// ELL-Column: thread t of workgroup b takes column 256 b + t and walks its
// slots.  With kCache the rows of up to kEcCache slots stay in registers
// between the marking and the adding pass; otherwise they are read twice.
template <typename V, typename X, bool kCache>
__global__ void __launch_bounds__(kBlock)
k_spmv_ell_col_pg(int n, int width, int bw, const V* __restrict__ ev, const int* __restrict__ er,
                  const X* __restrict__ x, X* __restrict__ y) {
    __shared__ PgSmem<X> sm;
    const int j0 = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock;
    const int j = j0 + (int)threadIdx.x;
    const bool live = j < n;
    int lo, nwin;
    window(n, j0, min((int64_t)n, (int64_t)j0 + kBlock) - 1, bw, lo, nwin);
    if (nwin > kPgWindow) {
        // window too wide for the page table: one global atomic per entry
        if (!live) return;
        const X xj = x[j];
        size_t off = (size_t)j;
        for (int k = 0; k < width; ++k, off += (size_t)n) {
            const X v = (X)widen(ld_nt(&ev[off]));
            if (v != (X)0) add_global(&y[er[off]], v * xj);
        }
        return;
    }
    for (int pg = threadIdx.x; pg < nwin; pg += kBlock) sm.slot[pg] = 0;
    __syncthreads();
    int rows[kCache ? kEcCache : 1];
    if constexpr (kCache) {
#pragma unroll
        for (int k = 0; k < kEcCache; ++k) {
            rows[k] = -1;
            if (k < width) {
                rows[k] = live ? er[(size_t)k * n + j] : -1;
                mark_page(sm.slot, live ? page_in(rows[k], lo, nwin) : -1);
            }
        }
    } else {
        size_t off = (size_t)j;
        for (int k = 0; k < width; ++k, off += (size_t)n) {
            mark_page(sm.slot, live ? page_in(er[off], lo, nwin) : -1);
        }
    }
    const int used = number_pages(sm, nwin);
    clear_acc(sm, used);
    if (live) {
        const X xj = x[j];
        if constexpr (kCache) {
#pragma unroll
            for (int k = 0; k < kEcCache; ++k) {
                if (k < width) {
                    const X v = (X)widen(ld_nt(&ev[(size_t)k * n + j]));
                    if (v != (X)0) add_row(sm, lo, nwin, rows[k], v * xj, y);
                }
            }
        } else {
            size_t off = (size_t)j;
            for (int k = 0; k < width; ++k, off += (size_t)n) {
                const X v = (X)widen(ld_nt(&ev[off]));
                if (v != (X)0) add_row(sm, lo, nwin, er[off], v * xj, y);
            }
        }
    }
    flush(sm, used, lo, y);
}

// COO-Column: workgroup b takes entries [8192 b, 8192 (b+1)); thread t holds
// entries 256 e + t, e < 32, whose rows stay in registers.
template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_coo_col_pg(int n, int64_t nnz, int bw, const int* __restrict__ jcol, const int* __restrict__ irow_t,
                  const V* __restrict__ val_t, const X* __restrict__ x, X* __restrict__ y) {
    __shared__ PgSmem<X> sm;
    const int64_t t0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kCcChunk;
    const int cnt = (int)min((int64_t)kCcChunk, nnz - t0);
    const int tid = threadIdx.x;
    int lo, nwin;
    window(n, jcol[t0], jcol[t0 + cnt - 1], bw, lo, nwin);
    if (nwin > kPgWindow) {
        // the chunk's columns span too wide a window: one global atomic per entry
        for (int q = tid; q < cnt; q += kBlock)
            add_global(&y[irow_t[t0 + q]], (X)widen(val_t[t0 + q]) * x[jcol[t0 + q]]);
        return;
    }
    for (int pg = tid; pg < nwin; pg += kBlock) sm.slot[pg] = 0;
    __syncthreads();
    int rows[kCcPer];
#pragma unroll
    for (int e = 0; e < kCcPer; ++e) {
        const int q = e * kBlock + tid;
        rows[e] = q < cnt ? irow_t[t0 + q] : -1;
        mark_page(sm.slot, q < cnt ? page_in(rows[e], lo, nwin) : -1);
    }
    const int used = number_pages(sm, nwin);
    clear_acc(sm, used);
#pragma unroll
    for (int e = 0; e < kCcPer; ++e) {
        const int q = e * kBlock + tid;
        if (q < cnt) add_row(sm, lo, nwin, rows[e], (X)widen(ld_nt(&val_t[t0 + q])) * x[jcol[t0 + q]], y);
    }
    flush(sm, used, lo, y);
}

bool col_paged_fits(int n, int bw) {
    // every ELL-Column workgroup's window fits the page table
    (void)n;
    return bw >= 0 && (int64_t)kBlock + 2 * (int64_t)bw + 2 * kPgRows <= (int64_t)kPgWindow * kPgRows;
}

#define COLPG_DISPATCH(dtype, CALL)                                  \
    switch (dtype) {                                                 \
        case 0: { typedef double V; typedef double X; CALL; break; } \
        case 1: { typedef float V; typedef float X; CALL; break; }   \
        case 2: { typedef bf16_t V; typedef float X; CALL; break; }  \
        default: { typedef f16_t V; typedef float X; CALL; break; }  \
    }

hipError_t launch_spmv_ell_col_paged(int dtype, int n, int width, int bw, const void* ev, const int* er,
                                     const void* x, void* y, hipStream_t s) {
    const int xb = dtype == 0 ? 8 : 4;
    hipError_t e = launch_fill_zero(y, (int64_t)n * xb, s);
    if (e != hipSuccess || width == 0) return e;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    if (width <= kEcCache) {
        COLPG_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_ell_col_pg<V, X, true>), grid, dim3(kBlock), 0, s, n,
                                                 width, bw, (const V*)ev, er, (const X*)x, (X*)y));
    } else {
        COLPG_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_ell_col_pg<V, X, false>), grid, dim3(kBlock), 0, s, n,
                                                 width, bw, (const V*)ev, er, (const X*)x, (X*)y));
    }
    return hipGetLastError();
}

hipError_t launch_spmv_coo_col_paged(int dtype, int n, int64_t nnz, int bw, const int* jcol, const int* irow_t,
                                     const void* val_t, const void* x, void* y, hipStream_t s) {
    const int xb = dtype == 0 ? 8 : 4;
    hipError_t e = launch_fill_zero(y, (int64_t)n * xb, s);
    if (e != hipSuccess || nnz == 0) return e;
    const int64_t blocks = (nnz + kCcChunk - 1) / kCcChunk;
    COLPG_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_coo_col_pg<V, X>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                                             n, nnz, bw, jcol, irow_t, (const V*)val_t, (const X*)x, (X*)y));
    return hipGetLastError();
}

#undef COLPG_DISPATCH

}  // namespace spmvat
