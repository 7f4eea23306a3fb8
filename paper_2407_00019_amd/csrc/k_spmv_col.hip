// Column-format SpMV (Fig. 1: the entries of column j add val * x(j) into
// y(row)) with y privatised in LDS page by page, for matrices of limited
// bandwidth: the GPU form of the figures' private copies of Y, restricted
// to the rows a workgroup actually touches.
//
// A workgroup owns 1024 consecutive columns (ELL-Column, 4 adjacent columns
// per thread, vector loads; 256 columns when n is not a multiple of 4) or
// 4096 consecutive entries (COO-Column, 4 consecutive entries per thread and
// step).  Every row its entries add into lies in the window
// [first column - bw, last column + bw], bw = max |i - j|.  The window is
// cut into pages of 64 rows.  The workgroup
//   1. marks the pages its entries touch (only the first lane of each run
//      of equal pages in a row of 16 lanes stores the mark),
//   2. numbers the marked pages with a scan: page k gets partial-sum slot k,
//   3. adds each product into its row's LDS partial sum (LDS atomics),
//   4. adds every non-zero partial sum into y with one global atomic.
// On a stencil a workgroup's entries fall into a few narrow bands of rows,
// each row collecting several of them, so the global atomics that bound
// the per-entry kernels drop by that factor.  Entries on pages past the LDS
// capacity, and whole workgroups whose window is too wide, add straight
// into y.  y is cleared first; the order of the additions depends on
// scheduling, as with the per-entry kernels.
//
// Sizes measured on the 27-point 128^3 stencil (binary64): ELL-Column with
// 1, 2 and 4 columns per thread took 224, 198 and 180 us (4 columns with
// fewer than 64 partial-sum pages spill past the capacity: 240-450 us);
// COO-Column with 8192-, 4096- and 2048-entry chunks of single entries took
// 344, 309 and 334 us, 4096 entries as pairs 256 us and as quads 237 us.
#include "common.h"
#include "kernels.h"

namespace spmvat {

namespace {

constexpr int kPgBits = 6;
constexpr int kPgRows = 1 << kPgBits;        // rows per page
constexpr int kPgWindow = 1024;              // pages of a window: 65,536 rows
constexpr int kPgPer = kPgWindow / kBlock;   // window pages per thread in the numbering scan
static_assert(kPgWindow % kBlock == 0, "the numbering scan gives each thread whole pages");
constexpr int kEcVec = 4;                    // ELL-Column: adjacent columns per thread (n % 4 == 0)
constexpr int kEcAccBytes = 32768;           // its partial sums: 64 binary64 / 128 binary32 pages
constexpr int kEcHeld = 32;                  // ELL-Column widths whose rows stay in registers between the passes
constexpr int kEc1AccBytes = 20480;          // one column per thread: 40 / 80 pages
constexpr int kCcVec = 4;                    // COO-Column: consecutive entries per thread and step
constexpr int kCcChunk = 4096;               // entries per workgroup
constexpr int kCcSteps = kCcChunk / (kCcVec * kBlock);
constexpr int kCcAccBytes = 16384;           // its partial sums: 32 binary64 / 64 binary32 pages
static_assert(kCcChunk % (kCcVec * kBlock) == 0, "a chunk is whole steps");

template <typename X, int kBytes>
struct PgSmem {
    using Acc = X;
    static constexpr int kCap = kBytes / (int)sizeof(X) / kPgRows;   // pages that get a partial sum
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

// Marks window page pg (< 0: nothing).  Every lane of the wave calls it,
// all active.  A lane stores only when the lane below it in its row of 16
// lanes (a DPP row shift, no LDS traffic) holds another page; the first
// lane of each row always stores, so every page held by some lane is
// marked.
__device__ __forceinline__ void mark_page(int* slot, int pg) {
    constexpr int kRowShr1 = 0x111;
    const int below = __builtin_amdgcn_update_dpp(-2, pg, kRowShr1, 0xf, 0xf, false);
    if (pg >= 0 && below != pg)
        __hip_atomic_store(&slot[pg], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Turns the marks of slot[0 .. nwin) into partial-sum slots in page order
// (-1 for unmarked pages and for marked pages past the capacity), fills
// page_of and returns the number of slots used.  Starts and ends with a
// barrier.
template <class S>
__device__ __forceinline__ int number_pages(S& sm, int nwin) {
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
            if (s < S::kCap) {
                v = s;
                sm.page_of[s] = pg;
            }
            ++s;
        }
        sm.slot[pg] = v;
    }
    __syncthreads();
    return min(total, S::kCap);
}

template <class S>
__device__ __forceinline__ void clear_acc(S& sm, int used) {
    for (int t = threadIdx.x; t < used * kPgRows; t += kBlock) sm.acc[t] = (typename S::Acc)0;
    __syncthreads();
}

// Window page of row r, or -1 when r lies outside the window.
__device__ __forceinline__ int page_in(int r, int lo, int nwin) {
    const int d = r - lo;
    return (r >= 0 && d >= 0 && (d >> kPgBits) < nwin) ? (d >> kPgBits) : -1;
}

// Adds v into row r: its LDS partial sum when its page has a slot, else y.
template <class S, typename X>
__device__ __forceinline__ void add_row(S& sm, int lo, int nwin, int r, X v, X* y) {
    const int pg = page_in(r, lo, nwin);
    const int s = pg >= 0 ? sm.slot[pg] : -1;
    if (s >= 0) add_lds(&sm.acc[s * kPgRows + ((r - lo) & (kPgRows - 1))], v);
    else add_global(&y[r], v);
}

// Adds v into the row at offset o of the window (o < nwin * 64).
template <class S, typename X>
__device__ __forceinline__ void add_off(S& sm, int lo, uint32_t o, X v, X* y) {
    const int s = sm.slot[o >> kPgBits];
    if (s >= 0) add_lds(&sm.acc[s * kPgRows + (int)(o & (kPgRows - 1))], v);
    else add_global(&y[lo + (int)o], v);
}

// One global atomic per row whose partial sum is not zero (a row that got
// no product keeps +0.0, and adding +0.0 would change nothing).  Starts
// with a barrier.
template <class S, typename X>
__device__ __forceinline__ void flush(S& sm, int used, int lo, X* y) {
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

// C consecutive indices (C = 1 or 4; p aligned to 4 C bytes).
template <int C>
__device__ __forceinline__ void load_idx(const int* p, int (&r)[C]) {
    if constexpr (C == 4) {
        const int4 v = *reinterpret_cast<const int4*>(p);
        r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
    } else {
        r[0] = p[0];
    }
}

// C consecutive values through non-temporal loads (p aligned to C values).
template <typename V, int C>
__device__ __forceinline__ void load_val(const V* p, V (&v)[C]) {
    if constexpr (C == 4) {
        load2_nt(p, v[0], v[1]);
        load2_nt(p + 2, v[2], v[3]);
    } else {
        v[0] = ld_nt(p);
    }
}

}  // namespace

// ELL-Column: thread t of workgroup b takes the C adjacent columns
// C (256 b + t) .. + C-1 and walks their slots twice: the first pass loads
// the rows and marks their pages, the second loads the values and adds.
// Up to kEcHeld slots the rows stay in registers between the passes, as
// 16-bit offsets into the window (0xffff: outside it, loaded again); wider
// matrices, and windows of the full 65,536 rows, load them again.  C = 4
// needs n % 4 == 0 (every slot's column group aligned).  Padding slots
// (value +0.0) add nothing.
template <typename V, typename X, int C, int kBytes>
__global__ void __launch_bounds__(kBlock)
k_spmv_ell_col_pg(int n, int width, int bw, const V* __restrict__ ev, const int* __restrict__ er,
                  const X* __restrict__ x, X* __restrict__ y) {
    __shared__ PgSmem<X, kBytes> sm;
    const int j0 = (int)xcd_block(blockIdx.x, gridDim.x) * (C * kBlock);
    const int j = j0 + C * (int)threadIdx.x;
    const bool live = j < n;
    int lo, nwin;
    window(n, j0, min((int64_t)n, (int64_t)j0 + C * kBlock) - 1, bw, lo, nwin);
    if (nwin > kPgWindow) {
        // window too wide for the page table: one global atomic per entry
        if (!live) return;
        for (int c = 0; c < C; ++c) {
            const X xj = x[j + c];
            size_t off = (size_t)j + c;
            for (int k = 0; k < width; ++k, off += (size_t)n) {
                const X v = (X)widen(ld_nt(&ev[off]));
                if (v != (X)0) add_global(&y[er[off]], v * xj);
            }
        }
        return;
    }
    for (int pg = threadIdx.x; pg < nwin; pg += kBlock) sm.slot[pg] = 0;
    __syncthreads();
    if (width <= kEcHeld && nwin < kPgWindow) {
        // rows held as 16-bit window offsets, two to a register
        constexpr uint32_t kOut = 0xffffu;   // above every offset of a window under 1024 pages
        uint32_t held[(kEcHeld * C + 1) / 2];
        // a predicate, not a break, so that the loop unrolls and the held
        // offsets keep compile-time register indices
#pragma unroll
        for (int k = 0; k < kEcHeld; ++k) {
            if (k < width) {
                int r[C];
#pragma unroll
                for (int c = 0; c < C; ++c) r[c] = -1;
                if (live) load_idx<C>(&er[(size_t)j + (size_t)k * n], r);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int pg = page_in(r[c], lo, nwin);
                    mark_page(sm.slot, pg);
                    const uint32_t o = pg >= 0 ? (uint32_t)(r[c] - lo) : kOut;
                    const int h = k * C + c;
                    if (h & 1) held[h >> 1] |= o << 16;
                    else held[h >> 1] = o;
                }
            }
        }
        const int used = number_pages(sm, nwin);
        clear_acc(sm, used);
        if (live) {
            X xs[C];
#pragma unroll
            for (int c = 0; c < C; ++c) xs[c] = x[j + c];
#pragma unroll
            for (int k = 0; k < kEcHeld; ++k) {
                if (k < width) {
                    const size_t off = (size_t)j + (size_t)k * n;
                    V v[C];
                    load_val<V, C>(&ev[off], v);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const int h = k * C + c;
                        const uint32_t o = (held[h >> 1] >> (16 * (h & 1))) & 0xffffu;
                        const X w = (X)widen(v[c]);
                        if (w != (X)0) {
                            if (o != kOut) add_off(sm, lo, o, w * xs[c], y);
                            else add_row(sm, lo, nwin, er[off + c], w * xs[c], y);
                        }
                    }
                }
            }
        }
        flush(sm, used, lo, y);
        return;
    }
    size_t off = (size_t)j;
    for (int k = 0; k < width; ++k, off += (size_t)n) {
        int r[C];
#pragma unroll
        for (int c = 0; c < C; ++c) r[c] = -1;
        if (live) load_idx<C>(&er[off], r);
#pragma unroll
        for (int c = 0; c < C; ++c) mark_page(sm.slot, page_in(r[c], lo, nwin));
    }
    const int used = number_pages(sm, nwin);
    clear_acc(sm, used);
    if (live) {
        X xs[C];
#pragma unroll
        for (int c = 0; c < C; ++c) xs[c] = x[j + c];
        off = (size_t)j;
        for (int k = 0; k < width; ++k, off += (size_t)n) {
            int r[C];
            V v[C];
            load_idx<C>(&er[off], r);
            load_val<V, C>(&ev[off], v);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const X w = (X)widen(v[c]);
                if (w != (X)0) add_row(sm, lo, nwin, r[c], w * xs[c], y);
            }
        }
    }
    flush(sm, used, lo, y);
}

// COO-Column: workgroup b takes entries [4096 b, 4096 (b+1)); at step e
// thread t holds the 4 consecutive entries 4 (256 e + t) .. + 3, loaded as
// vectors, and keeps their rows in registers between the passes.
template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_coo_col_pg(int n, int64_t nnz, int bw, const int* __restrict__ jcol, const int* __restrict__ irow_t,
                  const V* __restrict__ val_t, const X* __restrict__ x, X* __restrict__ y) {
    constexpr int C = kCcVec;
    __shared__ PgSmem<X, kCcAccBytes> sm;
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
    int rows[kCcSteps][C];
#pragma unroll
    for (int e = 0; e < kCcSteps; ++e) {
        const int q = C * (e * kBlock + tid);
#pragma unroll
        for (int c = 0; c < C; ++c) rows[e][c] = -1;
        if (q + C <= cnt) {
            load_idx<C>(&irow_t[t0 + q], rows[e]);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (q + c < cnt) rows[e][c] = irow_t[t0 + q + c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) mark_page(sm.slot, page_in(rows[e][c], lo, nwin));
    }
    const int used = number_pages(sm, nwin);
    clear_acc(sm, used);
#pragma unroll
    for (int e = 0; e < kCcSteps; ++e) {
        const int q = C * (e * kBlock + tid);
        if (q + C <= cnt) {
            V v[C];
            int col[C];
            load_val<V, C>(&val_t[t0 + q], v);
            load_idx<C>(&jcol[t0 + q], col);
#pragma unroll
            for (int c = 0; c < C; ++c) add_row(sm, lo, nwin, rows[e][c], (X)widen(v[c]) * x[col[c]], y);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (q + c < cnt)
                    add_row(sm, lo, nwin, rows[e][c], (X)widen(val_t[t0 + q + c]) * x[jcol[t0 + q + c]], y);
        }
    }
    flush(sm, used, lo, y);
}

bool col_paged_fits(int n, int bw) {
    // every ELL-Column workgroup's window fits the page table
    const int cols = (n % kEcVec == 0 ? kEcVec : 1) * kBlock;
    return bw >= 0 && (int64_t)cols + 2 * (int64_t)bw + 2 * kPgRows <= (int64_t)kPgWindow * kPgRows;
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
    if (n % kEcVec == 0) {
        const dim3 grid((unsigned)(n / (kEcVec * kBlock) + (n % (kEcVec * kBlock) != 0)));
        COLPG_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_ell_col_pg<V, X, kEcVec, kEcAccBytes>), grid, dim3(kBlock),
                                                 0, s, n, width, bw, (const V*)ev, er, (const X*)x, (X*)y));
    } else {
        const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
        COLPG_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_ell_col_pg<V, X, 1, kEc1AccBytes>), grid, dim3(kBlock), 0, s,
                                                 n, width, bw, (const V*)ev, er, (const X*)x, (X*)y));
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
