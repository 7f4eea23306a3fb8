// Run-time transformations of section 2.1 on gfx950.
//
//  * expand_ptr   COO-Row IROW from the row pointer, and COO-Column's column
//                 index from the CCS column pointer (Phase II).
//  * CRS -> CCS   Phase I: column counts (global atomics), exclusive scan
//                 into column pointers, scatter of packed (position, row)
//                 keys through per-column atomic cursors, then a per-column
//                 sort of the keys by CRS position.  The sort turns the
//                 scheduling-dependent scatter order into the paper's stable
//                 order (by row, then by position within the row), so every
//                 output array is deterministic and bit-exact.
//  * ELL pack     slot-major VAL(n, width) / index arrays with zero padding.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace spmvat {

typedef unsigned long long u64;

// ------------------------------------------------------------ helpers

// Exclusive scan of one int per thread over a 256-thread workgroup.
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int& total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) sh[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) {
        int t = sh[k];
        pre += (k < w) ? t : 0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Loads ptr[r0 .. r0+rows] of one 256-line tile into LDS.
__device__ __forceinline__ void load_ptr_tile(const int* __restrict__ ptr, int r0, int rows, int* sp) {
    for (int t = threadIdx.x; t <= rows; t += kBlock) sp[t] = ptr[r0 + t];
    __syncthreads();
}

// -------------------------------------------------------- ptr expansion
// Workgroup = 256 consecutive lines.  Each lane writes its own line index
// over its positions into an LDS image of the tile's slice of the output,
// which is then stored with coalesced writes.

constexpr int kExpandCap = 8192;

__global__ void __launch_bounds__(kBlock)
k_expand_ptr(int n, const int* __restrict__ ptr, int* __restrict__ out) {
    __shared__ int sp[kBlock + 1];
    __shared__ int so[kExpandCap];
    const int r0 = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock;
    const int rows = min(kBlock, n - r0);
    const int t = threadIdx.x;
    load_ptr_tile(ptr, r0, rows, sp);
    const int end = sp[rows];
    const int a = t < rows ? sp[t] : end, b = t < rows ? sp[t + 1] : end;
    for (int c0 = sp[0]; c0 < end; c0 += kExpandCap) {
        const int cl = min(kExpandCap, end - c0);
        const int lo = max(a, c0), hi = min(b, c0 + cl);
        for (int p = lo; p < hi; ++p) so[p - c0] = r0 + t;
        __syncthreads();
        for (int q = t; q < cl; q += kBlock) out[c0 + q] = so[q];
        __syncthreads();
    }
}

hipError_t launch_expand_ptr(int n, const int* ptr, int* out, hipStream_t s) {
    unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_expand_ptr, dim3(blocks), dim3(kBlock), 0, s, n, ptr, out);
    return hipGetLastError();
}

// ------------------------------------------------ Phase I: column counts
// and the scatter.  Matrices of small bandwidth use the LDS-privatised
// kernels below (a tile's columns all fall in a window that fits in LDS).
// Otherwise both walk a tile of 256 rows with one row per lane: the tile's
// column indices (contiguous in CRS) are staged in LDS with coalesced loads,
// then every lane steps through its own row.  For banded and stencil
// matrices the lanes of a wave then touch consecutive columns at each step,
// so a wave's atomics coalesce into a few cache lines.

constexpr int kRowTileCap = 8192;   // column indices staged per pass

template <bool kScatter>
__global__ void __launch_bounds__(kBlock)
k_col_walk(int n, const int* __restrict__ irp, const int* __restrict__ icol, int* __restrict__ counter,
           u64* __restrict__ keys) {
    __shared__ int sp[kBlock + 1];
    __shared__ int sc[kRowTileCap];
    const int r0 = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock;
    const int rows = min(kBlock, n - r0);
    const int t = threadIdx.x;
    for (int c = t; c <= rows; c += kBlock) sp[c] = irp[r0 + c];
    __syncthreads();
    const int end = sp[rows];
    const int a = t < rows ? sp[t] : end, b = t < rows ? sp[t + 1] : end;
    for (int c0 = sp[0]; c0 < end; c0 += kRowTileCap) {
        const int cl = min(kRowTileCap, end - c0);
        for (int q = t; q < cl; q += kBlock) sc[q] = icol[c0 + q];
        __syncthreads();
        const int lo = max(a, c0), hi = min(b, c0 + cl);
        for (int p = lo; p < hi; ++p) {
            const int c = sc[p - c0];
            if (kScatter) {
                const int slot = atomicAdd(&counter[c], 1);
                keys[slot] = ((u64)(uint32_t)p << 32) | (uint32_t)(r0 + t);
            } else {
                atomicAdd(&counter[c], 1);
            }
        }
        __syncthreads();
    }
}

// Column counts with LDS privatisation, for matrices of small bandwidth bw
// (max |i - j|): every column of rows [r0, r0 + R) lies in
// [r0 - bw, r0 + R - 1 + bw], so a workgroup counts its rows' entries into
// that window of bins in LDS (contiguous, coalesced reads of icol; LDS
// atomics) and adds each non-zero bin to the global count with one atomic.
// On the 27-point stencil a bin collects the 1-3 entries of one x-line, so
// the global atomics drop threefold.  A column outside the window (only if
// the CRS arrays changed after the plan was made) goes straight to the
// global count.
constexpr int kPrivBins = 36864;            // 144 KiB of LDS: one workgroup per CU
constexpr int kPrivThreads = 1024;          // 16 waves hide the reads' latency
constexpr int kPrivMinRows = 1024;          // below this many rows per window, use the walk

__global__ void __launch_bounds__(kPrivThreads)
k_col_count_priv(int n, int bw, int rows_per_tile, const int* __restrict__ irp, const int* __restrict__ icol,
                 int* __restrict__ counter) {
    __shared__ int bins[kPrivBins];
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int r0 = tile * rows_per_tile;
    const int r1 = min(n, r0 + rows_per_tile);
    const int lo = max(0, r0 - bw);
    const int hi = (int)min((int64_t)n, (int64_t)r1 + bw);
    const int width = hi - lo;                  // <= rows_per_tile + 2 bw <= kPrivBins (host check)
    for (int c = threadIdx.x; c < width; c += kPrivThreads) bins[c] = 0;
    __syncthreads();
    const int e0 = irp[r0], e1 = irp[r1];
    constexpr int kUnroll = 4;
    for (int base = e0; base < e1; base += kPrivThreads * kUnroll) {
        // clamped, unconditional loads (base < e1): all in flight together
        int c[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) c[u] = icol[min(base + u * kPrivThreads + (int)threadIdx.x, e1 - 1)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (base + u * kPrivThreads + (int)threadIdx.x >= e1) continue;
            const unsigned off = (unsigned)(c[u] - lo);
            if (off < (unsigned)width) atomicAdd(&bins[off], 1);
            else atomicAdd(&counter[c[u]], 1);
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < width; c += kPrivThreads) {
        const int v = bins[c];
        if (v) atomicAdd(&counter[lo + c], v);
    }
}

hipError_t launch_col_count(int n, int bw, const int* irp, const int* icol, int* cnt, hipStream_t s) {
    // privatised counts when a window of at least kPrivMinRows rows fits
    int rows = 0;
    if (bw >= 0 && (int64_t)2 * bw + kPrivMinRows <= kPrivBins) {
        rows = std::min(8192, (int)((kPrivBins - 2 * (int64_t)bw) / kBlock * kBlock));
        rows = std::min(rows, ((n + kBlock - 1) / kBlock) * kBlock);
    }
    if (rows >= kPrivMinRows || (rows > 0 && rows >= n)) {
        const unsigned tiles = (unsigned)((n + rows - 1) / rows);
        hipLaunchKernelGGL(k_col_count_priv, dim3(tiles), dim3(kPrivThreads), 0, s, n, bw, rows, irp, icol, cnt);
        return hipGetLastError();
    }
    unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_col_walk<false>, dim3(blocks), dim3(kBlock), 0, s, n, irp, icol, cnt, nullptr);
    return hipGetLastError();
}

// ------------------------------------- Phase I: exclusive scan of counts
// Reduce-then-scan over tiles of 4096 counts: (A) tile sums, longest
// column, and lists of the columns too long for the one-thread sort;
// (B) one workgroup scans the tile sums; (C) each tile rescans with its
// offset and writes ccp and the scatter cursors.

constexpr int kScanPer = kScanTile / kBlock;   // 16 counts per thread

__global__ void __launch_bounds__(kBlock)
k_scan_reduce(int n, const int* __restrict__ cnt, int* __restrict__ bsum, int* __restrict__ bmax,
              int* __restrict__ mid_list, int* __restrict__ long_list, ColSummary* __restrict__ sum) {
    __shared__ int sh[kBlock / kWave];
    __shared__ int shm[kBlock / kWave];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int s = 0, mx = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        const int j = base + e;
        if (j < n) {
            const int c = cnt[j];
            s += c;
            mx = max(mx, c);
            if (c > kSortSmall && mid_list) {   // lists only for the per-column sort
                if (c <= kSortMid) mid_list[atomicAdd(&sum->n_mid, 1)] = j;
                else long_list[atomicAdd(&sum->n_long, 1)] = j;
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) shm[threadIdx.x / kWave] = mx;
    int total;
    block_excl_scan(s, sh, total);   // its barriers also publish shm
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = total;
        int m = shm[0];
        for (int w = 1; w < kBlock / kWave; ++w) m = max(m, shm[w]);
        bmax[blockIdx.x] = m;
    }
}

__global__ void __launch_bounds__(kBlock)
k_scan_top(int nb, int n, int* __restrict__ bsum, const int* __restrict__ bmax, int* __restrict__ ccp,
           ColSummary* __restrict__ sum) {
    __shared__ int sh[kBlock / kWave];
    __shared__ int shm[kBlock / kWave];
    int carry = 0, mx = 0;
    for (int base = 0; base < nb; base += kBlock) {
        const int j = base + threadIdx.x;
        const int v = j < nb ? bsum[j] : 0;
        if (j < nb) mx = max(mx, bmax[j]);
        int total;
        const int ex = block_excl_scan(v, sh, total);
        if (j < nb) bsum[j] = carry + ex;
        carry += total;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) shm[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = shm[0];
        for (int w = 1; w < kBlock / kWave; ++w) m = max(m, shm[w]);
        sum->total = carry;
        sum->max_len = m;
        ccp[n] = carry;
    }
}

__global__ void __launch_bounds__(kBlock)
k_scan_apply(int n, const int* cnt, const int* __restrict__ bsum, int* __restrict__ ccp, int* cursor) {
    // cnt and cursor are one array: every count is read before the same
    // thread overwrites it with its cursor (no restrict on either)
    __shared__ int sh[kBlock / kWave];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int c[kScanPer];
    int s = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        c[e] = (base + e < n) ? cnt[base + e] : 0;
        s += c[e];
    }
    int total;
    int run = bsum[blockIdx.x] + block_excl_scan(s, sh, total);
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        if (base + e < n) {
            ccp[base + e] = run;
            cursor[base + e] = run;
        }
        run += c[e];
    }
}

size_t col_scan_bsum_count(int n) { return (size_t)((n + kScanTile - 1) / kScanTile); }

// (start, end) of each listed column, for one copy to the host.
__global__ void __launch_bounds__(kBlock)
k_col_extents(int count, const int* __restrict__ list, const int* __restrict__ ccp, int* __restrict__ ext) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    const int j = list[i];
    ext[2 * i] = ccp[j];
    ext[2 * i + 1] = ccp[j + 1];
}

hipError_t launch_col_extents(int count, const int* list, const int* ccp, int* ext, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_col_extents, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, count,
                       list, ccp, ext);
    return hipGetLastError();
}

hipError_t launch_col_scan(int n, const int* cnt, int* ccp, int* cursor, int* bsum, int* mid_list,
                           int* long_list, ColSummary* sum, hipStream_t s) {
    const int nb = (int)col_scan_bsum_count(n);
    int* bmax = bsum + nb;
    hipError_t e = hipMemsetAsync(sum, 0, sizeof(ColSummary), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, n, cnt, bsum, bmax, mid_list, long_list, sum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, nb, n, bsum, bmax, ccp, sum);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0, s, n, cnt, bsum, ccp, cursor);
    return hipGetLastError();
}

// ------------------------------------------------- Phase I: the scatter
// Each CRS entry (position q, row r, column c) claims a slot of column c
// through its cursor and stores the key (q << 32 | r) there.  Slot order
// inside a column depends on scheduling; the sort below fixes it.

// The scatter with LDS privatisation (same window as the counts): a
// workgroup counts its rows' entries per window column in LDS, reserves one
// contiguous range of slots per touched column with a single global atomic,
// then hands out slots inside those ranges with LDS atomics.  The row of an
// entry comes from a binary search over the tile's row pointers in LDS.
constexpr int kScatRows = 4096;                       // rows per tile at most
constexpr int kScatBins = 40960 - (kScatRows + 1) - 63;   // just under the 160 KiB of LDS a workgroup may hold

__global__ void __launch_bounds__(kPrivThreads)
k_ccs_scatter_priv(int n, int bw, int rows_per_tile, const int* __restrict__ irp, const int* __restrict__ icol,
                   int* __restrict__ cursor, u64* __restrict__ keys) {
    __shared__ int bins[kScatBins];
    __shared__ int sp[kScatRows + 1];
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int r0 = tile * rows_per_tile;
    const int rows = min(n, r0 + rows_per_tile) - r0;
    const int lo = max(0, r0 - bw);
    const int hi = (int)min((int64_t)n, (int64_t)r0 + rows + bw);
    const int width = hi - lo;                  // <= rows_per_tile + 2 bw <= kScatBins (host check)
    for (int c = threadIdx.x; c < width; c += kPrivThreads) bins[c] = 0;
    for (int i = threadIdx.x; i <= rows; i += kPrivThreads) sp[i] = irp[r0 + i];
    __syncthreads();
    const int e0 = sp[0], e1 = sp[rows];
    constexpr int kUnroll = 4;
    // (1) entries per window column
    for (int base = e0; base < e1; base += kPrivThreads * kUnroll) {
        int c[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) c[u] = icol[min(base + u * kPrivThreads + (int)threadIdx.x, e1 - 1)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (base + u * kPrivThreads + (int)threadIdx.x >= e1) continue;
            const unsigned off = (unsigned)(c[u] - lo);
            if (off < (unsigned)width) atomicAdd(&bins[off], 1);
        }
    }
    __syncthreads();
    // (2) one reservation per touched column; the bin becomes its cursor
    for (int c = threadIdx.x; c < width; c += kPrivThreads) {
        const int v = bins[c];
        if (v) bins[c] = atomicAdd(&cursor[lo + c], v);
    }
    __syncthreads();
    // (3) slots inside the reserved ranges
    for (int base = e0; base < e1; base += kPrivThreads * kUnroll) {
        int c[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) c[u] = icol[min(base + u * kPrivThreads + (int)threadIdx.x, e1 - 1)];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int p = base + u * kPrivThreads + (int)threadIdx.x;
            if (p >= e1) continue;
            const int row = r0 + last_le(sp, 0, rows - 1, p);
            const unsigned off = (unsigned)(c[u] - lo);
            const int slot = off < (unsigned)width ? atomicAdd(&bins[off], 1) : atomicAdd(&cursor[c[u]], 1);
            keys[slot] = ((u64)(uint32_t)p << 32) | (uint32_t)row;
        }
    }
}

bool ccs_privatised(int bw) { return bw >= 0 && (int64_t)2 * bw + kPrivMinRows <= kScatBins; }

hipError_t launch_ccs_scatter(int n, int bw, const int* irp, const int* icol, int* cursor, u64* keys,
                              hipStream_t s) {
    int rows = 0;
    if (bw >= 0 && (int64_t)2 * bw + kPrivMinRows <= kScatBins) {
        rows = std::min(kScatRows, (int)((kScatBins - 2 * (int64_t)bw) / kBlock * kBlock));
        rows = std::min(rows, ((n + kBlock - 1) / kBlock) * kBlock);
    }
    if (rows >= kPrivMinRows || (rows > 0 && rows >= n)) {
        const unsigned tiles = (unsigned)((n + rows - 1) / rows);
        hipLaunchKernelGGL(k_ccs_scatter_priv, dim3(tiles), dim3(kPrivThreads), 0, s, n, bw, rows, irp, icol, cursor,
                           keys);
        return hipGetLastError();
    }
    unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_col_walk<true>, dim3(blocks), dim3(kBlock), 0, s, n, irp, icol, cursor, keys);
    return hipGetLastError();
}

// --------------------------------------- Phase I: per-column key sort
// Keys are unique (one per CRS position), so sorting them by value gives
// the one stable order.  Columns of up to kSortSmall entries: ranked by a
// workgroup in LDS (below).  Up to kSortMid: one workgroup per column,
// bitonic sort in LDS.  Longer: chunks sorted in
// LDS, then merge passes in global memory.  Every path ends by emitting
// irow_t[q] = row and val_t[q] = val[position] for its column.

template <typename R>
__device__ __forceinline__ void emit(int q, u64 key, const R* __restrict__ val, int* __restrict__ irow_t,
                                     R* __restrict__ val_t) {
    irow_t[q] = (int)(uint32_t)key;
    val_t[q] = val[key >> 32];
}

// Columns of up to kSortSmall entries: a workgroup takes 256 consecutive
// columns, stages the keys of as many whole columns as fit (kRankCap) in LDS,
// and gives each key its rank among the keys of its column (a linear count;
// lanes of one column read the same LDS words, which broadcast).  The rank is
// the key's final offset in its column, so it is emitted straight away.
constexpr int kRankCap = 3072;

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_sort_rank(int n, const int* __restrict__ ccp, const u64* __restrict__ keys, const R* __restrict__ val,
            int* __restrict__ irow_t, R* __restrict__ val_t) {
    __shared__ int sp[kBlock + 1];
    __shared__ unsigned long long s_long[kBlock / kWave];
    __shared__ u64 sk[kRankCap];
    __shared__ uint8_t sc[kRankCap];     // column of each staged key, relative to j0
    const int j0 = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock;
    const int cols = min(kBlock, n - j0);
    const int t = threadIdx.x;
    for (int c = t; c <= cols; c += kBlock) sp[c] = ccp[j0 + c];
    __syncthreads();
    // columns left to the workgroup and multi-pass sorts, as a 256-bit mask
    const bool lng = t < cols && (sp[t + 1] - sp[t]) > kSortSmall;
    const unsigned long long m = __ballot(lng);
    if ((t & (kWave - 1)) == 0) s_long[t / kWave] = m;
    __syncthreads();

    int c0 = 0;
    while (c0 < cols) {
        // first long column at or after c0 (cols if none)
        int fl = cols;
        for (int w = c0 / kWave; w < kBlock / kWave; ++w) {
            unsigned long long word = s_long[w];
            if (w == c0 / kWave) word &= ~0ull << (c0 % kWave);
            if (word) { fl = min(cols, w * kWave + __ffsll((long long)word) - 1); break; }
        }
        if (fl == c0) { ++c0; continue; }
        // largest c1 in (c0, fl] whose keys fit in LDS; one short column always fits
        int lo = c0 + 1, hi = fl;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sp[mid] - sp[c0] <= kRankCap) lo = mid; else hi = mid - 1;
        }
        const int c1 = lo;
        const int base = sp[c0], span = sp[c1] - base;
        for (int q = t; q < span; q += kBlock) sk[q] = keys[base + q];
        if (t >= c0 && t < c1)
            for (int q = sp[t] - base; q < sp[t + 1] - base; ++q) sc[q] = (uint8_t)t;
        __syncthreads();
        for (int q = t; q < span; q += kBlock) {
            const u64 key = sk[q];
            const int c = sc[q];
            const int s = sp[c] - base, e = sp[c + 1] - base;
            int rank = 0, k2 = s;
            for (; k2 + 4 <= e; k2 += 4)
                rank += (int)(sk[k2] < key) + (int)(sk[k2 + 1] < key) + (int)(sk[k2 + 2] < key) +
                        (int)(sk[k2 + 3] < key);
            for (; k2 < e; ++k2) rank += (int)(sk[k2] < key);
            emit<R>(sp[c] + rank, key, val, irow_t, val_t);
        }
        __syncthreads();
        c0 = c1;
    }
}

// Bitonic sort of up to kSortMid keys in LDS (pad with all-ones).
__device__ void lds_bitonic(u64* sh, int len, int cap) {
    int p = 1;
    while (p < len) p <<= 1;
    for (int i = len + threadIdx.x; i < p; i += kBlock) sh[i] = ~0ull;
    __syncthreads();
    for (int k = 2; k <= p; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < p; i += kBlock) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const u64 a = sh[i], b = sh[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) { sh[i] = b; sh[ixj] = a; }
                }
            }
            __syncthreads();
        }
    }
    (void)cap;
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_sort_mid(const int* __restrict__ list, const int* __restrict__ ccp, u64* __restrict__ keys,
           const R* __restrict__ val, int* __restrict__ irow_t, R* __restrict__ val_t) {
    __shared__ u64 sh[kSortMid];
    const int j = list[blockIdx.x];
    const int s = ccp[j], len = ccp[j + 1] - s;
    for (int i = threadIdx.x; i < len; i += kBlock) sh[i] = keys[s + i];
    lds_bitonic(sh, len, kSortMid);
    for (int i = threadIdx.x; i < len; i += kBlock) emit<R>(s + i, sh[i], val, irow_t, val_t);
}

// Long columns: sort chunks of kSortMid keys in place.
__global__ void __launch_bounds__(kBlock)
k_sort_chunks(int start, int len, u64* __restrict__ keys) {
    __shared__ u64 sh[kSortMid];
    const int c0 = blockIdx.x * kSortMid;
    const int cl = min(kSortMid, len - c0);
    u64* src = keys + start + c0;
    for (int i = threadIdx.x; i < cl; i += kBlock) sh[i] = src[i];
    lds_bitonic(sh, cl, kSortMid);
    for (int i = threadIdx.x; i < cl; i += kBlock) src[i] = sh[i];
}

// Number of keys in [lo, hi) of a sorted run that are < key.
__device__ __forceinline__ int count_less(const u64* a, int lo, int hi, u64 key) {
    int l = lo, h = hi;
    while (l < h) {
        const int m = (l + h) >> 1;
        if (a[m] < key) l = m + 1; else h = m;
    }
    return l - lo;
}

// One merge pass: sorted runs of width w pair up into runs of 2w.  Each key
// lands at its index in its run plus its rank in the partner run.
__global__ void __launch_bounds__(kBlock)
k_merge_pass(int len, int w, const u64* __restrict__ src, u64* __restrict__ dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len) return;
    const u64 key = src[i];
    const int g = (int)(((int64_t)i / (2 * (int64_t)w)) * 2 * w);
    const int mid = (int)min((int64_t)g + w, (int64_t)len);
    const int end = (int)min((int64_t)g + 2 * (int64_t)w, (int64_t)len);
    int out;
    if (i < mid) out = i + count_less(src, mid, end, key);
    else out = g + (i - mid) + count_less(src, g, mid, key);
    dst[out] = key;
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_emit_range(int start, int len, const u64* __restrict__ sorted, const R* __restrict__ val,
             int* __restrict__ irow_t, R* __restrict__ val_t) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < len) emit<R>(start + i, sorted[i], val, irow_t, val_t);
}

// Columns longer than the merge scratch: each key's final index is its index
// in its (sorted) chunk plus the number of smaller keys in every other chunk.
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_rank_emit(int start, int len, const u64* __restrict__ keys, const R* __restrict__ val, int* __restrict__ irow_t,
            R* __restrict__ val_t) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len) return;
    const u64* a = keys + start;
    const u64 key = a[i];
    const int mine = i / kSortMid;
    int rank = i - mine * kSortMid;
    const int chunks = (len + kSortMid - 1) / kSortMid;
    for (int c = 0; c < chunks; ++c) {
        if (c == mine) continue;
        rank += count_less(a, c * kSortMid, min(len, (c + 1) * kSortMid), key);
    }
    emit<R>(start + rank, key, val, irow_t, val_t);
}

template <typename R>
static hipError_t rank_emit_t(int start, int len, const u64* keys, const void* val, int* irow_t, void* val_t,
                              hipStream_t s) {
    unsigned blocks = (unsigned)((len + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_rank_emit<R>, dim3(blocks), dim3(kBlock), 0, s, start, len, keys, (const R*)val, irow_t,
                       (R*)val_t);
    return hipGetLastError();
}

template <typename R>
static hipError_t sort_small_t(int n, const int* ccp, u64* keys, const void* val, int* irow_t, void* val_t,
                               hipStream_t s) {
    unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_sort_rank<R>, dim3(blocks), dim3(kBlock), 0, s, n, ccp, keys,
                       (const R*)val, irow_t, (R*)val_t);
    return hipGetLastError();
}

hipError_t launch_ccs_sort_small(int n, const int* ccp, u64* keys, const void* val, int vbytes,
                                 int* irow_t, void* val_t, hipStream_t s) {
    switch (vbytes) {
        case 8: return sort_small_t<uint64_t>(n, ccp, keys, val, irow_t, val_t, s);
        case 4: return sort_small_t<uint32_t>(n, ccp, keys, val, irow_t, val_t, s);
        default: return sort_small_t<uint16_t>(n, ccp, keys, val, irow_t, val_t, s);
    }
}

template <typename R>
static hipError_t sort_mid_t(int count, const int* list, const int* ccp, u64* keys, const void* val,
                             int* irow_t, void* val_t, hipStream_t s) {
    hipLaunchKernelGGL(k_sort_mid<R>, dim3(count), dim3(kBlock), 0, s, list, ccp, keys, (const R*)val,
                       irow_t, (R*)val_t);
    return hipGetLastError();
}

hipError_t launch_ccs_sort_mid(int count, const int* list, const int* ccp, u64* keys, const void* val,
                               int vbytes, int* irow_t, void* val_t, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (vbytes) {
        case 8: return sort_mid_t<uint64_t>(count, list, ccp, keys, val, irow_t, val_t, s);
        case 4: return sort_mid_t<uint32_t>(count, list, ccp, keys, val, irow_t, val_t, s);
        default: return sort_mid_t<uint16_t>(count, list, ccp, keys, val, irow_t, val_t, s);
    }
}

template <typename R>
static hipError_t emit_t(int start, int len, const u64* sorted, const void* val, int* irow_t,
                         void* val_t, hipStream_t s) {
    unsigned blocks = (unsigned)((len + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_emit_range<R>, dim3(blocks), dim3(kBlock), 0, s, start, len, sorted,
                       (const R*)val, irow_t, (R*)val_t);
    return hipGetLastError();
}

hipError_t launch_ccs_sort_long(int start, int len, u64* keys, u64* tmp, const void* val, int vbytes,
                                int* irow_t, void* val_t, hipStream_t s) {
    const unsigned chunks = (unsigned)((len + kSortMid - 1) / kSortMid);
    hipLaunchKernelGGL(k_sort_chunks, dim3(chunks), dim3(kBlock), 0, s, start, len, keys);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tmp == nullptr) {
        switch (vbytes) {
            case 8: return rank_emit_t<uint64_t>(start, len, keys, val, irow_t, val_t, s);
            case 4: return rank_emit_t<uint32_t>(start, len, keys, val, irow_t, val_t, s);
            default: return rank_emit_t<uint16_t>(start, len, keys, val, irow_t, val_t, s);
        }
    }
    u64* src = keys + start;
    u64* dst = tmp;
    const unsigned blocks = (unsigned)((len + kBlock - 1) / kBlock);
    for (int64_t w = kSortMid; w < len; w *= 2) {
        hipLaunchKernelGGL(k_merge_pass, dim3(blocks), dim3(kBlock), 0, s, len, (int)w, src, dst);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        u64* t = src; src = dst; dst = t;
    }
    switch (vbytes) {
        case 8: return emit_t<uint64_t>(start, len, src, val, irow_t, val_t, s);
        case 4: return emit_t<uint32_t>(start, len, src, val, irow_t, val_t, s);
        default: return emit_t<uint16_t>(start, len, src, val, irow_t, val_t, s);
    }
}

// ------------------------------------------------------------- ELL pack
// Workgroup tile = 64 consecutive lines x 32 slots.  The tile's stored
// entries are read contiguously (a line's entries are consecutive, and so
// are consecutive lines'), each finding its line in a table of line numbers
// the lines first write into LDS, transposed through LDS, and written one
// slot plane at a time: 64 consecutive lines of slot k are 64 consecutive
// elements of the slot-major arrays.  Padding: value bits 0 (+0.0), index =
// line.

constexpr int kEllRows = 64;
constexpr int kEllSlots = 32;
constexpr int kEllPitch = kEllRows + 1;   // pads LDS rows against bank conflicts

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_ell_pack(int n, int width, const int* __restrict__ ptr, const int* __restrict__ idx, const R* __restrict__ val,
           R* __restrict__ ev, int* __restrict__ ei) {
    __shared__ R tv[kEllSlots * kEllPitch];
    __shared__ int ti[kEllSlots * kEllPitch];
    __shared__ int pre[kEllRows + 1];
    __shared__ int sa[kEllRows];
    __shared__ int scnt[kEllRows];
    __shared__ unsigned char line_of[kEllRows * kEllSlots];
    const int t = threadIdx.x;
    const int i0 = (int)xcd_block(blockIdx.x, gridDim.x) * kEllRows;
    const int rows = min(kEllRows, n - i0);
    const int k0 = blockIdx.y * kEllSlots;
    const int kw = min(kEllSlots, width - k0);
    if (t < kEllRows) {
        int cnt = 0;
        if (t < rows) {
            const int a = ptr[i0 + t];
            cnt = min(max(ptr[i0 + t + 1] - a - k0, 0), kw);
            sa[t] = a + k0;
        }
        scnt[t] = cnt;
        // exclusive scan of the counts over the first wave
        int x = cnt;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int y = __shfl_up(x, off, kWave);
            if (t >= off) x += y;
        }
        pre[t] = x - cnt;
        if (t == kEllRows - 1) pre[kEllRows] = x;
    }
    __syncthreads();
    const int total = pre[kEllRows];
    // each line marks its entries' positions with its number, so that every
    // entry finds its line with one LDS read
    if (t < rows)
        for (int k = 0; k < scnt[t]; ++k) line_of[pre[t] + k] = (unsigned char)t;
    __syncthreads();
#pragma unroll 8
    for (int f = t; f < total; f += kBlock) {
        const int r = line_of[f];
        const int k = f - pre[r];
        tv[k * kEllPitch + r] = val[sa[r] + k];
        ti[k * kEllPitch + r] = idx[sa[r] + k];
    }
    __syncthreads();
    const int r = t & (kEllRows - 1);
    if (r < rows) {
        for (int k = t / kEllRows; k < kw; k += kBlock / kEllRows) {
            const size_t off = (size_t)(k0 + k) * (size_t)n + (size_t)(i0 + r);
            if (k < scnt[r]) {
                ev[off] = tv[k * kEllPitch + r];
                ei[off] = ti[k * kEllPitch + r];
            } else {
                ev[off] = (R)0;
                ei[off] = i0 + r;
            }
        }
    }
}

template <typename R>
static hipError_t ell_pack_t(int n, int width, const int* ptr, const int* idx, const void* val, void* ev,
                             int* ei, hipStream_t s) {
    dim3 grid((unsigned)((n + kEllRows - 1) / kEllRows), (unsigned)((width + kEllSlots - 1) / kEllSlots));
    hipLaunchKernelGGL(k_ell_pack<R>, grid, dim3(kBlock), 0, s, n, width, ptr, idx, (const R*)val, (R*)ev, ei);
    return hipGetLastError();
}

hipError_t launch_ell_pack(int n, int width, const int* ptr, const int* idx, const void* val, int vbytes,
                           void* ell_val, int* ell_idx, hipStream_t s) {
    if (width == 0) return hipSuccess;
    switch (vbytes) {
        case 8: return ell_pack_t<uint64_t>(n, width, ptr, idx, val, ell_val, ell_idx, s);
        case 4: return ell_pack_t<uint32_t>(n, width, ptr, idx, val, ell_val, ell_idx, s);
        default: return ell_pack_t<uint16_t>(n, width, ptr, idx, val, ell_val, ell_idx, s);
    }
}

}  // namespace spmvat
