// CRS -> CCS (Phase I of section 2.1) as a least-significant-digit radix
// sort of the entries by column, for matrices whose columns are scattered.
//
// The column-wise form holds the entries ordered by column and, within a
// column, in CRS order (rows ascending, each row in storage order).  That is
// the CRS sequence sorted by column with a stable sort, and a stable sort
// by column equals passes of stable sorts by its 8-bit digits, least
// significant first.  Each pass:
//   hist     per tile of 2048 consecutive entries: entries per digit value,
//            into a digit-major table (digit d, tile t) -> d * tiles + t;
//   scan     the table, exclusively, in that order: the start of every
//            (digit, tile) run in the pass's output;
//   scatter  per tile: the entries ranked stably by digit inside the tile
//            (per-wave counts, their scan, ballot ranks inside a group of
//            64), laid out by digit in LDS and written out in that order,
//            so that each digit's run leaves the tile as one contiguous
//            stretch.
// Entries travel as (column, row, value); the rows of the first pass come
// from the row pointers (the COO-Row expansion), the last pass writes the
// rows and values straight into the CCS arrays and keeps the sorted columns,
// from which the column pointer follows.
#include "common.h"
#include "kernels.h"

namespace spmvat {

namespace {

constexpr int kRxBits = 8;
constexpr int kRxBins = 1 << kRxBits;
constexpr int kRxThreads = 256;
constexpr int kRxWaves = kRxThreads / kWave;
constexpr int kRxPer = 8;                             // entries per thread
constexpr int kRxTile = kRxThreads * kRxPer;          // entries per tile
constexpr int kRxGroups = kRxTile / kRxWaves / kWave; // groups of 64 per wave
constexpr int kRxScan = 4096;                         // table entries per scan workgroup
constexpr int kRxHistTiles = 4;                       // tiles per histogram workgroup
constexpr int kRxCcpPer = 8;                          // sorted columns per thread (column pointer)
static_assert(kRxThreads == kRxBins, "one thread per digit value in the tile scan");
static_assert(kRxScan % kRxThreads == 0, "the scan gives each thread whole runs");

__device__ __forceinline__ int rx_block_scan(int v, int* wsum, int* total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int u = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += u;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kRxWaves; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    if (total) *total = all;
    return before + incl - v;
}

}  // namespace

RadixGeom radix_geom(int n, int64_t nnz) {
    RadixGeom g{};
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
    g.passes = bits <= kRxBits ? 1 : (bits + kRxBits - 1) / kRxBits;
    g.tiles = (nnz + kRxTile - 1) / kRxTile;
    g.table = g.tiles * kRxBins;
    g.chunks = (g.table + kRxScan - 1) / kRxScan;
    return g;
}

// ------------------------------------------------------------------ hist

// kRxHistTiles tiles per workgroup; each thread counts 8 consecutive
// entries of a tile (two 16-byte loads).
__global__ void __launch_bounds__(kRxThreads)
k_rx_hist(int64_t nnz, int64_t tiles, int shift, const int* __restrict__ col, int* __restrict__ table) {
    static_assert(kRxPer == 8, "two 16-byte loads per thread and tile");
    __shared__ int h[kRxHistTiles * kRxBins];
    const int64_t tb = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kRxHistTiles;
    for (int i = threadIdx.x; i < kRxHistTiles * kRxBins; i += kRxThreads) h[i] = 0;
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < kRxHistTiles; ++tt) {
        const int64_t q0 = (tb + tt) * kRxTile + (int64_t)threadIdx.x * kRxPer;
        if (tb + tt >= tiles || q0 >= nnz) continue;
        int c[kRxPer];
        if (q0 + kRxPer <= nnz) {
            const int4 a = *reinterpret_cast<const int4*>(col + q0);
            const int4 b = *reinterpret_cast<const int4*>(col + q0 + 4);
            c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w; c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
        } else {
#pragma unroll
            for (int k = 0; k < kRxPer; ++k) c[k] = q0 + k < nnz ? col[q0 + k] : -1;
        }
#pragma unroll
        for (int k = 0; k < kRxPer; ++k)
            if (c[k] >= 0) atomicAdd(&h[tt * kRxBins + ((c[k] >> shift) & (kRxBins - 1))], 1);
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < kRxHistTiles; ++tt)
        if (tb + tt < tiles) table[(int64_t)threadIdx.x * tiles + tb + tt] = h[tt * kRxBins + threadIdx.x];
}

// ------------------------------------------------------------------ scan

__global__ void __launch_bounds__(kRxThreads)
k_rx_scan_reduce(int64_t m, const int* __restrict__ a, int* __restrict__ csum) {
    __shared__ int wsum[kRxWaves];
    const int64_t c0 = (int64_t)blockIdx.x * kRxScan;
    int s = 0;
    for (int k = threadIdx.x; k < kRxScan; k += kRxThreads)
        if (c0 + k < m) s += a[c0 + k];
    int total;
    rx_block_scan(s, wsum, &total);
    if (threadIdx.x == 0) csum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kRxThreads)
k_rx_scan_top(int64_t chunks, int* __restrict__ csum) {
    __shared__ int wsum[kRxWaves];
    int carry = 0;
    for (int64_t c0 = 0; c0 < chunks; c0 += kRxThreads) {
        const int64_t i = c0 + threadIdx.x;
        const int v = i < chunks ? csum[i] : 0;
        int total;
        const int ex = rx_block_scan(v, wsum, &total);
        if (i < chunks) csum[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(kRxThreads)
k_rx_scan_apply(int64_t m, int* __restrict__ a, const int* __restrict__ csum) {
    __shared__ int wsum[kRxWaves];
    constexpr int kPer = kRxScan / kRxThreads;
    const int64_t c0 = (int64_t)blockIdx.x * kRxScan + (int64_t)threadIdx.x * kPer;
    static_assert(kPer % 4 == 0, "a thread's counts are whole 16-byte vectors");
    // a thread's run by 16-byte loads and stores (the table is 256-byte
    // aligned and runs start at multiples of kPer); the last run of the
    // table one count at a time
    const bool whole = c0 + kPer <= m;
    int v[kPer];
    if (whole) {
        const int4* p = reinterpret_cast<const int4*>(a + c0);
#pragma unroll
        for (int q = 0; q < kPer / 4; ++q) {
            const int4 x = p[q];
            v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k) v[k] = c0 + k < m ? a[c0 + k] : 0;
    }
    int s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) s += v[k];
    int run = csum[blockIdx.x] + rx_block_scan(s, wsum, nullptr);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int x = v[k];
        v[k] = run;
        run += x;
    }
    if (whole) {
        int4* p = reinterpret_cast<int4*>(a + c0);
#pragma unroll
        for (int q = 0; q < kPer / 4; ++q) p[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (c0 + k < m) a[c0 + k] = v[k];
    }
}

// --------------------------------------------------------------- scatter

// One pass over a tile: wave w takes the tile's entries w * 512 .. + 511 as
// 8 groups of 64 in order, so that (wave, group, lane) is the entries'
// order.  The entries are held in registers between the count and the
// placement.  (Tiles of 1024, 2048, 4096 and 8192 entries took 3.20, 2.76,
// 3.02 and 4.20 ms on the power-law matrix.)
template <typename V>
__global__ void __launch_bounds__(kRxThreads)
k_rx_scatter(int64_t nnz, int64_t tiles, int shift, const int* __restrict__ col_in, const int* __restrict__ row_in,
             const V* __restrict__ val_in, const int* __restrict__ table, int* __restrict__ col_out,
             int* __restrict__ row_out, V* __restrict__ val_out) {
    __shared__ int cnt[kRxWaves * kRxBins];   // per-wave digit counts, then per-wave starts in the tile
    __shared__ int dstart[kRxBins];           // each digit's start in the tile
    __shared__ int goff[kRxBins];             // each digit's start in the pass's output
    __shared__ int wsum[kRxWaves];
    __shared__ int s_col[kRxTile];
    __shared__ int s_row[kRxTile];
    __shared__ V s_val[kRxTile];
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t0 = tile * kRxTile;
    const int cntt = (int)min((int64_t)kRxTile, nnz - t0);
    const int tid = threadIdx.x, w = tid / kWave, lane = tid & (kWave - 1);
    for (int i = tid; i < kRxWaves * kRxBins; i += kRxThreads) cnt[i] = 0;
    goff[tid] = table[(int64_t)tid * tiles + tile];
    __syncthreads();
    int c[kRxGroups], r[kRxGroups];
    V v[kRxGroups];
#pragma unroll
    for (int g = 0; g < kRxGroups; ++g) {
        const int q = (w * kRxGroups + g) * kWave + lane;
        c[g] = 0;
        r[g] = 0;
        v[g] = 0;
        if (q < cntt) {
            c[g] = col_in[t0 + q];
            r[g] = row_in[t0 + q];
            v[g] = ld_nt(&val_in[t0 + q]);
            atomicAdd(&cnt[w * kRxBins + ((c[g] >> shift) & (kRxBins - 1))], 1);
        }
    }
    __syncthreads();
    {
        // digit d = tid: its total in the tile, its start, each wave's start
        int tot = 0;
#pragma unroll
        for (int ww = 0; ww < kRxWaves; ++ww) tot += cnt[ww * kRxBins + tid];
        const int ex = rx_block_scan(tot, wsum, nullptr);
        dstart[tid] = ex;
        int run = ex;
#pragma unroll
        for (int ww = 0; ww < kRxWaves; ++ww) {
            const int k = cnt[ww * kRxBins + tid];
            cnt[ww * kRxBins + tid] = run;
            run += k;
        }
    }
    __syncthreads();
    int* cur = cnt + w * kRxBins;
    const uint64_t below = lanes_below();
#pragma unroll
    for (int g = 0; g < kRxGroups; ++g) {
        const int q = (w * kRxGroups + g) * kWave + lane;
        const bool valid = q < cntt;
        const uint32_t d = (uint32_t)(c[g] >> shift) & (kRxBins - 1);
        const uint64_t m = match_low_bits(d, kRxBits, __ballot(valid));
        const int rank = (int)__popcll(m & below);
        int slot = 0;
        if (valid) slot = cur[d];
        if (valid && rank == 0) cur[d] = slot + (int)__popcll(m);
        if (valid) {
            const int pos = slot + rank;
            s_col[pos] = c[g];
            s_row[pos] = r[g];
            s_val[pos] = v[g];
        }
    }
    __syncthreads();
    for (int i = tid; i < cntt; i += kRxThreads) {
        const int cc = s_col[i];
        const int d = (cc >> shift) & (kRxBins - 1);
        const int64_t o = (int64_t)goff[d] + (i - dstart[d]);
        col_out[o] = cc;
        row_out[o] = s_row[i];
        val_out[o] = s_val[i];
    }
}

// ------------------------------------------------------- column pointer

// From the columns in sorted order: ccp[j] is the first position whose
// column is at least j; the last position also fills the columns after it,
// and ccp[n] = nnz.  Each thread takes 8 consecutive positions.
__global__ void __launch_bounds__(kBlock)
k_rx_ccp(int n, int64_t nnz, const int* __restrict__ scol, int* __restrict__ ccp) {
    static_assert(kRxCcpPer == 8, "two 16-byte loads per thread");
    const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kRxCcpPer;
    if (i0 >= nnz) return;
    int c[kRxCcpPer];
    if (i0 + kRxCcpPer <= nnz) {
        const int4 a = *reinterpret_cast<const int4*>(scol + i0);
        const int4 b = *reinterpret_cast<const int4*>(scol + i0 + 4);
        c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w; c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kRxCcpPer; ++k) c[k] = i0 + k < nnz ? scol[i0 + k] : 0;
    }
    int pc = i0 > 0 ? scol[i0 - 1] : -1;
#pragma unroll
    for (int k = 0; k < kRxCcpPer; ++k) {
        const int64_t i = i0 + k;
        if (i >= nnz) break;
        for (int j = pc + 1; j <= c[k]; ++j) ccp[j] = (int)i;
        pc = c[k];
    }
    if (i0 + kRxCcpPer >= nnz)
        for (int j = pc + 1; j <= n; ++j) ccp[j] = (int)nnz;
}

// The longest column, and the total, into the summary (zeroed before).
__global__ void __launch_bounds__(kBlock)
k_rx_summary(int n, const int* __restrict__ ccp, ColSummary* __restrict__ sum) {
    __shared__ int wmax[kBlock / kWave];
    int m = 0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock)
        m = max(m, ccp[j + 1] - ccp[j]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / kWave; ++k) m = max(m, wmax[k]);
        if (m > 0) atomicMax(&sum->max_len, m);
        if (blockIdx.x == 0) sum->total = ccp[n];
    }
}

// ---------------------------------------------------------------- launcher

template <typename V>
static hipError_t run_radix(const RadixGeom& g, int n, int64_t nnz, const int* irp, const int* icol,
                            const void* val, const RadixWs& ws, int* ccp, int* irow_t, void* val_t,
                            ColSummary* sum, hipStream_t s) {
    hipError_t e = launch_fill_zero(sum, sizeof(ColSummary), s);
    if (e != hipSuccess || nnz == 0) return e;
    // the rows of the first pass: the COO-Row expansion of the row pointers
    if ((e = launch_expand_ptr(n, irp, ws.xrow, s)) != hipSuccess) return e;
    const int* cin = icol;
    const int* rin = ws.xrow;
    const V* vin = static_cast<const V*>(val);
    const int* scol = nullptr;
    for (int pass = 0; pass < g.passes; ++pass) {
        const int shift = pass * kRxBits;
        const bool last = pass == g.passes - 1;
        // alternate between the two buffers; the last pass writes the CCS
        // arrays and keeps its columns in the buffer it does not read
        const bool into_y = (pass % 2) == 0;
        int* cout = into_y ? ws.ycol : ws.xcol;
        int* rout = last ? irow_t : (into_y ? ws.yrow : ws.xrow);
        V* vout = last ? static_cast<V*>(val_t) : static_cast<V*>(into_y ? ws.yval : ws.xval);
        hipLaunchKernelGGL(k_rx_hist, dim3((unsigned)((g.tiles + kRxHistTiles - 1) / kRxHistTiles)), dim3(kRxThreads),
                           0, s, nnz, g.tiles, shift, cin, ws.table);
        hipLaunchKernelGGL(k_rx_scan_reduce, dim3((unsigned)g.chunks), dim3(kRxThreads), 0, s, g.table, ws.table,
                           ws.csum);
        hipLaunchKernelGGL(k_rx_scan_top, dim3(1), dim3(kRxThreads), 0, s, g.chunks, ws.csum);
        hipLaunchKernelGGL(k_rx_scan_apply, dim3((unsigned)g.chunks), dim3(kRxThreads), 0, s, g.table, ws.table,
                           ws.csum);
        hipLaunchKernelGGL(k_rx_scatter<V>, dim3((unsigned)g.tiles), dim3(kRxThreads), 0, s, nnz, g.tiles, shift,
                           cin, rin, vin, ws.table, cout, rout, vout);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cin = cout;
        rin = rout;
        vin = vout;
        scol = cout;
    }
    const int64_t per_block = (int64_t)kBlock * kRxCcpPer;
    hipLaunchKernelGGL(k_rx_ccp, dim3((unsigned)((nnz + per_block - 1) / per_block)), dim3(kBlock), 0, s, n, nnz, scol,
                       ccp);
    const int grid = (int)std::min<int64_t>(1024, ((int64_t)n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_rx_summary, dim3((unsigned)std::max(grid, 1)), dim3(kBlock), 0, s, n, ccp, sum);
    return hipGetLastError();
}

hipError_t launch_ccs_radix(const RadixGeom& g, int n, int64_t nnz, const int* irp, const int* icol,
                            const void* val, int vbytes, const RadixWs& ws, int* ccp, int* irow_t, void* val_t,
                            ColSummary* sum, hipStream_t s) {
    switch (vbytes) {
        case 8: return run_radix<uint64_t>(g, n, nnz, irp, icol, val, ws, ccp, irow_t, val_t, sum, s);
        case 4: return run_radix<uint32_t>(g, n, nnz, irp, icol, val, ws, ccp, irow_t, val_t, sum, s);
        case 2: return run_radix<uint16_t>(g, n, nnz, irp, icol, val, ws, ccp, irow_t, val_t, sum, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spmvat
