// CRS -> CCS (Phase I of section 2.1) as a two-level stable counting sort.
//
// The serial method counts the entries of every column, scans the counts
// into the column pointer and then places the entries, rows ascending and
// each row in storage order, at a per-column cursor.  On the GPU the same
// order comes from two stable passes, neither of which lets an atomic
// decide a position.  Built for matrices whose columns are scattered (large
// bandwidth), where per-entry global atomics on random columns are slow:
//
//   level 1  entries are distributed to column blocks of 1024 columns.  Each
//            workgroup owns a tile of consecutive rows; a bucket-major table
//            of per-(block, tile) counts is scanned so that every tile knows
//            where its run of each block starts, and inside a tile the waves
//            take consecutive stretches of entries and rank equal blocks by
//            wave ballots, so each block keeps the entries in CRS order.
//            The payload is a 32-bit key (column within the block : 10 bits,
//            row : 22 bits) and the value.
//   level 2  a workgroup takes one column block at a time, counts its
//            columns, scans them into the column pointer and places the
//            block's entries, again in order and ranked by ballots, into the
//            final arrays.  All writes of a block fall inside its own slice of
//            the output; the grid is sized so that the slices being written
//            at one time stay in the last-level cache.
//
// Bytes moved, nnz entries of V-byte values: level 1 reads icol twice and
// val once and writes (4 + V) per entry; level 2 reads the key array twice
// and the values once and writes (4 + V) per entry; the count table is
// (n / 1024) x (n / rows per tile) integers.  Applies for n <= 2^22.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace spmvat {

namespace {

constexpr int kBlkBits = kCcsBlockBits;
constexpr int kBlk = 1 << kBlkBits;
constexpr uint32_t kRowMask = (1u << kCcsRowBits) - 1;
constexpr int kBatch = 4;           // rounds of 64 entries loaded before any is placed
constexpr int kChunk = 4096;        // counts per workgroup of the table scan
constexpr int kMaxWaves = 16;
// level 2: waves per workgroup and workgroups of the persistent grid; the
// output slices of the blocks being placed at one time then stay within
// the last-level cache
constexpr int kPlaceWaves = 8;
constexpr int kPlaceThreads = kPlaceWaves * kWave;
constexpr int kPlaceGrid = 512;

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

template <int kBytes> struct Raw;
template <> struct Raw<8> { using type = unsigned long long; };
template <> struct Raw<4> { using type = uint32_t; };
template <> struct Raw<2> { using type = uint16_t; };

// Counting needs no order: one LDS atomic per valid lane.
__device__ __forceinline__ void count_keys(int* cnt, uint32_t key, bool valid) {
    if (valid) atomicAdd(&cnt[key], 1);
}

}  // namespace

CcsGeom ccs_geom(int n) {
    CcsGeom g{};
    g.nb = (n + kBlk - 1) / kBlk;
    int rows = 256;
    while (rows < 2048 && (int64_t)((n + rows - 1) / rows) * g.nb > (8ll << 20)) rows *= 2;
    g.rows = rows;
    g.tiles = (n + rows - 1) / rows;
    g.table = (int64_t)g.tiles * g.nb;
    g.chunks = (g.table + kChunk - 1) / kChunk;
    int bits = 0;
    while ((1 << bits) < g.nb) ++bits;
    g.nb_bits = bits;
    // waves per level-1 workgroup: per-wave block counters plus the tile's
    // row pointers must fit in 64 KiB of LDS
    g.waves = 4;
    while (g.waves > 1 && (size_t)(g.waves * g.nb + rows + 1) * 4 > 65536) g.waves /= 2;
    return g;
}

// ---------------------------------------------------------------- level 1

// Per tile: entries per column block, into table[block * tiles + tile].
__global__ void __launch_bounds__(kBlock)
k_bucket_count(int n, int rows_per_tile, int tiles, int nb, const int* __restrict__ irp,
               const int* __restrict__ icol, int* __restrict__ table) {
    extern __shared__ int cnt[];   // nb
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int r0 = tile * rows_per_tile;
    const int r1 = min(n, r0 + rows_per_tile);
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    const int e0 = irp[r0], e1 = irp[r1];
    for (int64_t base = e0; base < e1; base += blockDim.x) {
        const int64_t p = base + threadIdx.x;
        const bool valid = p < e1;
        const uint32_t b = valid ? (uint32_t)icol[p] >> kBlkBits : 0u;
        count_keys(cnt, b, valid);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) table[(int64_t)b * tiles + tile] = cnt[b];
}

// Exclusive scan of the table, in place: chunk sums, a scan of the sums by
// one workgroup, then each chunk rescanned with its offset.
__device__ __forceinline__ int block_exclusive_scan(int v, int* wsum, int* total) {
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
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    if (total) *total = all;
    return before + incl - v;
}

__global__ void __launch_bounds__(kBlock)
k_table_reduce(int64_t m, const int* __restrict__ a, int* __restrict__ csum) {
    __shared__ int wsum[kMaxWaves];
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    int s = 0;
    for (int k = threadIdx.x; k < kChunk; k += kBlock) {
        const int64_t i = c0 + k;
        if (i < m) s += a[i];
    }
    int total;
    block_exclusive_scan(s, wsum, &total);
    if (threadIdx.x == 0) csum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock)
k_table_top(int chunks, int* __restrict__ csum, ColSummary* __restrict__ sum) {
    __shared__ int wsum[kMaxWaves];
    int carry = 0;
    for (int c0 = 0; c0 < chunks; c0 += kBlock) {
        const int i = c0 + threadIdx.x;
        const int v = i < chunks ? csum[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, wsum, &total);
        if (i < chunks) csum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        sum->total = carry;
        sum->max_len = 0;
        sum->n_mid = 0;
        sum->n_long = 0;
    }
}

__global__ void __launch_bounds__(kBlock)
k_table_apply(int64_t m, int* __restrict__ a, const int* __restrict__ csum) {
    __shared__ int wsum[kMaxWaves];
    constexpr int kPer = kChunk / kBlock;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kPer;
    int v[kPer];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        v[k] = c0 + k < m ? a[c0 + k] : 0;
        s += v[k];
    }
    int run = csum[blockIdx.x] + block_exclusive_scan(s, wsum, nullptr);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (c0 + k < m) a[c0 + k] = run;
        run += v[k];
    }
}

// Per tile: each wave takes a consecutive stretch of the tile's entries,
// counts its blocks, takes its start in every block after the tile's start
// (from the scanned table) and the earlier waves' counts, then writes its
// entries in order, ranking equal blocks inside a round of 64 by ballots.
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_bucket_scatter(int n, int rows_per_tile, int tiles, int nb, int nb_bits, const int* __restrict__ irp,
                 const int* __restrict__ icol, const R* __restrict__ val, const int* __restrict__ table,
                 uint32_t* __restrict__ bkey, R* __restrict__ bval) {
    extern __shared__ int lds[];
    const int waves = blockDim.x / kWave;
    int* cur = lds;                     // waves x nb
    int* sp = lds + waves * nb;         // rows_per_tile + 1
    const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
    const int r0 = tile * rows_per_tile;
    const int rows = min(n, r0 + rows_per_tile) - r0;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < waves * nb; i += blockDim.x) cur[i] = 0;
    for (int i = threadIdx.x; i <= rows; i += blockDim.x) sp[i] = irp[r0 + i];
    __syncthreads();
    const int e0 = sp[0], e1 = sp[rows];
    const int64_t q = ((int64_t)(e1 - e0) + waves - 1) / waves;
    const int64_t ws = min64(e1, e0 + q * w), we = min64(e1, ws + q);
    int* mine = cur + w * nb;
    for (int64_t base = ws; base < we; base += kWave) {
        const int64_t p = base + lane;
        const bool valid = p < we;
        const uint32_t b = valid ? (uint32_t)icol[p] >> kBlkBits : 0u;
        count_keys(mine, b, valid);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int run = table[(int64_t)b * tiles + tile];
        for (int k = 0; k < waves; ++k) {
            const int c = cur[k * nb + b];
            cur[k * nb + b] = run;
            run += c;
        }
    }
    __syncthreads();
    if (ws >= we) return;
    // the row of this lane's first entry, then a walk as the entry advances
    int r = last_le(sp, 0, rows - 1, (int)min64(ws + lane, e1 - 1));
    for (int64_t base = ws; base < we; base += (int64_t)kWave * kBatch) {
        uint32_t col[kBatch];
        R v[kBatch];
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            const int64_t p = base + g * kWave + lane;
            col[g] = 0;
            if (p < we) { col[g] = (uint32_t)icol[p]; v[g] = val[p]; }
        }
#pragma unroll
        for (int g = 0; g < kBatch; ++g) {
            const int64_t p = base + g * kWave + lane;
            const bool valid = p < we;
            if (valid) while (sp[r + 1] <= p) ++r;
            const uint32_t b = col[g] >> kBlkBits;
            const uint64_t act = __ballot(valid);
            const uint64_t m = match_low_bits(b, nb_bits, act);
            const int rank = (int)__popcll(m & lanes_below());
            int slot = 0;
            if (valid) slot = mine[b];
            if (valid && rank == 0) mine[b] = slot + (int)__popcll(m);
            if (valid) {
                const int pos = slot + rank;
                bkey[pos] = ((col[g] & (kBlk - 1)) << kCcsRowBits) | (uint32_t)(r0 + r);
                bval[pos] = v[g];
            }
        }
    }
}

// ---------------------------------------------------------------- level 2

// Column blocks, one at a time per workgroup of a persistent grid: column
// counts, the column pointer of the block, then the ordered placement of the
// block's entries.  Each wave takes one eighth of the block's entries.
template <typename R>
__global__ void __launch_bounds__(kPlaceThreads)
k_block_place(int n, int64_t nnz, int nb, int tiles, const int* __restrict__ table,
              const uint32_t* __restrict__ bkey, const R* __restrict__ bval, int* __restrict__ ccp,
              int* __restrict__ irow_t, R* __restrict__ val_t, ColSummary* __restrict__ sum) {
    __shared__ int cur[kPlaceWaves * kBlk];
    __shared__ int wsum[kMaxWaves];
    __shared__ int wmax[kPlaceWaves];
    constexpr int kCols = kBlk / kPlaceThreads;   // columns owned by a thread in the scan
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    int* mine = cur + w * kBlk;
    int block_max = 0;
    for (int blk = blockIdx.x; blk < nb; blk += gridDim.x) {
        const int c0 = blk * kBlk;
        const int s = table[(int64_t)blk * tiles];
        const int e = blk + 1 < nb ? table[(int64_t)(blk + 1) * tiles] : (int)nnz;
        __syncthreads();   // the previous block's placement is done with cur
        for (int i = threadIdx.x; i < kPlaceWaves * kBlk; i += kPlaceThreads) cur[i] = 0;
        __syncthreads();
        const int64_t q = ((int64_t)(e - s) + kPlaceWaves - 1) / kPlaceWaves;
        const int64_t ws = min64(e, s + q * w), we = min64(e, ws + q);
        for (int64_t base = ws; base < we; base += kWave) {
            const int64_t p = base + lane;
            const bool valid = p < we;
            const uint32_t c = valid ? bkey[p] >> kCcsRowBits : 0u;
            count_keys(mine, c, valid);
        }
        __syncthreads();
        int tot[kCols], loc = 0;
#pragma unroll
        for (int k = 0; k < kCols; ++k) {
            const int c = threadIdx.x * kCols + k;
            tot[k] = 0;
            for (int v = 0; v < kPlaceWaves; ++v) tot[k] += cur[v * kBlk + c];
            loc += tot[k];
            block_max = max(block_max, tot[k]);
        }
        int run = s + block_exclusive_scan(loc, wsum, nullptr);
#pragma unroll
        for (int k = 0; k < kCols; ++k) {
            const int c = threadIdx.x * kCols + k;
            if (c0 + c < n) ccp[c0 + c] = run;
            int r = run;
            for (int v = 0; v < kPlaceWaves; ++v) {
                const int cv = cur[v * kBlk + c];
                cur[v * kBlk + c] = r;
                r += cv;
            }
            run += tot[k];
        }
        if (blk == nb - 1 && threadIdx.x == 0) ccp[n] = (int)nnz;
        __syncthreads();
        for (int64_t base = ws; base < we; base += (int64_t)kWave * kBatch) {
            uint32_t key[kBatch];
            R v[kBatch];
#pragma unroll
            for (int g = 0; g < kBatch; ++g) {
                const int64_t p = base + g * kWave + lane;
                key[g] = 0;
                if (p < we) { key[g] = bkey[p]; v[g] = bval[p]; }
            }
#pragma unroll
            for (int g = 0; g < kBatch; ++g) {
                const bool valid = base + g * kWave + lane < we;
                const uint32_t c = key[g] >> kCcsRowBits;
                const uint64_t act = __ballot(valid);
                const uint64_t m = match_low_bits(c, kBlkBits, act);
                const int rank = (int)__popcll(m & lanes_below());
                int slot = 0;
                if (valid) slot = mine[c];
                if (valid && rank == 0) mine[c] = slot + (int)__popcll(m);
                if (valid) {
                    irow_t[slot + rank] = (int)(key[g] & kRowMask);
                    val_t[slot + rank] = v[g];
                }
            }
        }
    }
    // longest column over the blocks this workgroup placed
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) block_max = max(block_max, __shfl_xor(block_max, off, kWave));
    if (lane == 0) wmax[w] = block_max;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = wmax[0];
        for (int k = 1; k < kPlaceWaves; ++k) m = max(m, wmax[k]);
        atomicMax(&sum->max_len, m);
    }
}

template <typename R>
hipError_t run_bucketed(const CcsGeom& g, int n, int64_t nnz, const int* irp, const int* icol, const void* val,
                        int* table, int* csum, uint32_t* bkey, void* bval, int* ccp, int* irow_t, void* val_t,
                        ColSummary* sum, hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_count, dim3(g.tiles), dim3(kBlock), g.nb * sizeof(int), s, n, g.rows, g.tiles,
                       g.nb, irp, icol, table);
    hipLaunchKernelGGL(k_table_reduce, dim3((unsigned)g.chunks), dim3(kBlock), 0, s, g.table, table, csum);
    hipLaunchKernelGGL(k_table_top, dim3(1), dim3(kBlock), 0, s, (int)g.chunks, csum, sum);
    hipLaunchKernelGGL(k_table_apply, dim3((unsigned)g.chunks), dim3(kBlock), 0, s, g.table, table, csum);
    const size_t lds = (size_t)(g.waves * g.nb + g.rows + 1) * sizeof(int);
    hipLaunchKernelGGL(k_bucket_scatter<R>, dim3(g.tiles), dim3(g.waves * kWave), lds, s, n, g.rows, g.tiles,
                       g.nb, g.nb_bits, irp, icol, static_cast<const R*>(val), table, bkey, static_cast<R*>(bval));
    hipLaunchKernelGGL(k_block_place<R>, dim3(std::min(g.nb, kPlaceGrid)), dim3(kPlaceThreads), 0, s, n, nnz, g.nb,
                       g.tiles, table, bkey,
                       static_cast<const R*>(bval), ccp, irow_t, static_cast<R*>(val_t), sum);
    return hipGetLastError();
}

hipError_t launch_ccs_bucketed(const CcsGeom& g, int n, int64_t nnz, const int* irp, const int* icol,
                               const void* val, int vbytes, int* table, int* csum, uint32_t* bkey, void* bval,
                               int* ccp, int* irow_t, void* val_t, ColSummary* sum, hipStream_t s) {
    switch (vbytes) {
        case 8: return run_bucketed<Raw<8>::type>(g, n, nnz, irp, icol, val, table, csum, bkey, bval, ccp, irow_t,
                                                   val_t, sum, s);
        case 4: return run_bucketed<Raw<4>::type>(g, n, nnz, irp, icol, val, table, csum, bkey, bval, ccp, irow_t,
                                                   val_t, sum, s);
        case 2: return run_bucketed<Raw<2>::type>(g, n, nnz, irp, icol, val, table, csum, bkey, bval, ccp, irow_t,
                                                   val_t, sum, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spmvat
