// CRS -> CCS (Phase I of section 2.1) for matrices of limited bandwidth, as
// a two-level stable counting sort whose stores are all coalesced.
//
// Rows are cut into tiles of R consecutive rows, columns into blocks of 64.
// Every entry of tile t lies in the column window [r0 - bw, r1 + bw)
// (bw = max |i - j| from the row statistics), so a tile only reaches the few
// blocks that window covers, and a count table over each tile's window
// blocks stays small.  Inside a tile each wave owns one consecutive stretch
// of the tile's entries.
//
//   count       per tile: entries per (wave stretch, window block).
//   blocks      one thread per block: a walk over the tiles whose window
//               covers the block, in tile order and wave order inside a
//               tile, turns the counts into each stretch's start inside the
//               block and sums the block's length; the block starts follow
//               by the shared scan kernels.
//   distribute  per tile: each wave moves its stretch, in storage order, to
//               the blocks (equal blocks inside a group of 64 ranked by
//               ballots), as a packed key (row, column within the block) and
//               the value.  A block then holds its entries in CRS order.
//               One tile's run inside a block is long, so stores coalesce.
//   place       one workgroup per block: column counts, the column pointer,
//               and the stable placement of the block's entries by column
//               (per-wave counts, ballot ranks) into LDS, written out in
//               order; blocks larger than the LDS stage write in place.
//
// CRS order inside each block, kept by a stable sort on the column, is the
// paper's order: rows ascending, each row's entries in storage order.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace spmvat {

namespace {

constexpr int kBcBits = 6;                 // columns per block: 64
constexpr int kBcCols = 1 << kBcBits;
constexpr int kBcRows = 2048;              // rows per tile
constexpr int kBcWaves = 16;               // waves per tile (count, distribute)
constexpr int kBcThreads = kBcWaves * kWave;
constexpr int kBcUnroll = 8;               // groups of 64 entries loaded ahead
constexpr int kPlWaves = 8;                // place: waves per block
constexpr int kPlThreads = kPlWaves * kWave;
constexpr int kPlStageBytes = 36 * 1024;   // place: LDS stage of rows and values
constexpr int kPlBlocks = 4;               // place: blocks per workgroup
constexpr int kPlPer = 4;                  // place: entries per lane and block held in registers
constexpr int kBcMaxWindowBlocks = 1536;   // count / distribute LDS: 16 waves x 1536 counters = 96 KiB

__device__ __forceinline__ int bc_lo(int t, int bw) { return max(0, t * kBcRows - bw); }
__device__ __forceinline__ int bc_hi(int n, int t, int bw) {
    const int64_t r1 = min((int64_t)n, (int64_t)(t + 1) * kBcRows);
    return (int)min((int64_t)n, r1 + bw);
}

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

// Wave w's stretch of [e0, e1) when the waves of a workgroup split it evenly.
__device__ __forceinline__ void stretch(int e0, int e1, int waves, int w, int& ws, int& we) {
    const int q = (e1 - e0 + waves - 1) / waves;
    ws = (int)min64(e1, (int64_t)e0 + (int64_t)q * w);
    we = (int)min64(e1, (int64_t)ws + q);
}

}  // namespace

WccsGeom wccs_geom(int n, int bw, int max_row) {
    (void)max_row;
    WccsGeom g{};
    g.rows = kBcRows;
    g.tiles = (n + kBcRows - 1) / kBcRows;
    g.nb = (n + kBcCols - 1) / kBcCols;
    const int64_t wmax = std::min<int64_t>(n, (int64_t)kBcRows + 2 * (int64_t)std::max(bw, 0));
    g.nwbmax = (int)((wmax + kBcCols - 1) / kBcCols) + 1;
    g.table = (int64_t)g.tiles * kBcWaves * g.nwbmax;
    int bits = 1;
    while ((1 << bits) < g.nwbmax) ++bits;
    g.wb_bits = bits;
    // the packed key keeps the row in 32 - kBcBits bits
    g.usable = bw >= 0 && n <= (1 << (32 - kBcBits)) && g.nwbmax <= kBcMaxWindowBlocks;
    return g;
}

// ------------------------------------------------------------------ count

__global__ void __launch_bounds__(kBcThreads)
k_bcs_count(int n, int bw, int nwbmax, const int* __restrict__ irp, const int* __restrict__ icol,
            int* __restrict__ table, WccsInfo* __restrict__ info) {
    extern __shared__ int lds_c[];   // kBcWaves x nwbmax
    const int t = (int)xcd_block(blockIdx.x, gridDim.x);
    const int r0 = t * kBcRows, r1 = min(n, r0 + kBcRows);
    const int b0 = bc_lo(t, bw) >> kBcBits, b1 = (bc_hi(n, t, bw) - 1) >> kBcBits;
    const int nwb = b1 - b0 + 1;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < kBcWaves * nwb; i += kBcThreads) lds_c[(i / nwb) * nwbmax + i % nwb] = 0;
    __syncthreads();
    int ws, we;
    stretch(irp[r0], irp[r1], kBcWaves, w, ws, we);
    int* mine = lds_c + w * nwbmax;
    bool outside = false;
    for (int base = ws; base < we; base += kWave * kBcUnroll) {
        int c[kBcUnroll];
#pragma unroll
        for (int u = 0; u < kBcUnroll; ++u) c[u] = icol[min(base + u * kWave + lane, we - 1)];
#pragma unroll
        for (int u = 0; u < kBcUnroll; ++u) {
            if (base + u * kWave + lane >= we) continue;
            const unsigned wb = (unsigned)((c[u] >> kBcBits) - b0);
            if (wb < (unsigned)nwb) atomicAdd(&mine[wb], 1);
            else outside = true;
        }
    }
    if (outside) atomicOr(&info->flags, kWccsOutside);
    __syncthreads();
    int* trow = table + (int64_t)t * kBcWaves * nwbmax;
    for (int i = threadIdx.x; i < kBcWaves * nwb; i += kBcThreads) {
        const int ww = i / nwb, wb = i % nwb;
        trow[ww * nwbmax + wb] = lds_c[ww * nwbmax + wb];
    }
}

// ----------------------------------------------------------------- blocks

__global__ void __launch_bounds__(kBlock)
k_bcs_blocks(int n, int bw, int tiles, int nb, int nwbmax, int* __restrict__ table, int* __restrict__ bcnt) {
    const int b = (int)blockIdx.x * kBlock + (int)threadIdx.x;
    if (b >= nb) return;
    // tiles whose window blocks [lo / 64, (hi - 1) / 64] hold b: a range a
    // little wider than needed, checked per tile
    const int64_t c0 = (int64_t)b * kBcCols;
    const int64_t a = c0 - bw - kBcRows;
    const int tlo = a <= 0 ? 0 : (int)(a / kBcRows);
    const int thi = (int)min64((int64_t)tiles - 1, (c0 + kBcCols - 1 + bw) / kBcRows);
    int run = 0;
    for (int t = tlo; t <= thi; ++t) {
        const int b0 = bc_lo(t, bw) >> kBcBits, b1 = (bc_hi(n, t, bw) - 1) >> kBcBits;
        if (b < b0 || b > b1) continue;
        int* p = table + (int64_t)t * kBcWaves * nwbmax + (b - b0);
#pragma unroll 4
        for (int w = 0; w < kBcWaves; ++w) {
            const int v = p[w * nwbmax];
            p[w * nwbmax] = run;
            run += v;
        }
    }
    bcnt[b] = run;
}

// ------------------------------------------------------------- distribute

template <typename V>
__global__ void __launch_bounds__(kBcThreads)
k_bcs_distribute(int n, int bw, int nwbmax, int wb_bits, const int* __restrict__ irp, const int* __restrict__ icol,
                 const V* __restrict__ val, const int* __restrict__ table, const int* __restrict__ bstart,
                 uint32_t* __restrict__ key, V* __restrict__ sval) {
    extern __shared__ int lds_d[];   // kBcWaves x nwbmax cursors, then kBcRows + 1 row pointers
    int* sp = lds_d + kBcWaves * nwbmax;
    const int t = (int)xcd_block(blockIdx.x, gridDim.x);
    const int r0 = t * kBcRows, rows = min(n, r0 + kBcRows) - r0;
    const int b0 = bc_lo(t, bw) >> kBcBits, b1 = (bc_hi(n, t, bw) - 1) >> kBcBits;
    const int nwb = b1 - b0 + 1;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int* trow = table + (int64_t)t * kBcWaves * nwbmax;
    for (int i = threadIdx.x; i < kBcWaves * nwb; i += kBcThreads) {
        const int ww = i / nwb, wb = i % nwb;
        lds_d[ww * nwbmax + wb] = bstart[b0 + wb] + trow[ww * nwbmax + wb];
    }
    for (int i = threadIdx.x; i <= rows; i += kBcThreads) sp[i] = irp[r0 + i];
    __syncthreads();
    int ws, we;
    stretch(sp[0], sp[rows], kBcWaves, w, ws, we);
    if (ws >= we) return;
    int* cur = lds_d + w * nwbmax;
    int r = last_le(sp, 0, rows - 1, min(ws + lane, we - 1));
    const uint64_t below = lanes_below();
    for (int base = ws; base < we; base += kWave * kBcUnroll) {
        int col[kBcUnroll];
        V v[kBcUnroll];
#pragma unroll
        for (int u = 0; u < kBcUnroll; ++u) {
            const int p = base + u * kWave + lane;
            col[u] = b0 << kBcBits;
            v[u] = 0;
            if (p < we) { col[u] = icol[p]; v[u] = ld_nt(val + p); }
        }
#pragma unroll
        for (int u = 0; u < kBcUnroll; ++u) {
            const int p = base + u * kWave + lane;
            const int wb = (col[u] >> kBcBits) - b0;
            // entries outside the window (flagged by the count) are left out
            const bool valid = p < we && (unsigned)wb < (unsigned)nwb;
            if (p < we) while (sp[r + 1] <= p) ++r;
            const uint64_t act = __ballot(valid);
            const uint64_t m = match_low_bits((uint32_t)(valid ? wb : 0), wb_bits, act);
            const int rank = (int)__popcll(m & below);
            int slot = 0;
            if (valid) slot = cur[wb];
            if (valid && rank == 0) cur[wb] = slot + (int)__popcll(m);
            if (valid) {
                key[slot + rank] = ((uint32_t)(r0 + r) << kBcBits) | (uint32_t)(col[u] & (kBcCols - 1));
                sval[slot + rank] = v[u];
            }
        }
    }
}

// ------------------------------------------------------------------ place

template <typename V>
struct PlaceSmem {
    static constexpr int kCap = kPlStageBytes / (4 + (int)sizeof(V));
    int cnt[kPlWaves * kBcCols];
    int colptr[kBcCols + 1];
    int s_row[kCap];
    V s_val[kCap];
};

// Column lengths of block b from the per-wave counts, the column pointer,
// the longest column and each wave's start inside every column, in wave
// order (the first wave; lane j owns column j).  Between two barriers.
template <typename V>
__device__ __forceinline__ void place_columns(PlaceSmem<V>& sm, int n, int nb, int b, int s, int e, int* ccp,
                                              WccsInfo* info) {
    const int lane = threadIdx.x & (kWave - 1);
    if (threadIdx.x >= kWave) return;
    const int c0 = b * kBcCols, ncols = min(kBcCols, n - c0);
    int tot = 0;
    for (int ww = 0; ww < kPlWaves; ++ww) tot += sm.cnt[ww * kBcCols + lane];
    int incl = tot;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int u = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += u;
    }
    int run = incl - tot;
    sm.colptr[lane] = run;
    if (lane < ncols) ccp[c0 + lane] = s + run;
    if (b == nb - 1 && lane == 0) ccp[n] = e;
    for (int ww = 0; ww < kPlWaves; ++ww) {
        const int c = sm.cnt[ww * kBcCols + lane];
        sm.cnt[ww * kBcCols + lane] = run;
        run += c;
    }
    int mx = tot;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
    // every block would otherwise hit the one counter with an atomic; most
    // blocks see it already at their maximum
    if (lane == 0 && mx > __hip_atomic_load(&info->kmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&info->kmax, mx);
}

// Stable placement of one group of 64 consecutive entries of a wave's
// stretch (p < we valid): rank among the group's entries of the same column
// by ballots, slot from the wave's cursor of that column.
template <typename V>
__device__ __forceinline__ void place_group(PlaceSmem<V>& sm, int* mine, int p, int we, uint32_t k, V v, bool staged,
                                            int s, int* irow_t, V* val_t) {
    const bool valid = p < we;
    const uint32_t lc = k & (kBcCols - 1);
    const uint64_t mm = match_low_bits(lc, kBcBits, __ballot(valid));
    const int rank = (int)__popcll(mm & lanes_below());
    int slot = 0;
    if (valid) slot = mine[lc];
    if (valid && rank == 0) mine[lc] = slot + (int)__popcll(mm);
    if (valid) {
        const int q = slot + rank;
        if (staged) { sm.s_row[q] = (int)(k >> kBcBits); sm.s_val[q] = v; }
        else { irow_t[s + q] = (int)(k >> kBcBits); val_t[s + q] = v; }
    }
}

// Block b on its own: entries read once to count and again to place.
template <typename V>
__device__ void place_block(PlaceSmem<V>& sm, int n, int nb, int b, const int* bstart, const uint32_t* key,
                            const V* sval, int* ccp, int* irow_t, V* val_t, WccsInfo* info) {
    const int s = bstart[b], e = bstart[b + 1], m = e - s;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    __syncthreads();   // the previous block's stage is written out
    for (int i = threadIdx.x; i < kPlWaves * kBcCols; i += kPlThreads) sm.cnt[i] = 0;
    __syncthreads();
    int ws, we;
    stretch(s, e, kPlWaves, w, ws, we);
    int* mine = sm.cnt + w * kBcCols;
    for (int p = ws + lane; p < we; p += kWave) atomicAdd(&mine[key[p] & (kBcCols - 1)], 1);
    __syncthreads();
    place_columns(sm, n, nb, b, s, e, ccp, info);
    __syncthreads();
    const bool staged = m <= PlaceSmem<V>::kCap;
    for (int base = ws; base < we; base += kWave) {
        const int p = base + lane;
        uint32_t k = 0;
        V v = 0;
        if (p < we) { k = key[p]; v = sval[p]; }
        place_group(sm, mine, p, we, k, v, staged, s, irow_t, val_t);
    }
    if (!staged) return;
    __syncthreads();
    for (int q = threadIdx.x; q < m; q += kPlThreads) {
        irow_t[s + q] = sm.s_row[q];
        val_t[s + q] = sm.s_val[q];
    }
}

// One workgroup per kPlBlocks consecutive blocks.  When every block of the
// group fits the stage and its wave stretches fit kPlPer groups of 64, all
// of the group's entries are loaded into registers at once, so one round
// trip to memory serves several blocks; each block is then counted,
// numbered, placed in LDS and written out in turn.  Otherwise the blocks
// are placed one by one, reading their entries twice.
template <typename V>
__global__ void __launch_bounds__(kPlThreads)
k_bcs_place(int n, int nb, const int* __restrict__ bstart, const uint32_t* __restrict__ key,
            const V* __restrict__ sval, int* __restrict__ ccp, int* __restrict__ irow_t, V* __restrict__ val_t,
            WccsInfo* __restrict__ info) {
    __shared__ PlaceSmem<V> sm;
    const int b0 = (int)xcd_block(blockIdx.x, gridDim.x) * kPlBlocks;
    const int nblk = min(kPlBlocks, nb - b0);
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    bool held = true;
    for (int i = 0; i < nblk; ++i) {
        const int m = bstart[b0 + i + 1] - bstart[b0 + i];
        held = held && m <= PlaceSmem<V>::kCap && (m + kPlWaves - 1) / kPlWaves <= kPlPer * kWave;
    }
    if (!held) {
        for (int i = 0; i < nblk; ++i) place_block(sm, n, nb, b0 + i, bstart, key, sval, ccp, irow_t, val_t, info);
        return;
    }
    uint32_t kk[kPlBlocks][kPlPer];
    V vv[kPlBlocks][kPlPer];
#pragma unroll
    for (int i = 0; i < kPlBlocks; ++i) {
        int ws = 0, we = 0;
        if (i < nblk) stretch(bstart[b0 + i], bstart[b0 + i + 1], kPlWaves, w, ws, we);
#pragma unroll
        for (int u = 0; u < kPlPer; ++u) {
            const int p = ws + u * kWave + lane;
            kk[i][u] = 0;
            vv[i][u] = 0;
            if (p < we) { kk[i][u] = key[p]; vv[i][u] = sval[p]; }
        }
    }
#pragma unroll
    for (int i = 0; i < kPlBlocks; ++i) {
        if (i >= nblk) break;
        const int b = b0 + i;
        const int s = bstart[b], e = bstart[b + 1], m = e - s;
        int ws, we;
        stretch(s, e, kPlWaves, w, ws, we);
        int* mine = sm.cnt + w * kBcCols;
        __syncthreads();   // the previous block's stage is written out
        for (int t = threadIdx.x; t < kPlWaves * kBcCols; t += kPlThreads) sm.cnt[t] = 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPlPer; ++u)
            if (ws + u * kWave + lane < we) atomicAdd(&mine[kk[i][u] & (kBcCols - 1)], 1);
        __syncthreads();
        place_columns(sm, n, nb, b, s, e, ccp, info);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPlPer; ++u)
            if (ws + u * kWave < we) place_group(sm, mine, ws + u * kWave + lane, we, kk[i][u], vv[i][u], true, s, irow_t,
                                                 val_t);
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += kPlThreads) {
            irow_t[s + q] = sm.s_row[q];
            val_t[s + q] = sm.s_val[q];
        }
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_wccs_front(const WccsGeom& g, int n, int bw, const int* irp, const int* icol, int* table,
                             int* bcnt, WccsInfo* info, hipStream_t s) {
    hipError_t e = launch_fill_zero(info, sizeof(WccsInfo), s);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)kBcWaves * g.nwbmax * 4;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bcs_count), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bcs_count, dim3((unsigned)g.tiles), dim3(kBcThreads), lds, s, n, bw, g.nwbmax, irp, icol,
                       table, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bcs_blocks, dim3((unsigned)((g.nb + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, bw,
                       g.tiles, g.nb, g.nwbmax, table, bcnt);
    return hipGetLastError();
}

template <typename V>
static hipError_t wccs_back_t(const WccsGeom& g, int n, int bw, const int* irp, const int* icol, const void* val,
                              const int* table, const int* bstart, uint32_t* key, void* sval, int* ccp, int* irow_t,
                              void* val_t, WccsInfo* info, hipStream_t s) {
    const size_t lds = (size_t)kBcWaves * g.nwbmax * 4 + (size_t)(kBcRows + 1) * 4;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bcs_distribute<V>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bcs_distribute<V>, dim3((unsigned)g.tiles), dim3(kBcThreads), lds, s, n, bw, g.nwbmax,
                       g.wb_bits, irp, icol, (const V*)val, table, bstart, key, (V*)sval);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bcs_place<V>, dim3((unsigned)((g.nb + kPlBlocks - 1) / kPlBlocks)), dim3(kPlThreads), 0, s,
                       n, g.nb, bstart, key, (const V*)sval, ccp, irow_t, (V*)val_t, info);
    return hipGetLastError();
}

hipError_t launch_wccs_back(const WccsGeom& g, int n, int bw, int vbytes, const int* irp, const int* icol,
                            const void* val, const int* table, const int* bstart, uint32_t* key, void* sval,
                            int* ccp, int* irow_t, void* val_t, WccsInfo* info, hipStream_t s) {
    switch (vbytes) {
        case 8:
            return wccs_back_t<uint64_t>(g, n, bw, irp, icol, val, table, bstart, key, sval, ccp, irow_t, val_t,
                                         info, s);
        case 4:
            return wccs_back_t<uint32_t>(g, n, bw, irp, icol, val, table, bstart, key, sval, ccp, irow_t, val_t,
                                         info, s);
        default:
            return wccs_back_t<uint16_t>(g, n, bw, irp, icol, val, table, bstart, key, sval, ccp, irow_t, val_t,
                                         info, s);
    }
}

}  // namespace spmvat
