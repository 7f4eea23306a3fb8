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
//   count       per wave stretch (one wave per workgroup): entries per
//               window block.
//   blocks      lane j of a workgroup on block 64 g + j: a scan over the
//               tiles whose window covers the block, in tile order and wave
//               order inside a tile, turns the counts into each stretch's
//               start inside the block and sums the block's length.
//   scan        the block starts, by one workgroup (by the shared scan
//               kernels past 131,072 blocks).
//   distribute  per tile: each wave moves its stretch, in storage order, to
//               the blocks (equal blocks inside a group of 64 ranked through
//               the wave's LDS lane masks), as a packed key (row, column
//               within the block) and the value.  A block then holds its
//               entries in CRS order.  One tile's run inside a block is
//               long, so stores coalesce.
//   place       4 blocks per workgroup: column counts, the column pointer,
//               and the stable placement of each block's entries by column
//               (per-wave counts, ranks from LDS lane masks) into LDS,
//               written out in order; blocks larger than the LDS stage write
//               in place.
//
// CRS order inside each block, kept by a stable sort on the column, is the
// paper's order: rows ascending, each row's entries in storage order.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "lane_match.h"

namespace spmvat {

namespace {

constexpr int kBcBits = 6;                 // columns per block: 64
constexpr int kBcCols = 1 << kBcBits;
constexpr int kBcRows = 2048;              // rows per tile
constexpr int kBcWaves = 16;               // waves per tile (count, distribute)
constexpr int kBcThreads = kBcWaves * kWave;
constexpr int kBcUnroll = 8;               // groups of 64 entries (count: of 64 quads) loaded ahead
constexpr int kPlWaves = 8;                // place: waves per block
constexpr int kPlThreads = kPlWaves * kWave;
constexpr int kPlStageBytes = 36 * 1024;   // place: LDS stage of rows and values
constexpr int kPlBlocks = 4;               // place: blocks per workgroup
constexpr int kPlPer = 4;                  // place: entries per lane and block held in registers
constexpr int kBcMaxWindowBlocks = 1536;   // distribute LDS: 16 waves x 1536 counters = 96 KiB
constexpr int kBkWaves = 8;                // blocks kernel: waves per workgroup of 64 blocks
constexpr int kBkMaxTiles = 64;            // blocks kernel: tiles whose window can hold one of its 64 blocks

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
    g.stretches = (int64_t)g.tiles * kBcWaves;
    g.table = g.stretches * g.nwbmax;
    int bits = 1;
    while ((1 << bits) < g.nwbmax) ++bits;
    g.wb_bits = bits;
    // the packed key keeps the row in 32 - kBcBits bits
    // tiles a workgroup of the blocks kernel walks (64 blocks): bounded by
    // the window limit already, checked against its LDS table all the same
    const int64_t span = std::min<int64_t>(g.tiles, (4095 + 2 * (int64_t)std::max(bw, 0) + 2 * kBcRows - 1) / kBcRows + 2);
    g.usable = bw >= 0 && n <= (1 << (32 - kBcBits)) && g.nwbmax <= kBcMaxWindowBlocks && span <= kBkMaxTiles;
    return g;
}

// ------------------------------------------------------------------ count

__global__ void __launch_bounds__(kWave)
k_bcs_count(int n, int bw, int nwbmax, const int* __restrict__ irp, const int* __restrict__ icol,
            int* __restrict__ table, int* __restrict__ sflag, WccsInfo* __restrict__ info) {
    extern __shared__ int lds_c[];   // nwbmax
    const int tw = (int)xcd_block(blockIdx.x, gridDim.x);
    const int t = tw / kBcWaves;
    const int r0 = t * kBcRows, r1 = min(n, r0 + kBcRows);
    const int b0 = bc_lo(t, bw) >> kBcBits, b1 = (bc_hi(n, t, bw) - 1) >> kBcBits;
    const int nwb = b1 - b0 + 1;
    const int w = tw % kBcWaves, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < nwb; i += kWave) lds_c[i] = 0;
    __syncthreads();
    int ws, we;
    stretch(irp[r0], irp[r1], kBcWaves, w, ws, we);
    int* mine = lds_c;
    bool outside = false;
    // counting needs no order: a lane takes aligned quads of the stretch by
    // 16-byte loads (the head and tail entries one by one) and adds one LDS
    // atomic per run of entries of equal block it meets
    int cur = -1, cnt = 0;
    auto take = [&](int c) {
        const unsigned wb = (unsigned)((c >> kBcBits) - b0);
        if (wb >= (unsigned)nwb) { outside = true; return; }
        if ((int)wb != cur) {
            if (cnt) atomicAdd(&mine[cur], cnt);
            cur = (int)wb;
            cnt = 0;
        }
        ++cnt;
    };
    const int qa = min(we, (ws + 3) & ~3), qb = max(qa, we & ~3);
    if (lane < qa - ws) take(icol[ws + lane]);
    if (lane < we - qb) take(icol[qb + lane]);
    const int4* q4 = reinterpret_cast<const int4*>(icol + qa);
    const int nq = (qb - qa) >> 2;
    for (int base = 0; base < nq; base += kWave * kBcUnroll) {
        int4 v[kBcUnroll];
#pragma unroll
        for (int u = 0; u < kBcUnroll; ++u) {
            const int q = base + u * kWave + lane;
            v[u] = q < nq ? q4[q] : make_int4(-1, -1, -1, -1);
        }
#pragma unroll
        for (int u = 0; u < kBcUnroll; ++u) {
            if (base + u * kWave + lane >= nq) break;
            take(v[u].x); take(v[u].y); take(v[u].z); take(v[u].w);
        }
    }
    if (cnt) atomicAdd(&mine[cur], cnt);
    // every stretch writes its flag, so nothing needs clearing first; the
    // route's record is cleared here, before the blocks kernel flags it and
    // the placement raises its longest column
    const bool any_out = __ballot(outside) != 0;
    if (lane == 0) {
        sflag[(int64_t)t * kBcWaves + w] = any_out ? 1 : 0;
        if (tw == 0) { info->flags = 0; info->kmax = 0; }
    }
    __syncthreads();
    int* trow = table + ((int64_t)t * kBcWaves + w) * nwbmax;
    for (int i = threadIdx.x; i < nwb; i += kWave) trow[i] = lds_c[i];
}

// ----------------------------------------------------------------- blocks

// Tiles whose window can hold a block of [g * 64, g * 64 + 64): a range a
// little wider than needed, checked per tile.
__device__ __forceinline__ void bk_tiles(int n, int bw, int tiles, int g, int& tlo, int& thi) {
    const int64_t cf = (int64_t)g * kWave * kBcCols;
    const int64_t cl = min64((int64_t)n, cf + (int64_t)kWave * kBcCols) - 1;
    const int64_t a = cf - bw - kBcRows;
    tlo = a <= 0 ? 0 : (int)(a / kBcRows);
    thi = (int)min64((int64_t)tiles - 1, (cl + bw) / kBcRows);
}

// Lane j owns block g * 64 + j.  First the block's count in every tile
// (summed over the tile's waves), then their exclusive scan in tile order,
// then each wave stretch's start inside the block, in tile order and wave
// order inside a tile; the block starts follow by the shared scan kernels.
__global__ void __launch_bounds__(kBkWaves * kWave)
k_bcs_blocks(int n, int bw, int tiles, int nb, int nwbmax, int64_t stretches, int* __restrict__ table,
             int* __restrict__ bcnt, const int* __restrict__ sflag, WccsInfo* __restrict__ info) {
    __shared__ int tot[kBkMaxTiles][kWave];
    {
        bool out = false;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < stretches;
             i += (int64_t)gridDim.x * blockDim.x)
            out |= sflag[i] != 0;
        if (__ballot(out) != 0 && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&info->flags, kWccsOutside);
    }
    const int g = (int)xcd_block(blockIdx.x, gridDim.x);
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int b = g * kWave + lane;
    int tlo, thi;
    bk_tiles(n, bw, tiles, g, tlo, thi);
    for (int t = tlo + w; t <= thi; t += kBkWaves) {
        const int b0 = bc_lo(t, bw) >> kBcBits, b1 = (bc_hi(n, t, bw) - 1) >> kBcBits;
        int sum = 0;
        if (b < nb && b >= b0 && b <= b1) {
            const int* p = table + (int64_t)t * kBcWaves * nwbmax + (b - b0);
#pragma unroll
            for (int ww = 0; ww < kBcWaves; ++ww) sum += p[ww * nwbmax];
        }
        tot[t - tlo][lane] = sum;
    }
    __syncthreads();
    if (w == 0) {
        int run = 0;
        for (int t = tlo; t <= thi; ++t) {
            const int v = tot[t - tlo][lane];
            tot[t - tlo][lane] = run;
            run += v;
        }
        if (b < nb) bcnt[b] = run;
    }
    __syncthreads();
    for (int t = tlo + w; t <= thi; t += kBkWaves) {
        const int b0 = bc_lo(t, bw) >> kBcBits, b1 = (bc_hi(n, t, bw) - 1) >> kBcBits;
        if (b >= nb || b < b0 || b > b1) continue;
        int* p = table + (int64_t)t * kBcWaves * nwbmax + (b - b0);
        int run = tot[t - tlo][lane];
        int v[kBcWaves];
#pragma unroll
        for (int ww = 0; ww < kBcWaves; ++ww) v[ww] = p[ww * nwbmax];
#pragma unroll
        for (int ww = 0; ww < kBcWaves; ++ww) {
            p[ww * nwbmax] = run;
            run += v[ww];
        }
    }
}

// ------------------------------------------------------------------- scan

constexpr int kBsThreads = 1024;
constexpr int kBsPer = 16;                        // counts a thread takes per chunk (four 16-byte loads)
constexpr int kBsChunk = kBsThreads * kBsPer;
constexpr int kBsMax = 8 * kBsChunk;              // block counts scanned by one workgroup

// Block starts by one workgroup, a chunk of 16,384 counts at a time: each
// thread loads 16 consecutive counts, a workgroup scan of the threads' sums
// gives each its start, and the chunk's total carries into the next.
__global__ void __launch_bounds__(kBsThreads)
k_bcs_scan(int nb, const int* __restrict__ bcnt, int* __restrict__ bstart, ColSummary* __restrict__ sum) {
    __shared__ int wtot[kBsThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    int carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kBsChunk) {
        const int i0 = c0 + t * kBsPer;
        const bool whole = i0 + kBsPer <= nb;
        int v[kBsPer];
        if (whole) {
            const int4* p = reinterpret_cast<const int4*>(bcnt + i0);
#pragma unroll
            for (int q = 0; q < kBsPer / 4; ++q) {
                const int4 x = p[q];
                v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kBsPer; ++k) v[k] = i0 + k < nb ? bcnt[i0 + k] : 0;
        }
        int local = 0;
#pragma unroll
        for (int k = 0; k < kBsPer; ++k) local += v[k];
        int incl = local;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int y = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += y;
        }
        if (lane == kWave - 1) wtot[w] = incl;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int k = 0; k < kBsThreads / kWave; ++k) {
            before += k < w ? wtot[k] : 0;
            total += wtot[k];
        }
        int run = carry + before + incl - local;
#pragma unroll
        for (int k = 0; k < kBsPer; ++k) {
            const int x = v[k];
            v[k] = run;
            run += x;
        }
        if (whole) {
            int4* p = reinterpret_cast<int4*>(bstart + i0);
#pragma unroll
            for (int q = 0; q < kBsPer / 4; ++q) p[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < kBsPer; ++k)
                if (i0 + k < nb) bstart[i0 + k] = v[k];
        }
        carry += total;
        __syncthreads();   // wtot is read above before the next chunk writes it
    }
    if (t == 0) {
        bstart[nb] = carry;
        sum->total = carry;
        sum->max_len = 0;
        sum->n_mid = 0;
        sum->n_long = 0;
    }
}

// ------------------------------------------------------------- distribute

template <typename V>
__global__ void __launch_bounds__(kBcThreads)
k_bcs_distribute(int n, int bw, int nwbmax, int wb_bits, const int* __restrict__ irp, const int* __restrict__ icol,
                 const V* __restrict__ val, const int* __restrict__ table, const int* __restrict__ bstart,
                 uint32_t* __restrict__ key, V* __restrict__ sval) {
    // LDS: kBcWaves x kLaneMaskSlots lane masks, kBcWaves x nwbmax cursors,
    // kBcRows + 1 row pointers
    extern __shared__ unsigned long long lds_m[];
    int* lds_d = reinterpret_cast<int*>(lds_m + kBcWaves * kLaneMaskSlots);
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
    for (int i = threadIdx.x; i < kBcWaves * kLaneMaskSlots; i += kBcThreads) lds_m[i] = 0;
    __syncthreads();
    int ws, we;
    stretch(sp[0], sp[rows], kBcWaves, w, ws, we);
    if (ws >= we) return;
    int* cur = lds_d + w * nwbmax;
    unsigned long long* masks = lds_m + w * kLaneMaskSlots;
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
            const uint32_t kw = valid ? (uint32_t)wb : 0u;
            // equal window blocks: the low bits through the LDS lane masks,
            // the rest (two or three bits at most) by ballots
            uint64_t m = match_lds(kw & (kLaneMaskSlots - 1), valid, masks);
            if (wb_bits > kLaneMaskBits)
                m &= match_low_bits(kw >> kLaneMaskBits, wb_bits - kLaneMaskBits, __ballot(valid));
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
    unsigned long long masks[kPlWaves][kBcCols];   // per wave: lane masks of the 64 columns
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
// from the wave's LDS lane masks, slot from the wave's cursor of that column.
template <typename V>
__device__ __forceinline__ void place_group(PlaceSmem<V>& sm, int* mine, int p, int we, uint32_t k, V v, bool staged,
                                            int s, int* irow_t, V* val_t) {
    const bool valid = p < we;
    const uint32_t lc = k & (kBcCols - 1);
    const uint64_t mm = match_lds(lc, valid, sm.masks[threadIdx.x / kWave]);
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
    for (int i = threadIdx.x; i < kPlWaves * kBcCols; i += kPlThreads) (&sm.masks[0][0])[i] = 0;
    __syncthreads();
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
                             int* bcnt, int* sflag, WccsInfo* info, hipStream_t s) {
    const size_t lds = (size_t)g.nwbmax * 4;
    hipLaunchKernelGGL(k_bcs_count, dim3((unsigned)g.stretches), dim3(kWave), lds, s, n, bw, g.nwbmax, irp, icol,
                       table, sflag, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int groups = (g.nb + kWave - 1) / kWave;
    hipLaunchKernelGGL(k_bcs_blocks, dim3((unsigned)groups), dim3(kBkWaves * kWave), 0, s, n, bw, g.tiles, g.nb,
                       g.nwbmax, g.stretches, table, bcnt, sflag, info);
    return hipGetLastError();
}

hipError_t launch_wccs_scan(const WccsGeom& g, int* bcnt, int* bstart, int* bsum, ColSummary* sum, hipStream_t s) {
    if (g.nb > kBsMax) return launch_col_scan(g.nb, bcnt, bstart, bcnt, bsum, nullptr, nullptr, sum, s);
    hipLaunchKernelGGL(k_bcs_scan, dim3(1), dim3(kBsThreads), 0, s, g.nb, bcnt, bstart, sum);
    return hipGetLastError();
}

template <typename V>
static hipError_t wccs_back_t(const WccsGeom& g, int n, int bw, const int* irp, const int* icol, const void* val,
                              const int* table, const int* bstart, uint32_t* key, void* sval, int* ccp, int* irow_t,
                              void* val_t, WccsInfo* info, hipStream_t s) {
    const size_t lds = (size_t)kBcWaves * kLaneMaskSlots * 8 + (size_t)kBcWaves * g.nwbmax * 4 + (size_t)(kBcRows + 1) * 4;
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
