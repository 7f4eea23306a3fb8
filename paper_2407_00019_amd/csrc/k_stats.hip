// Row statistics behind D_mat (Eq. (4)), the CRS contract check and the
// matrix bandwidth.
//
// One pass reads irp and icol once.  A workgroup takes tiles of 256 rows:
// the tile's row pointers give the exact integer moments sum l_i,
// sum l_i^2 and the extreme row lengths; the tile's column indices
// (contiguous in CRS) are staged in LDS with 16-byte loads, and every lane
// walks a contiguous run of them of equal length, tracking the row each
// entry belongs to, to check the column range and take the bandwidth
// max |i - j| (the locality feature of the cost model).  Per-workgroup
// partials go to the plan workspace and one workgroup folds them: exact
// integers, no atomics.  Bytes read: 4(n+1) + 4 nnz.
#include "common.h"
#include "kernels.h"

namespace spmvat {

constexpr int kStatsBlocks = 2048;   // workgroups of the first stage (partials in plan workspace)
constexpr int kStatsCap = 4096;      // column indices staged per chunk (17 KiB of LDS: 6 workgroups per CU)

// one pad word after every 32 staged indices: lanes walking runs of 32
// entries then read 33 words apart, in distinct LDS banks
__device__ __forceinline__ int pad32(int q) { return q + (q >> 5); }

__global__ void __launch_bounds__(kBlock)
k_row_stats(int n, int64_t nnz, const int* __restrict__ irp, const int* __restrict__ icol,
            RowStats* __restrict__ partial) {
    __shared__ RowStats sh[kBlock / kWave];
    __shared__ int sp[kBlock + 1];
    __shared__ int sc[kStatsCap + kStatsCap / 32];
    unsigned long long s1 = 0, s2 = 0;
    int mx = 0, band = 0;
    uint32_t mn = 0xffffffffu, fl = 0, bad = 0;
    const int t = threadIdx.x;
    const int tiles = (n + kBlock - 1) / kBlock;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int r0 = tile * kBlock;
        const int rows = min(kBlock, n - r0);
        __syncthreads();   // the previous tile's readers of sp are done
        for (int c = t; c <= rows; c += kBlock) sp[c] = irp[r0 + c];
        __syncthreads();
        int dec = 0;
        if (t < rows) {
            const long long l = (long long)sp[t + 1] - sp[t];
            if (l < 0) {
                dec = 1;
            } else {
                s1 += (unsigned long long)l;
                s2 += (unsigned long long)(l * l);
                mx = max(mx, (int)l);
                mn = min(mn, (uint32_t)l);
            }
        }
        if (dec) fl |= 4u;
        const int beg = sp[0], end = sp[rows];
        // a decreasing or out-of-range pointer is flagged (here or by the
        // irp[0] / irp[n] checks); the tile's entries are then not walked
        if (__syncthreads_or(dec) || beg < 0 || (int64_t)end > nnz || beg > end) continue;
        for (int c0 = beg; c0 < end; c0 += kStatsCap) {
            const int cl = min(kStatsCap, end - c0);
            // stage icol[c0, c0 + cl): aligned quads [qa, qb) by 16-byte
            // loads, the head [c0, qa) and tail [qb, c0 + cl) one by one
            const int qa = (c0 + 3) & ~3, qb = (c0 + cl) & ~3;
            if (qa < qb) {
                const int nq = (qb - qa) >> 2;
                const int4* q4 = reinterpret_cast<const int4*>(icol + qa);
#pragma unroll 4
                for (int q = t; q < nq; q += kBlock) {
                    const int4 v = q4[q];
                    const int o = qa - c0 + 4 * q;
                    sc[pad32(o)] = v.x; sc[pad32(o + 1)] = v.y; sc[pad32(o + 2)] = v.z; sc[pad32(o + 3)] = v.w;
                }
                if (t < qa - c0) sc[pad32(t)] = icol[c0 + t];
                if (t < c0 + cl - qb) sc[pad32(qb - c0 + t)] = icol[qb + t];
            } else if (t < cl) {
                sc[pad32(t)] = icol[c0 + t];
            }
            __syncthreads();
            const int per = (cl + kBlock - 1) / kBlock;
            const int lo = min(cl, t * per), hi = min(cl, lo + per);
            if (lo < hi) {
                // the row of entry c0 + lo: the last r with sp[r] <= c0 + lo
                int r = last_le(sp, 0, rows - 1, c0 + lo);
                int next = sp[r + 1];
                for (int q = lo; q < hi; ++q) {
                    while (next <= c0 + q) next = sp[++r + 1];
                    const int c = sc[pad32(q)];
                    bad |= (uint32_t)c >= (uint32_t)n;
                    const long long d = (long long)c - (r0 + r);
                    band = max(band, (int)min(d < 0 ? -d : d, (long long)INT32_MAX));
                }
            }
            __syncthreads();
        }
    }
    if (blockIdx.x == 0 && t == 0) {
        if (irp[0] != 0) fl |= 1u;
        if ((int64_t)irp[n] != nnz) fl |= 2u;
    }
    if (bad) fl |= 8u;

    // workgroup reduction: wave butterflies, then the 4 wave results in LDS
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, kWave);
        s2 += __shfl_xor(s2, off, kWave);
        mx = max(mx, __shfl_xor(mx, off, kWave));
        band = max(band, __shfl_xor(band, off, kWave));
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, kWave));
        fl |= (uint32_t)__shfl_xor((int)fl, off, kWave);
    }
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[w].s1 = s1; sh[w].s2 = s2; sh[w].max_len = mx; sh[w].min_len = mn; sh[w].flags = fl; sh[w].max_band = band;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RowStats r = sh[0];
        for (int k = 1; k < kBlock / kWave; ++k) {
            r.s1 += sh[k].s1; r.s2 += sh[k].s2;
            r.max_len = max(r.max_len, sh[k].max_len); r.min_len = min(r.min_len, sh[k].min_len);
            r.flags |= sh[k].flags; r.max_band = max(r.max_band, sh[k].max_band);
        }
        partial[blockIdx.x] = r;
    }
}

// Second stage: one workgroup folds the per-workgroup partials in a fixed
// order (exact integers, so the order does not change the result anyway).
__global__ void __launch_bounds__(kBlock)
k_row_stats_final(int nparts, const RowStats* __restrict__ partial, RowStats* __restrict__ out,
                  RowStats* __restrict__ host_out) {
    __shared__ RowStats sh[kBlock / kWave];
    unsigned long long s1 = 0, s2 = 0;
    int mx = 0, band = 0;
    uint32_t mn = 0xffffffffu, fl = 0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        const RowStats r = partial[b];
        s1 += r.s1; s2 += r.s2; mx = max(mx, r.max_len); mn = min(mn, r.min_len); fl |= r.flags;
        band = max(band, r.max_band);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, kWave);
        s2 += __shfl_xor(s2, off, kWave);
        mx = max(mx, __shfl_xor(mx, off, kWave));
        band = max(band, __shfl_xor(band, off, kWave));
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, kWave));
        fl |= (uint32_t)__shfl_xor((int)fl, off, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[w].s1 = s1; sh[w].s2 = s2; sh[w].max_len = mx; sh[w].min_len = mn; sh[w].flags = fl; sh[w].max_band = band;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RowStats r = sh[0];
        for (int k = 1; k < kBlock / kWave; ++k) {
            r.s1 += sh[k].s1; r.s2 += sh[k].s2;
            r.max_len = max(r.max_len, sh[k].max_len); r.min_len = min(r.min_len, sh[k].min_len);
            r.flags |= sh[k].flags; r.max_band = max(r.max_band, sh[k].max_band);
        }
        *out = r;
        if (host_out) *host_out = r;   // pinned host memory: read after the stream synchronises
    }
}

size_t row_stats_partial_count() { return kStatsBlocks; }

hipError_t launch_row_stats(int n, int64_t nnz, const int* irp, const int* icol, RowStats* partial,
                            RowStats* out, RowStats* host_out, hipStream_t s) {
    int64_t blocks = ((int64_t)n + kBlock - 1) / kBlock;
    if (blocks > kStatsBlocks) blocks = kStatsBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_row_stats, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, nnz, irp, icol, partial);
    hipLaunchKernelGGL(k_row_stats_final, dim3(1), dim3(kBlock), 0, s, (int)blocks, partial, out, host_out);
    return hipGetLastError();
}

}  // namespace spmvat
