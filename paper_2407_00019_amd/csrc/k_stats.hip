// Row statistics behind D_mat (Eq. (4)) and the CRS contract check.
//
// One pass over irp gives the exact integer moments sum l_i, sum l_i^2 and
// the extreme row lengths; a second grid-stride pass over icol checks the
// column range.  Per-workgroup partials go to the plan workspace and one
// workgroup folds them: exact integers, no atomics.  Bytes read:
// 4(n+1) + 4 nnz.
#include "common.h"
#include "kernels.h"

namespace spmvat {

constexpr int kStatsBlocks = 1024;   // workgroups of the first stage (partials in plan workspace)

__global__ void __launch_bounds__(kBlock)
k_row_stats(int n, int64_t nnz, const int* __restrict__ irp, const int* __restrict__ icol,
            RowStats* __restrict__ partial) {
    __shared__ RowStats sh[kBlock / kWave];
    unsigned long long s1 = 0, s2 = 0;
    int mx = 0;
    uint32_t mn = 0xffffffffu, fl = 0;
    const int tid = blockIdx.x * kBlock + threadIdx.x;
    const int stride = gridDim.x * kBlock;
    for (int i = tid; i < n; i += stride) {
        const int a = irp[i], b = irp[i + 1];
        const long long l = (long long)b - a;
        if (l < 0) { fl |= 4u; continue; }
        s1 += (unsigned long long)l;
        s2 += (unsigned long long)(l * l);
        mx = max(mx, (int)l);
        mn = min(mn, (uint32_t)l);
    }
    if (tid == 0) {
        if (irp[0] != 0) fl |= 1u;
        if ((int64_t)irp[n] != nnz) fl |= 2u;
    }
    // column range, 4 indices per load
    const int64_t nv = nnz >> 2;
    const int4* ic4 = reinterpret_cast<const int4*>(icol);
    uint32_t bad = 0;
    for (int64_t q = tid; q < nv; q += stride) {
        const int4 c = ic4[q];
        bad |= ((uint32_t)c.x >= (uint32_t)n) | ((uint32_t)c.y >= (uint32_t)n) |
               ((uint32_t)c.z >= (uint32_t)n) | ((uint32_t)c.w >= (uint32_t)n);
    }
    for (int64_t p = (nv << 2) + tid; p < nnz; p += stride) bad |= (uint32_t)icol[p] >= (uint32_t)n;
    if (bad) fl |= 8u;

    // workgroup reduction: wave butterflies, then the 4 wave results in LDS
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, kWave);
        s2 += __shfl_xor(s2, off, kWave);
        mx = max(mx, __shfl_xor(mx, off, kWave));
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, kWave));
        fl |= (uint32_t)__shfl_xor((int)fl, off, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[w].s1 = s1; sh[w].s2 = s2; sh[w].max_len = mx; sh[w].min_len = mn; sh[w].flags = fl; sh[w].pad = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RowStats r = sh[0];
        for (int k = 1; k < kBlock / kWave; ++k) {
            r.s1 += sh[k].s1; r.s2 += sh[k].s2;
            r.max_len = max(r.max_len, sh[k].max_len); r.min_len = min(r.min_len, sh[k].min_len);
            r.flags |= sh[k].flags;
        }
        partial[blockIdx.x] = r;
    }
}

// Second stage: one workgroup folds the per-workgroup partials in a fixed
// order (exact integers, so the order does not change the result anyway).
__global__ void __launch_bounds__(kBlock)
k_row_stats_final(int nparts, const RowStats* __restrict__ partial, RowStats* __restrict__ out) {
    __shared__ RowStats sh[kBlock / kWave];
    unsigned long long s1 = 0, s2 = 0;
    int mx = 0;
    uint32_t mn = 0xffffffffu, fl = 0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        const RowStats r = partial[b];
        s1 += r.s1; s2 += r.s2; mx = max(mx, r.max_len); mn = min(mn, r.min_len); fl |= r.flags;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, kWave);
        s2 += __shfl_xor(s2, off, kWave);
        mx = max(mx, __shfl_xor(mx, off, kWave));
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, kWave));
        fl |= (uint32_t)__shfl_xor((int)fl, off, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sh[w].s1 = s1; sh[w].s2 = s2; sh[w].max_len = mx; sh[w].min_len = mn; sh[w].flags = fl; sh[w].pad = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        RowStats r = sh[0];
        for (int k = 1; k < kBlock / kWave; ++k) {
            r.s1 += sh[k].s1; r.s2 += sh[k].s2;
            r.max_len = max(r.max_len, sh[k].max_len); r.min_len = min(r.min_len, sh[k].min_len);
            r.flags |= sh[k].flags;
        }
        *out = r;
    }
}

size_t row_stats_partial_count() { return kStatsBlocks; }

hipError_t launch_row_stats(int n, int64_t nnz, const int* irp, const int* icol, RowStats* partial,
                            RowStats* out, hipStream_t s) {
    const int64_t work = n > (nnz >> 2) ? n : (nnz >> 2);
    int64_t blocks = (work + kBlock - 1) / kBlock;
    if (blocks > kStatsBlocks) blocks = kStatsBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_row_stats, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, nnz, irp, icol, partial);
    hipLaunchKernelGGL(k_row_stats_final, dim3(1), dim3(kBlock), 0, s, (int)blocks, partial, out);
    return hipGetLastError();
}

}  // namespace spmvat
