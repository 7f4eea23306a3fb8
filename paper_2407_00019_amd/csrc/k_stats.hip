// Row statistics behind D_mat (Eq. (4)) and the CRS contract check.
//
// One pass over irp gives the exact integer moments sum l_i, sum l_i^2 and
// the extreme row lengths; a second grid-stride pass over icol checks the
// column range.  Per-workgroup partials are merged with integer atomics, so
// the result is exact and independent of scheduling.  Bytes read:
// 4(n+1) + 4 nnz.
#include "common.h"
#include "kernels.h"

namespace spmvat {

__global__ void __launch_bounds__(kBlock)
k_row_stats(int n, int64_t nnz, const int* __restrict__ irp, const int* __restrict__ icol,
            RowStats* __restrict__ out) {
    unsigned long long s1 = 0, s2 = 0;
    int mx = 0;
    uint32_t mn = 0xffffffffu, fl = 0;
    const int tid = blockIdx.x * kBlock + threadIdx.x;
    const int stride = gridDim.x * kBlock;
    for (int i = tid; i < n; i += stride) {
        int a = irp[i], b = irp[i + 1];
        long long l = (long long)b - a;
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
    for (int64_t q = tid; q < nv; q += stride) {
        int4 c = ic4[q];
        bool bad = (uint32_t)c.x >= (uint32_t)n || (uint32_t)c.y >= (uint32_t)n ||
                   (uint32_t)c.z >= (uint32_t)n || (uint32_t)c.w >= (uint32_t)n;
        if (bad) fl |= 8u;
    }
    for (int64_t p = (nv << 2) + tid; p < nnz; p += stride)
        if ((uint32_t)icol[p] >= (uint32_t)n) fl |= 8u;

    // workgroup reduction: wave butterflies, then one lane per wave
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, kWave);
        s2 += __shfl_xor(s2, off, kWave);
        mx = max(mx, __shfl_xor(mx, off, kWave));
        mn = min(mn, (uint32_t)__shfl_xor((int)mn, off, kWave));
        fl |= (uint32_t)__shfl_xor((int)fl, off, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (s1) atomicAdd(&out->s1, s1);
        if (s2) atomicAdd(&out->s2, s2);
        atomicMax(&out->max_len, mx);
        atomicMin(&out->min_len, mn);
        if (fl) atomicOr(&out->flags, fl);
    }
}

hipError_t launch_row_stats(int n, int64_t nnz, const int* irp, const int* icol, RowStats* out,
                            hipStream_t s) {
    hipError_t e = hipMemsetAsync(out, 0, sizeof(RowStats), s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(&out->min_len, 0xff, sizeof(uint32_t), s);
    if (e != hipSuccess) return e;
    int64_t work = n > (nnz >> 2) ? n : (nnz >> 2);
    int64_t blocks = (work + kBlock - 1) / kBlock;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_row_stats, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, nnz, irp, icol, out);
    return hipGetLastError();
}

}  // namespace spmvat
