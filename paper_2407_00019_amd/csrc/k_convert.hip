// Reduced-precision value storage: binary64 -> binary32 / bfloat16 /
// binary16, round to nearest with ties to even, taken straight from the
// binary64 bit pattern (integer arithmetic, no intermediate binary32 step,
// so no double rounding).  Overflow gives +-inf; NaN stays a quiet NaN.
#include "common.h"
#include "kernels.h"

namespace spmvat {

// Target format: mb stored significand bits, eb exponent bits; emin/emax are
// the normal exponent range.
__device__ __forceinline__ uint32_t narrow_bits(double v, int mb, int eb, int emin, int emax) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t sign = (uint32_t)(b >> 63);
    const int e = (int)((b >> 52) & 0x7ff);
    const uint64_t m = b & ((1ull << 52) - 1);
    const uint32_t inf = ((1u << eb) - 1u) << mb;
    uint32_t out;
    if (e == 0x7ff) {
        out = m ? (inf | (1u << (mb - 1))) : inf;
    } else if (e == 0) {
        out = 0;                                   // +-0 and binary64 subnormals (< 2^-1022)
    } else {
        const int ex = e - 1023;
        const uint64_t sig = (1ull << 52) | m;     // 53-bit significand
        int shift = 52 - mb;                       // keep mb+1 bits
        if (ex < emin) shift += emin - ex;         // subnormal: fixed quantum 2^(emin-mb)
        uint64_t q;
        if (shift > 60) {
            q = 0;                                 // far below half the smallest subnormal
        } else {
            q = sig >> shift;
            const uint64_t rem = sig & ((1ull << shift) - 1);
            const uint64_t half = 1ull << (shift - 1);
            if (rem > half || (rem == half && (q & 1))) ++q;
        }
        if (ex < emin) {
            out = (uint32_t)q;                     // 2^mb here is the smallest normal: field 1
        } else {
            int ee = ex;
            if (q >> (mb + 1)) { q >>= 1; ++ee; }  // rounding carried into the exponent
            out = ee > emax ? inf : (((uint32_t)(ee - emin + 1) << mb) | ((uint32_t)q & ((1u << mb) - 1u)));
        }
    }
    return (sign << (eb + mb)) | out;
}

template <int TO>
__device__ __forceinline__ uint32_t narrow_to(double v) {
    if (TO == 1) return narrow_bits(v, 23, 8, -126, 127);
    if (TO == 2) return narrow_bits(v, 7, 8, -126, 127);
    return narrow_bits(v, 10, 5, -14, 15);
}

constexpr int kConvPer = 4;   // values per thread: two 16-byte loads, one 16- or 8-byte store

// One pass, each thread converting 4 consecutive values (the arrays are
// 16-byte aligned); the last thread takes the tail one value at a time.  A
// grid of one-shot threads streams faster than a grid-stride loop here.
template <int TO>
__global__ void __launch_bounds__(kBlock) k_convert(int64_t m, const double* __restrict__ in, void* __restrict__ out) {
    const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kConvPer;
    if (i0 >= m) return;
    if (i0 + kConvPer <= m) {
        const double2 a = *reinterpret_cast<const double2*>(in + i0);
        const double2 b = *reinterpret_cast<const double2*>(in + i0 + 2);
        const uint32_t o0 = narrow_to<TO>(a.x), o1 = narrow_to<TO>(a.y), o2 = narrow_to<TO>(b.x), o3 = narrow_to<TO>(b.y);
        if (TO == 1) *reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(out) + i0) = make_uint4(o0, o1, o2, o3);
        else *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(out) + i0) = make_uint2(o0 | (o1 << 16), o2 | (o3 << 16));
        return;
    }
    for (int64_t i = i0; i < m; ++i) {
        const uint32_t o = narrow_to<TO>(in[i]);
        if (TO == 1) reinterpret_cast<uint32_t*>(out)[i] = o;
        else reinterpret_cast<uint16_t*>(out)[i] = (uint16_t)o;
    }
}

hipError_t launch_convert(int to, int64_t m, const double* in, void* out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int64_t per_block = (int64_t)kBlock * kConvPer;
    const dim3 grid((unsigned)((m + per_block - 1) / per_block));
    if (to == 1) hipLaunchKernelGGL(k_convert<1>, grid, dim3(kBlock), 0, s, m, in, out);
    else if (to == 2) hipLaunchKernelGGL(k_convert<2>, grid, dim3(kBlock), 0, s, m, in, out);
    else hipLaunchKernelGGL(k_convert<3>, grid, dim3(kBlock), 0, s, m, in, out);
    return hipGetLastError();
}

}  // namespace spmvat
