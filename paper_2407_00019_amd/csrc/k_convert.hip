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
__global__ void __launch_bounds__(kBlock) k_convert(int64_t m, const double* __restrict__ in, void* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const double v = in[i];
        if (TO == 1) reinterpret_cast<uint32_t*>(out)[i] = narrow_bits(v, 23, 8, -126, 127);
        else if (TO == 2) reinterpret_cast<uint16_t*>(out)[i] = (uint16_t)narrow_bits(v, 7, 8, -126, 127);
        else reinterpret_cast<uint16_t*>(out)[i] = (uint16_t)narrow_bits(v, 10, 5, -14, 15);
    }
}

hipError_t launch_convert(int to, int64_t m, const double* in, void* out, hipStream_t s) {
    int64_t blocks = (m + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    if (to == 1) hipLaunchKernelGGL(k_convert<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, m, in, out);
    else if (to == 2) hipLaunchKernelGGL(k_convert<2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, m, in, out);
    else hipLaunchKernelGGL(k_convert<3>, dim3((unsigned)blocks), dim3(kBlock), 0, s, m, in, out);
    return hipGetLastError();
}

}  // namespace spmvat
