// Device-side helpers shared by the spmvat kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmvat {

constexpr int kBlock = 256;   // threads per workgroup: 4 waves of 64
constexpr int kWave = 64;
constexpr int kXcds = 8;      // MI355X: 8 XCDs, each with its own 4 MB L2

// Workgroups are dispatched round-robin over the XCDs (hardware block b runs
// on XCD b % 8).  Renumbering so that each XCD receives one contiguous range
// of logical blocks keeps neighbouring rows -- and the x entries they gather --
// inside one XCD's L2.  A bijection on [0, nblocks).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks) {
    uint32_t per = nblocks / kXcds, rem = nblocks % kXcds;
    uint32_t xcd = b % kXcds, idx = b / kXcds;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Value storage types.  F64 values pair with F64 x/y; the reduced formats
// pair with F32 x/y and F32 accumulation.
struct bf16_t { uint16_t bits; };
struct f16_t { uint16_t bits; };

template <typename V> struct acc_of { using type = float; };
template <> struct acc_of<double> { using type = double; };

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(bf16_t v) { return __uint_as_float((uint32_t)v.bits << 16); }
__device__ __forceinline__ float widen(f16_t v) {
    _Float16 h;
    __builtin_memcpy(&h, &v.bits, 2);
    return (float)h;
}

// Streaming loads that should not displace the x vector from the caches.
template <typename T> __device__ __forceinline__ T ld_nt(const T* p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ bf16_t ld_nt(const bf16_t* p) {
    bf16_t r;
    r.bits = __builtin_nontemporal_load(&p->bits);
    return r;
}
template <> __device__ __forceinline__ f16_t ld_nt(const f16_t* p) {
    f16_t r;
    r.bits = __builtin_nontemporal_load(&p->bits);
    return r;
}

// Two consecutive elements through one non-temporal load (p must be aligned
// to twice the element size).
template <typename T>
__device__ __forceinline__ void load2_nt(const T* p, T& a, T& b) {
    if constexpr (sizeof(T) == 8) {
        typedef unsigned long long v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
        const unsigned long long lo = v.x, hi = v.y;
        __builtin_memcpy(&a, &lo, 8);
        __builtin_memcpy(&b, &hi, 8);
    } else if constexpr (sizeof(T) == 4) {
        const unsigned long long v = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
        const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        __builtin_memcpy(&a, &lo, 4);
        __builtin_memcpy(&b, &hi, 4);
    } else {
        const uint32_t v = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
        const uint16_t lo = (uint16_t)v, hi = (uint16_t)(v >> 16);
        __builtin_memcpy(&a, &lo, 2);
        __builtin_memcpy(&b, &hi, 2);
    }
}

// Raw element types used when values are only moved (transformations).
template <int B> struct raw_of;
template <> struct raw_of<8> { using type = uint64_t; };
template <> struct raw_of<4> { using type = uint32_t; };
template <> struct raw_of<2> { using type = uint16_t; };

// Largest r in [lo, hi] with a[r] <= q, for a non-decreasing a with a[lo] <= q.
__device__ __forceinline__ int last_le(const int* a, int lo, int hi, int q) {
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Lanes of the wave whose `bits` low bits of key equal this lane's, among
// the lanes in `active`.  Every lane of the wave must call it.
__device__ __forceinline__ uint64_t match_low_bits(uint32_t key, int bits, uint64_t active) {
    uint64_t m = active;
    for (int i = 0; i < bits; ++i) {
        const uint32_t bit = (key >> i) & 1u;
        const uint64_t b = __ballot(bit);
        m &= bit ? b : ~b;
    }
    return m;
}

// Mask of the lanes below this one in its wave.
__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace spmvat
