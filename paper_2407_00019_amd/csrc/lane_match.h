// Ranking equal keys inside a wave through a table of lane masks in LDS.
#pragma once
#include "common.h"

namespace spmvat {

constexpr int kLaneMaskBits = 8;                     // key bits a table of lane masks covers
constexpr int kLaneMaskSlots = 1 << kLaneMaskBits;   // its slots, one per key

// Lanes among `valid` whose key equals this lane's (key < the table's
// slots), from a per-wave table of 64-bit lane masks in LDS that is all
// zero before and after the call: each lane ORs its bit into its key's
// mask, reads the mask back and clears it.  An OR does not depend on the
// order in which the lanes' updates land, and a wave's LDS operations run in
// order, so the read sees the bit of every lane with that key.  Three LDS
// operations stand in for one ballot per key bit (each ballot costs several
// wave-wide vector instructions).  Every lane of the wave must call it.
__device__ __forceinline__ uint64_t match_lds(uint32_t key, bool valid, unsigned long long* masks) {
    const int lane = threadIdx.x & (kWave - 1);
    if (valid) __hip_atomic_fetch_or(&masks[key], 1ull << lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_wave_barrier();
    uint64_t mm = 0;
    if (valid) mm = __hip_atomic_load(&masks[key], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_wave_barrier();
    if (valid) __hip_atomic_store(&masks[key], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __builtin_amdgcn_wave_barrier();
    return mm;
}

}  // namespace spmvat
