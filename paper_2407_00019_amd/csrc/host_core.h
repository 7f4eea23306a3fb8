// Host-only parts of libspmvat: the device-memory offset allocator of the
// server, D_mat from exact row moments (Eq. (4)) and the auto-tuner's
// decision (section 2.2).  No HIP header: host_core.cpp also builds with the
// plain host compiler and its sanitizers.
#pragma once
#include <cstddef>
#include <cstdint>
#include <map>

#include "../../include/spmvat.h"

// First-fit offset allocator over [0, cap), 256-byte grain, free blocks kept
// coalesced.  Not thread-safe: the server holds its own lock around it.
struct spmv_arena {
    static constexpr size_t kGrain = 256;
    std::map<size_t, size_t> free_;   // offset -> size
    size_t cap = 0;
    size_t free_bytes = 0;

    explicit spmv_arena(size_t bytes);
    // bytes rounded up to the grain (at least one grain); 0 when that does
    // not fit in size_t
    static size_t round(size_t bytes);
    int64_t alloc(size_t bytes);            // -1 when no free block fits
    // Returns [off, off + bytes) to the free list.  The range must be one
    // that alloc() gave out (same size) and not yet released; false, and
    // no change, when it lies outside the arena or overlaps a free block.
    bool release(int64_t off, size_t bytes);
    size_t largest() const;
};

namespace spmvat {

inline int vbytes_of(spmv_dtype t) { return t == SPMV_F64 ? 8 : t == SPMV_F32 ? 4 : 2; }
inline int xbytes_of(spmv_dtype t) { return t == SPMV_F64 ? 8 : 4; }
inline bool valid_dtype(int t) { return t >= SPMV_F64 && t <= SPMV_F16; }

// Fills mu, sigma and d_mat of *st from n and the exact moments
// s1 = sum l_i and s2 = sum l_i^2 of the row lengths (Eq. (4)): with
// num = n s2 - s1^2 rounded once to binary64, sigma = sqrt(num) / n and
// D_mat = sqrt(num) / s1 (0 for an empty matrix).
void dmat_from_moments(int32_t n, uint64_t s1, uint64_t s2, spmv_stats* st);

}  // namespace spmvat
