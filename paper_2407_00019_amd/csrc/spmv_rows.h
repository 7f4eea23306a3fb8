// Row bodies shared by the single-matrix SpMV kernels and the serving
// loop's batched step kernel, so that a row is summed the same way in both.
#pragma once
#include "common.h"

namespace spmvat {

constexpr int kStreamCap = 2048;   // products staged in LDS per chunk
constexpr int kStreamLong = 256;   // rows longer than this are summed by the whole workgroup

// LDS of the stream CRS body.
template <typename X>
struct StreamSmem {
    X prod[kStreamCap];
    int sp[kBlock + 1];
    unsigned long long s_long[kBlock / kWave];
    X s_red[kBlock / kWave];
};

// Stream CRS: G lanes per row, rows r0 .. r0 + rows - 1 (rows <= 256/G) by
// one workgroup.  The rows' entries, contiguous in CRS, are read coalesced
// in chunks and their products kept in LDS; the lanes of a row take its
// staged products in a stride of G (storage order when G = 1, four LDS reads
// in flight ahead of the adds) and meet in a butterfly at the end; rows of
// more than 256 entries are summed by the whole workgroup.  Stores
// alpha * (A x)_i.  Every thread of the workgroup must call it.
template <typename V, typename X, int G>
__device__ __forceinline__ void crs_stream_rows(int r0, int rows, const int* __restrict__ irp,
                                                const int* __restrict__ icol, const V* __restrict__ val,
                                                const X* __restrict__ x, X* __restrict__ y, X alpha,
                                                StreamSmem<X>& sm) {
    X* prod = sm.prod;
    int* sp = sm.sp;
    unsigned long long* s_long = sm.s_long;
    X* s_red = sm.s_red;
    const int t = threadIdx.x;
    for (int c = t; c <= rows; c += kBlock) sp[c] = irp[r0 + c];
    __syncthreads();
    const int end = sp[rows];
    const int row = t / G, lane = t % G;
    const int a = row < rows ? sp[row] : end, b = row < rows ? sp[row + 1] : end;
    const bool lng = (b - a) > kStreamLong;
    // long rows as a bit mask indexed by row (thread t tests row t)
    const bool lt = t < rows && (sp[t + 1] - sp[t]) > kStreamLong;
    const unsigned long long m = __ballot(lt);
    if ((t & (kWave - 1)) == 0) s_long[t / kWave] = m;
    __syncthreads();
    bool any_long = false;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) any_long |= s_long[w] != 0;
    X s = 0;
    for (int c0 = sp[0]; c0 < end; c0 += kStreamCap) {
        const int cl = min(kStreamCap, end - c0);
#pragma unroll 4
        for (int q = t; q < cl; q += kBlock)
            prod[q] = (X)widen(ld_nt(&val[c0 + q])) * x[ld_nt(&icol[c0 + q])];
        __syncthreads();
        if (!lng) {
            const int lo = max(a, c0) - c0, hi = min(b, c0 + cl) - c0;
            int p = lo + lane;
            for (; p + 3 * G < hi; p += 4 * G) {
                const X q0 = prod[p], q1 = prod[p + G], q2 = prod[p + 2 * G], q3 = prod[p + 3 * G];
                s += q0; s += q1; s += q2; s += q3;
            }
            for (; p < hi; p += G) s += prod[p];
        }
        if (any_long) {
            // each long row in turn: the workgroup sums its part of the chunk
            for (int w = 0; w < kBlock / kWave; ++w) {
                unsigned long long bits = s_long[w];
                while (bits) {
                    const int r = w * kWave + __ffsll((long long)bits) - 1;
                    bits &= bits - 1;
                    const int lo = max(sp[r], c0) - c0, hi = min(sp[r + 1], c0 + cl) - c0;
                    if (lo >= hi) continue;
                    X part = 0;
                    for (int q = lo + t; q < hi; q += kBlock) part += prod[q];
#pragma unroll
                    for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, kWave);
                    if ((t & (kWave - 1)) == 0) s_red[t / kWave] = part;
                    __syncthreads();
                    if (t == r * G) {
                        X tot = 0;
#pragma unroll
                        for (int k2 = 0; k2 < kBlock / kWave; ++k2) tot += s_red[k2];
                        s += tot;
                    }
                    __syncthreads();
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
    if (lane == 0 && row < rows) y[r0 + row] = s * alpha;
}

// ELL-Row, Fig. 3: row i sums its slots in order (slot-major layout).
template <typename V, typename X>
__device__ __forceinline__ void ell_row_one(int i, int n, int width, const V* __restrict__ ev,
                                            const int* __restrict__ ec, const X* __restrict__ x,
                                            X* __restrict__ y, X alpha) {
    X s = 0;
    size_t off = (size_t)i;
#pragma unroll 8
    for (int k = 0; k < width; ++k, off += (size_t)n)
        s += (X)widen(ld_nt(&ev[off])) * x[ld_nt(&ec[off])];
    y[i] = s * alpha;
}

}  // namespace spmvat
