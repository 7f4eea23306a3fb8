// SpMV y = A x in every format of the method (section 3 and the CRS
// baseline), templated over the value storage type V and the vector /
// accumulator type X (double for double values, float otherwise).
//
//  CRS scalar     one thread per row (the plain CRS loop).
//  CRS vector     a power-of-two lane group per row, coalesced row loads,
//                 butterfly reduction inside the group.
//  CRS stream     a workgroup takes 256/G rows; their entries, contiguous
//                 in CRS, are read coalesced in chunks and their products
//                 kept in LDS; each row is then summed by G lanes (G = 1: by
//                 its own thread in storage order), except rows of more than
//                 256 entries, which the whole workgroup reduces.  G grows
//                 with the mean row length and on small matrices.
//  ELL-Row        Fig. 3: thread per row, slot loop inside, slot-major loads
//                 coalesced across the wave; no reduction step.  Matrices
//                 with few rows and wide rows take Fig. 4's outer-parallel
//                 form instead: a row's slots split over P threads.
//  ELL-Column     thread per column, y(row) += val * x(col) with atomics.
//  COO-Row        Fig. 2's entry-chunk partition as a segmented reduction:
//                 8 consecutive entries per thread, a segmented scan across
//                 the workgroup, workgroup carries folded in by a second
//                 kernel in workgroup order -- deterministic.
//  COO-Column     Fig. 1: chunks of entries in column order; inside a
//                 chunk one lane per column, y(row) += ... with atomics.
#include <mutex>

#include "../../include/spmvat.h"
#include "common.h"
#include "kernels.h"
#include "spmv_rows.h"

namespace spmvat {

template <typename X>
__device__ __forceinline__ void atomic_add(X* p, X v) { unsafeAtomicAdd(p, v); }

// ------------------------------------------------------------- CRS

template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_crs_scalar(int n, const int* __restrict__ irp, const int* __restrict__ icol, const V* __restrict__ val,
                  const X* __restrict__ x, X* __restrict__ y, X alpha) {
    const int i = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int a = irp[i], b = irp[i + 1];
    X s = 0;
    for (int p = a; p < b; ++p) s += (X)widen(val[p]) * x[icol[p]];
    y[i] = s * alpha;
}

template <typename V, typename X, int W>
__global__ void __launch_bounds__(kBlock)
k_spmv_crs_vector(int n, const int* __restrict__ irp, const int* __restrict__ icol, const V* __restrict__ val,
                  const X* __restrict__ x, X* __restrict__ y, X alpha) {
    constexpr int kRows = kBlock / W;
    const int row = (int)xcd_block(blockIdx.x, gridDim.x) * kRows + (int)threadIdx.x / W;
    const int lane = threadIdx.x % W;
    X s = 0;
    if (row < n) {
        const int a = irp[row], b = irp[row + 1];
        for (int p = a + lane; p < b; p += W) s += (X)widen(val[p]) * x[icol[p]];
    }
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) s += __shfl_down(s, off, W);
    if (lane == 0 && row < n) y[row] = s * alpha;
}

template <typename V, typename X, int G>
__global__ void __launch_bounds__(kBlock)
k_spmv_crs_stream(int n, const int* __restrict__ irp, const int* __restrict__ icol, const V* __restrict__ val,
                  const X* __restrict__ x, X* __restrict__ y, X alpha) {
    constexpr int kRows = kBlock / G;
    __shared__ StreamSmem<X> sm;
    const int r0 = (int)xcd_block(blockIdx.x, gridDim.x) * kRows;
    crs_stream_rows<V, X, G>(r0, min(kRows, n - r0), irp, icol, val, x, y, alpha, sm);
}

// ------------------------------------------------------------- ELL

constexpr int kEllUnrolled = 32;   // binary64 ELL-Row widths with a fully unrolled kernel
constexpr int kEllMaxParts = 16;   // most threads sharing one ELL-Row row

template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_ell_row(int n, int width, const V* __restrict__ ev, const int* __restrict__ ec, const X* __restrict__ x,
               X* __restrict__ y, X alpha) {
    const int i = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    ell_row_one<V, X>(i, n, width, ev, ec, x, y, alpha);
}

// Two consecutive rows per thread: one 2-element load per slot for values
// and indices (n even keeps every k*n + i pair aligned).  W > 0 is the
// width known at compile time: the slot loop is unrolled whole, so every
// load of a thread is in flight before the first product; W = 0 takes the
// width at run time.
template <typename V, typename X, int W>
__global__ void __launch_bounds__(kBlock)
k_spmv_ell_row2(int n, int width, const V* __restrict__ ev, const int* __restrict__ ec, const X* __restrict__ x,
                X* __restrict__ y, X alpha) {
    const int i = ((int)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) * 2;
    if (i >= n) return;
    X s0 = 0, s1 = 0;
    size_t off = (size_t)i;
    auto slot = [&](size_t o) {
        V v0, v1;
        int c0, c1;
        load2_nt(&ev[o], v0, v1);
        load2_nt(&ec[o], c0, c1);
        s0 += (X)widen(v0) * x[c0];
        s1 += (X)widen(v1) * x[c1];
    };
    if constexpr (W > 0) {
#pragma unroll
        for (int k = 0; k < W; ++k, off += (size_t)n) slot(off);
    } else {
#pragma unroll 8
        for (int k = 0; k < width; ++k, off += (size_t)n) slot(off);
    }
    y[i] = s0 * alpha;
    y[i + 1] = s1 * alpha;
}

// Fig. 4's outer-parallel ELL-Row for matrices with few rows: the slots of
// a row are split over P threads (part p takes slots p, p + P, ...), each
// part sums its slots in order, and the P partial sums meet in LDS and are
// added in part order (the paper's private partial y and serial reduction,
// at the granularity of one row).  A workgroup holds 256/P rows, part-major,
// so each wave's loads cover consecutive rows of one slot plane when
// 256/P >= 64.
template <typename V, typename X, int P>
__global__ void __launch_bounds__(kBlock)
k_spmv_ell_row_split(int n, int width, const V* __restrict__ ev, const int* __restrict__ ec,
                     const X* __restrict__ x, X* __restrict__ y, X alpha) {
    constexpr int kRows = kBlock / P;
    __shared__ X part[kBlock];
    const int r = (int)threadIdx.x % kRows, p = (int)threadIdx.x / kRows;
    const int i = (int)xcd_block(blockIdx.x, gridDim.x) * kRows + r;
    X s = 0;
    if (i < n) {
        size_t off = (size_t)p * n + i;
#pragma unroll 4
        for (int k = p; k < width; k += P, off += (size_t)P * n) s += (X)widen(ld_nt(&ev[off])) * x[ld_nt(&ec[off])];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (p == 0 && i < n) {
#pragma unroll
        for (int q = 1; q < P; ++q) s += part[q * kRows + r];
        y[i] = s * alpha;
    }
}

template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_ell_col(int n, int width, const V* __restrict__ ev, const int* __restrict__ er, const X* __restrict__ x,
               X* __restrict__ y) {
    const int j = (int)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (j >= n) return;
    const X xj = x[j];
    size_t off = (size_t)j;
    for (int k = 0; k < width; ++k, off += (size_t)n) {
        const X v = (X)widen(ev[off]);
        if (v != (X)0) atomic_add(&y[er[off]], v * xj);
    }
}

// ------------------------------------------------------------- COO

// COO-Column: a workgroup takes a contiguous chunk of kCooColTile entries
// (the entry-range partition of Fig. 1), stages rows and values in LDS,
// finds where each column starts inside the chunk, and gives each lane one
// column to walk.  Entries of a column are in row order, so at every step
// the lanes of a wave add into nearby rows and the atomics coalesce; a
// column cut by the chunk boundary is simply added from both chunks.
constexpr int kCooColTile = 2048;
constexpr int kCooColPer = kCooColTile / kBlock;   // 8 entries per thread for the head scan

template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_coo_col(int64_t nnz, const int* __restrict__ jcol, const int* __restrict__ irow_t,
               const V* __restrict__ val_t, const X* __restrict__ x, X* __restrict__ y) {
    __shared__ int s_row[kCooColTile];
    __shared__ V s_val[kCooColTile];
    __shared__ int s_head[kCooColTile + 1];
    __shared__ int s_col[kCooColTile];
    __shared__ int s_w[kBlock / kWave];
    const int64_t t0 = (int64_t)blockIdx.x * kCooColTile;
    const int cnt = (int)min((int64_t)kCooColTile, nnz - t0);
    const int t = threadIdx.x;
    for (int q = t; q < cnt; q += kBlock) {
        s_row[q] = irow_t[t0 + q];
        s_val[q] = val_t[t0 + q];
    }
    // column starts inside the chunk: thread t looks at entries 8t .. 8t+7
    int prev = (t0 + t * kCooColPer > 0 && t * kCooColPer < cnt) ? jcol[t0 + t * kCooColPer - 1] : -1;
    if (t0 == 0 && t == 0) prev = -1;
    int cols[kCooColPer];
    int heads = 0;
#pragma unroll
    for (int e = 0; e < kCooColPer; ++e) {
        const int q = t * kCooColPer + e;
        cols[e] = q < cnt ? jcol[t0 + q] : -1;
        const bool h = q < cnt && (q == 0 || cols[e] != prev);
        heads += h;
        prev = q < cnt ? cols[e] : prev;
    }
    // exclusive scan of the head counts over the workgroup
    const int lane = t & (kWave - 1), w = t / kWave;
    int xs = heads;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int yv = __shfl_up(xs, off, kWave);
        if (lane >= off) xs += yv;
    }
    if (lane == kWave - 1) s_w[w] = xs;
    __syncthreads();
    int pre = 0, nh = 0;
#pragma unroll
    for (int k = 0; k < kBlock / kWave; ++k) {
        pre += k < w ? s_w[k] : 0;
        nh += s_w[k];
    }
    int pos = pre + xs - heads;
    int last = (t * kCooColPer > 0 && t * kCooColPer < cnt) ? jcol[t0 + t * kCooColPer - 1] : -1;
    if (t == 0) last = -1;
#pragma unroll
    for (int e = 0; e < kCooColPer; ++e) {
        const int q = t * kCooColPer + e;
        if (q < cnt && (q == 0 || cols[e] != last)) {
            s_head[pos] = q;
            s_col[pos] = cols[e];
            ++pos;
        }
        if (q < cnt) last = cols[e];
    }
    if (t == 0) s_head[nh] = cnt;
    __syncthreads();
    for (int h = t; h < nh; h += kBlock) {
        const X xj = x[s_col[h]];
        const int e = s_head[h + 1];
        for (int q = s_head[h]; q < e; ++q) {
            const X v = (X)widen(s_val[q]);
            atomic_add(&y[s_row[q]], v * xj);
        }
    }
}

// Eight consecutive elements through 16-byte loads (the caller guarantees
// 16-byte alignment of p).
template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ p, T (&o)[8]) {
    constexpr int nv = (int)sizeof(T) * 8 / 16;
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint4 t[nv];
#pragma unroll
    for (int k = 0; k < nv; ++k) t[k] = q[k];
    __builtin_memcpy(&o[0], &t[0], sizeof(T) * 8);
}

template <typename V, typename X>
__global__ void __launch_bounds__(kBlock)
k_spmv_coo_row(int n, int64_t nnz, const int* __restrict__ irow, const int* __restrict__ icol,
               const V* __restrict__ val, const X* __restrict__ x, X* __restrict__ y,
               Carry<X>* __restrict__ carries) {
    constexpr int E = kCooPerThread;
    __shared__ int s_first[kBlock];
    __shared__ int s_wrow[kBlock / kWave];
    __shared__ X s_wval[kBlock / kWave];

    const int64_t tile0 = (int64_t)blockIdx.x * kCooTile;
    const int64_t base = tile0 + (int64_t)threadIdx.x * E;
    int r[E];
    X pr[E];
    if (base + E <= nnz) {
        int c[E];
        V v[E];
        load8(irow + base, r);
        load8(icol + base, c);
        load8(val + base, v);
#pragma unroll
        for (int e = 0; e < E; ++e) pr[e] = (X)widen(v[e]) * x[c[e]];
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t p = base + e;
            if (p < nnz) { r[e] = irow[p]; pr[e] = (X)widen(val[p]) * x[icol[p]]; }
            else { r[e] = n; pr[e] = 0; }
        }
    }
    s_first[threadIdx.x] = r[0];

    // trailing run of this thread's entries
    X tail = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e > 0 && r[e] != r[e - 1]) tail = 0;
        tail += pr[e];
    }
    // inclusive segmented scan of (row, tail) over the wave; rows are
    // sorted, so equal rows at both ends of a range mean one run
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int srow = r[E - 1];
    X sval = tail;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int orow = __shfl_up(srow, off, kWave);
        const X oval = __shfl_up(sval, off, kWave);
        if (lane >= off && orow == srow) sval += oval;
    }
    if (lane == kWave - 1) { s_wrow[w] = srow; s_wval[w] = sval; }
    __syncthreads();
    int prow = -1;
    X pval = 0;
    for (int k = 0; k < w; ++k) {
        const int wr = s_wrow[k];
        const X wv = s_wval[k];
        if (wr == prow) pval += wv; else { prow = wr; pval = wv; }
    }
    if (prow == srow) sval += pval;
    // exclusive value = inclusive value of the previous thread
    int crow = __shfl_up(srow, 1, kWave);
    X cval = __shfl_up(sval, 1, kWave);
    if (lane == 0) { crow = prow; cval = pval; }

    X acc = (crow == r[0]) ? cval : (X)0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e > 0 && r[e] != r[e - 1]) {
            if (r[e - 1] < n) y[r[e - 1]] = acc;
            acc = 0;
        }
        acc += pr[e];
    }
    int next;
    if (threadIdx.x + 1 < kBlock) next = s_first[threadIdx.x + 1];
    else next = (tile0 + kCooTile < nnz) ? irow[tile0 + kCooTile] : -2;
    const bool cont = (next == r[E - 1]);
    if (!cont && r[E - 1] < n) y[r[E - 1]] = acc;
    if (threadIdx.x == kBlock - 1) {
        Carry<X> cr;
        cr.row = cont ? r[E - 1] : -1;
        cr.pad = 0;
        cr.val = cont ? acc : (X)0;
        carries[blockIdx.x] = cr;
    }
}

// Adds each row's carries from the workgroups it spans, in workgroup order.
template <typename X>
__global__ void __launch_bounds__(kBlock)
k_coo_fixup(int nb, const Carry<X>* __restrict__ c, X* __restrict__ y) {
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    const int r = c[b].row;
    if (r < 0 || (b > 0 && c[b - 1].row == r)) return;
    X s = c[b].val;
    for (int k = b + 1; k < nb && c[k].row == r; ++k) s += c[k].val;
    y[r] += s;
}

size_t coo_carry_bytes(int64_t nnz) {
    const int64_t nb = (nnz + kCooTile - 1) / kCooTile;
    return (size_t)(nb > 0 ? nb : 1) * sizeof(Carry<double>);
}

// x_{t+1} = 2^-shift y_t for the dependent SpMV chains of the server
// (a power-of-two scaling: exact unless the result leaves the normal range).
template <typename X>
__global__ void __launch_bounds__(kBlock) k_scale_pow2(int n, int shift, const X* __restrict__ in, X* __restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = ldexp(in[i], -shift);
}

// ---------------------------------------------------------- dispatch

__global__ void __launch_bounds__(kBlock) k_fill_zero(uint32_t* p, int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

hipError_t launch_scale_pow2(int dtype, int n, int shift, const void* in, void* out, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    if (dtype == 0)
        hipLaunchKernelGGL(k_scale_pow2<double>, dim3(blocks), dim3(kBlock), 0, s, n, shift, (const double*)in, (double*)out);
    else
        hipLaunchKernelGGL(k_scale_pow2<float>, dim3(blocks), dim3(kBlock), 0, s, n, shift, (const float*)in, (float*)out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* y, int64_t bytes, hipStream_t s) {
    const int64_t words = bytes / 4;
    int64_t blocks = (words + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint32_t*)y, words);
    return hipGetLastError();
}

static inline unsigned grid_for(int64_t items, int per_block) {
    return (unsigned)((items + per_block - 1) / per_block);
}

#define SPMV_DISPATCH(dtype, CALL)                                  \
    switch (dtype) {                                                \
        case 0: { typedef double V; typedef double X; CALL; break; } \
        case 1: { typedef float V; typedef float X; CALL; break; }   \
        case 2: { typedef bf16_t V; typedef float X; CALL; break; }  \
        default: { typedef f16_t V; typedef float X; CALL; break; }  \
    }

// Lanes per row for the stream kernel: about one per 32 entries of the mean
// row, doubled while the grid would hold fewer than 1024 workgroups and each
// lane still gets at least four entries (measured on banded and lognormal
// rows of 1e3 .. 2e6 rows and 3 .. 129 entries per row).
int crs_stream_lanes(int n, int64_t nnz) {
    const double mean = n > 0 ? (double)nnz / n : 0.0;
    int g = 1;
    while (g < 64 && 32.0 * (2 * g) <= mean) g *= 2;
    while (g < 64 && (int64_t)n * g / kBlock < 1024 && 4.0 * (2 * g) <= mean) g *= 2;
    return g;
}

hipError_t launch_spmv_crs_stream(int dtype, int n, int64_t nnz, const int* irp, const int* icol, const void* val,
                                  const void* x, void* y, double alpha, hipStream_t s) {
    const int g = crs_stream_lanes(n, nnz);
#define CRSS(G) hipLaunchKernelGGL((k_spmv_crs_stream<V, X, G>), dim3(grid_for(n, kBlock / G)), dim3(kBlock), 0, s, \
                                   n, irp, icol, (const V*)val, (const X*)x, (X*)y, (X)alpha)
    SPMV_DISPATCH(dtype, {
        switch (g) {
            case 1: CRSS(1); break;
            case 2: CRSS(2); break;
            case 4: CRSS(4); break;
            case 8: CRSS(8); break;
            case 16: CRSS(16); break;
            case 32: CRSS(32); break;
            default: CRSS(64); break;
        }
    });
#undef CRSS
    return hipGetLastError();
}

hipError_t launch_spmv_crs_scalar(int dtype, int n, const int* irp, const int* icol, const void* val,
                                  const void* x, void* y, double alpha, hipStream_t s) {
    SPMV_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_crs_scalar<V, X>), dim3(grid_for(n, kBlock)), dim3(kBlock),
                                            0, s, n, irp, icol, (const V*)val, (const X*)x, (X*)y, (X)alpha));
    return hipGetLastError();
}

template <typename V, typename X>
static void crs_vector_w(int width, int n, const int* irp, const int* icol, const void* val, const void* x,
                         void* y, double alpha, hipStream_t s) {
#define CRSV(W) hipLaunchKernelGGL((k_spmv_crs_vector<V, X, W>), dim3(grid_for(n, kBlock / W)), dim3(kBlock), 0, s, \
                                   n, irp, icol, (const V*)val, (const X*)x, (X*)y, (X)alpha)
    switch (width) {
        case 2: CRSV(2); break;
        case 4: CRSV(4); break;
        case 8: CRSV(8); break;
        case 16: CRSV(16); break;
        case 32: CRSV(32); break;
        default: CRSV(64); break;
    }
#undef CRSV
}

hipError_t launch_spmv_crs_vector(int dtype, int width, int n, const int* irp, const int* icol, const void* val,
                                  const void* x, void* y, double alpha, hipStream_t s) {
    SPMV_DISPATCH(dtype, (crs_vector_w<V, X>(width, n, irp, icol, val, x, y, alpha, s)));
    return hipGetLastError();
}

// Threads per row of ELL-Row: 1, doubled while the grid would hold fewer
// than 1024 workgroups and each thread keeps at least four slots.
int ell_row_parts(int n, int width) {
    int p = 1;
    while (p < kEllMaxParts && (int64_t)n * p / kBlock < 1024 && 4 * (2 * p) <= width) p *= 2;
    return p;
}

hipError_t launch_spmv_ell_row(int dtype, int n, int width, const void* ev, const int* ec, const void* x,
                               void* y, double alpha, hipStream_t s) {
    const int parts = ell_row_parts(n, width);
    if (parts > 1) {
#define ELLS(P) hipLaunchKernelGGL((k_spmv_ell_row_split<V, X, P>), dim3(grid_for(n, kBlock / P)), dim3(kBlock), 0, \
                                   s, n, width, (const V*)ev, ec, (const X*)x, (X*)y, (X)alpha)
        SPMV_DISPATCH(dtype, {
            switch (parts) {
                case 2: ELLS(2); break;
                case 4: ELLS(4); break;
                case 8: ELLS(8); break;
                default: ELLS(16); break;
            }
        });
#undef ELLS
        static_assert(kEllMaxParts == 16, "the switch above lists 2 .. kEllMaxParts");
    } else if (dtype == 0 && n % 2 == 0) {
        // binary64: two rows per thread measured faster; narrower values lose
        // parallelism without gaining wider loads, so they keep one row.
        // Widths up to kEllUnrolled get their own fully unrolled kernel.
        const dim3 grid(grid_for(n / 2, kBlock));
#define ELL2(W) hipLaunchKernelGGL((k_spmv_ell_row2<double, double, W>), grid, dim3(kBlock), 0, s, n, width, \
                                   (const double*)ev, ec, (const double*)x, (double*)y, alpha)
#define ELL2_CASE(W) case W: ELL2(W); break;
        switch (width) {
            ELL2_CASE(1) ELL2_CASE(2) ELL2_CASE(3) ELL2_CASE(4) ELL2_CASE(5) ELL2_CASE(6) ELL2_CASE(7) ELL2_CASE(8)
            ELL2_CASE(9) ELL2_CASE(10) ELL2_CASE(11) ELL2_CASE(12) ELL2_CASE(13) ELL2_CASE(14) ELL2_CASE(15)
            ELL2_CASE(16) ELL2_CASE(17) ELL2_CASE(18) ELL2_CASE(19) ELL2_CASE(20) ELL2_CASE(21) ELL2_CASE(22)
            ELL2_CASE(23) ELL2_CASE(24) ELL2_CASE(25) ELL2_CASE(26) ELL2_CASE(27) ELL2_CASE(28) ELL2_CASE(29)
            ELL2_CASE(30) ELL2_CASE(31) ELL2_CASE(32)
            default: ELL2(0); break;
        }
#undef ELL2_CASE
#undef ELL2
        static_assert(kEllUnrolled == 32, "the switch above lists widths 1 .. kEllUnrolled");
    } else {
        SPMV_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_ell_row<V, X>), dim3(grid_for(n, kBlock)), dim3(kBlock), 0,
                                                s, n, width, (const V*)ev, ec, (const X*)x, (X*)y, (X)alpha));
    }
    return hipGetLastError();
}

hipError_t launch_spmv_ell_col(int dtype, int n, int width, const void* ev, const int* er, const void* x,
                               void* y, hipStream_t s) {
    const int xb = dtype == 0 ? 8 : 4;
    hipError_t e = launch_fill_zero(y, (int64_t)n * xb, s);
    if (e != hipSuccess) return e;
    SPMV_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_ell_col<V, X>), dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s,
                                            n, width, (const V*)ev, er, (const X*)x, (X*)y));
    return hipGetLastError();
}

hipError_t launch_spmv_coo_col(int dtype, int64_t nnz, const int* jcol, const int* irow_t, const void* val_t,
                               const void* x, void* y, hipStream_t s) {
    const int64_t blocks = (nnz + kCooColTile - 1) / kCooColTile;
    if (blocks == 0) return hipSuccess;
    SPMV_DISPATCH(dtype, hipLaunchKernelGGL((k_spmv_coo_col<V, X>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                                            nnz, jcol, irow_t, (const V*)val_t, (const X*)x, (X*)y));
    return hipGetLastError();
}

hipError_t launch_spmv_coo_row(int dtype, int n, int64_t nnz, const int* irow, const int* icol, const void* val,
                               const void* x, void* y, void* carries, hipStream_t s) {
    const int nb = (int)((nnz + kCooTile - 1) / kCooTile);
    if (nb == 0) return hipSuccess;
    SPMV_DISPATCH(dtype, {
        hipLaunchKernelGGL((k_spmv_coo_row<V, X>), dim3(nb), dim3(kBlock), 0, s, n, nnz, irow, icol,
                           (const V*)val, (const X*)x, (X*)y, (Carry<X>*)carries);
        hipLaunchKernelGGL((k_coo_fixup<X>), dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, s, nb,
                           (const Carry<X>*)carries, (X*)y);
    });
    return hipGetLastError();
}

// ------------------------------------------ COO-Row SpMV without allocation
// The same two kernels as the plan path, with the per-workgroup carries in a
// fixed device array instead of the plan workspace.  Every GPU that runs it
// holds its own copy of the array; its address is looked up once per device
// (the array's name is not a device address in host code).

namespace {
constexpr size_t kScratchBytes = 1u << 20;   // carries of up to 65,536 workgroups
static_assert(sizeof(Carry<double>) == 16 && sizeof(Carry<float>) <= 16, "carry record size");
constexpr int64_t kScratchMaxNnz = (int64_t)(kScratchBytes / sizeof(Carry<double>)) * kCooTile;
static_assert(kScratchMaxNnz == SPMV_COO_ROW_NOALLOC_MAX_NNZ, "the header states the limit");
constexpr int kScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];

// Address of this device's copy of `scratch`, or null on failure.
void* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

int64_t coo_row_static_max_nnz() { return kScratchMaxNnz; }

hipError_t launch_spmv_coo_row_static(int dtype, int n, int64_t nnz, const int* irow, const int* icol,
                                      const void* val, const void* x, void* y, hipStream_t s) {
    void* carries = scratch_on_current_device();
    if (!carries) return hipErrorInvalidSymbol;
    // rows without entries get no store from the kernels: clear y first
    // (a fill kernel, so the call can be captured in a graph)
    hipError_t e = launch_fill_zero(y, (int64_t)n * (dtype == 0 ? 8 : 4), s);
    if (e != hipSuccess) return e;
    return launch_spmv_coo_row(dtype, n, nnz, irow, icol, val, x, y, carries, s);
}

}  // namespace spmvat
