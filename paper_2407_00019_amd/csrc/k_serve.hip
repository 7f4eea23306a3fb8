// Batched step of the serving loop: one launch advances one SpMV of the
// chain of every running job, x_{t+1} = alpha A x_t, each job in its own
// format (CRS with G lanes per row, or ELL-Row) and over its own arrays.
//
// A job's rows are cut into work items (256/G rows for CRS, 256 rows for
// ELL-Row); the items of all jobs are numbered consecutively, job after job,
// and a workgroup takes one item.  It finds its job from a coarse map (the
// job holding item 64 g, for every g) and a short walk over the jobs' first
// items.  Each row is summed by the same row body as the single-matrix
// kernels, so a job's result does not depend on what runs beside it.
#include "common.h"
#include "kernels.h"
#include "spmv_rows.h"

namespace spmvat {

__global__ void __launch_bounds__(kBlock)
k_serve_step(const ServeStep* __restrict__ jobs, int njobs, const int* __restrict__ coarse) {
    __shared__ StreamSmem<float> sm;
    const int item = (int)xcd_block(blockIdx.x, gridDim.x);
    int j = coarse[item >> kServeCoarseBits];
    while (j + 1 < njobs && jobs[j + 1].item0 <= item) ++j;
    const ServeStep d = jobs[j];
    const int b = item - d.item0;
    const int r0 = b * d.rows_per_item;
    const int rows = min(d.rows_per_item, d.n - r0);
    if (d.kind == kServeEll) {
        if ((int)threadIdx.x < rows)
            ell_row_one<float, float>(r0 + (int)threadIdx.x, d.n, d.param, d.val, d.a0, d.x, d.y, d.alpha);
        return;
    }
#define SERVE_CRS(G) crs_stream_rows<float, float, G>(r0, rows, d.a0, d.a1, d.val, d.x, d.y, d.alpha, sm)
    switch (d.param) {
        case 1: SERVE_CRS(1); break;
        case 2: SERVE_CRS(2); break;
        case 4: SERVE_CRS(4); break;
        case 8: SERVE_CRS(8); break;
        case 16: SERVE_CRS(16); break;
        case 32: SERVE_CRS(32); break;
        default: SERVE_CRS(64); break;
    }
#undef SERVE_CRS
}

int serve_crs_lanes(int n, int64_t nnz) {
    // one lane per 32 entries of the mean row (powers of two, 1 .. 64); the
    // doubling of the single-matrix rule for small grids is not needed here,
    // the batch fills the GPU
    const double mean = n > 0 ? (double)nnz / n : 0.0;
    int g = 1;
    while (g < 64 && 32.0 * (2 * g) <= mean) g *= 2;
    return g;
}

hipError_t launch_serve_step(const ServeStep* jobs, int njobs, const int* coarse, int items, hipStream_t s) {
    if (items <= 0) return hipSuccess;
    static_assert(kServeThreads == kBlock, "one thread per ELL-Row row of an item");
    hipLaunchKernelGGL(k_serve_step, dim3((unsigned)items), dim3(kBlock), 0, s, jobs, njobs, coarse);
    return hipGetLastError();
}

}  // namespace spmvat
