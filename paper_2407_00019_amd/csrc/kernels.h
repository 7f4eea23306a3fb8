// Host-side launchers of the spmvat kernels (internal to libspmvat.so).
// Each enqueues on `s` and returns the launch's hipError_t.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace spmvat {

// Output of the row-statistics kernel (one per plan, in plan workspace).
struct RowStats {
    unsigned long long s1, s2;   // sum l_i, sum l_i^2
    int32_t max_len;
    uint32_t min_len;            // starts at 0xffffffff
    uint32_t flags;              // 1 irp[0]!=0, 2 irp[n]!=nnz, 4 decreasing irp, 8 column out of range
    int32_t max_band;            // max |i - j| over every stored entry
};

// Column-count summary written by the CCS scan (read back by the host).
struct ColSummary {
    int32_t total;        // sum of counts (= nnz)
    int32_t max_len;      // longest column
    int32_t n_mid;        // columns with kSortSmall < len <= kSortMid
    int32_t n_long;       // columns with len > kSortMid
};

constexpr int kSortSmall = 512;   // ranked by a workgroup in LDS
constexpr int kSortMid = 8192;    // sorted by one workgroup in LDS
constexpr int kScanTile = 4096;   // counts per workgroup in the column scan

// Carry of the COO-Row segmented reduction: one per workgroup tile.
template <typename X> struct Carry { int32_t row; int32_t pad; X val; };
constexpr int kCooPerThread = 8;
constexpr int kCooTile = 256 * kCooPerThread;

// ---- statistics
size_t row_stats_partial_count();
// The result goes to out (device) and, when host_out is not null, to that
// pinned host address as well.
hipError_t launch_row_stats(int n, int64_t nnz, const int* irp, const int* icol, RowStats* partial,
                            RowStats* out, RowStats* host_out, hipStream_t s);

// ---- transformations
hipError_t launch_expand_ptr(int n, const int* ptr, int* out, hipStream_t s);
// Column counts (added into cnt); bw = the matrix bandwidth from the row
// statistics selects the LDS-privatised kernel when its window fits.
hipError_t launch_col_count(int n, int bw, const int* irp, const int* icol, int* cnt, hipStream_t s);
// mid_list = long_list = nullptr: no lists of long columns (n_mid, n_long stay 0)
hipError_t launch_col_scan(int n, const int* cnt, int* ccp, int* cursor, int* bsum,
                           int* mid_list, int* long_list, ColSummary* sum, hipStream_t s);
size_t col_scan_bsum_count(int n);   // per array; the scan needs two (sums, maxima)
// ext[2i], ext[2i+1] = ccp[list[i]], ccp[list[i] + 1]
hipError_t launch_col_extents(int count, const int* list, const int* ccp, int* ext, hipStream_t s);
hipError_t launch_ccs_scatter(int n, int bw, const int* irp, const int* icol, int* cursor,
                              unsigned long long* keys, hipStream_t s);
hipError_t launch_ccs_sort_small(int n, const int* ccp, unsigned long long* keys, const void* val,
                                 int vbytes, int* irow_t, void* val_t, hipStream_t s);
hipError_t launch_ccs_sort_mid(int count, const int* list, const int* ccp, unsigned long long* keys,
                               const void* val, int vbytes, int* irow_t, void* val_t, hipStream_t s);
// Sorts one long column [start, start+len) of keys, using tmp (len keys) as
// ping-pong space, and writes irow_t / val_t for it.  tmp = nullptr: rank
// across sorted chunks instead (no scratch, slower).
hipError_t launch_ccs_sort_long(int start, int len, unsigned long long* keys, unsigned long long* tmp,
                                const void* val, int vbytes, int* irow_t, void* val_t, hipStream_t s);
// The LDS-privatised counts and scatter apply (the window of a tile's
// columns fits in LDS) for matrix bandwidth bw.
bool ccs_privatised(int bw);
// Two-level stable counting sort (column blocks of 2^kCcsBlockBits columns,
// keys packing the column within the block above a kCcsRowBits-bit row):
// the CCS path for scattered columns with n <= 2^kCcsRowBits.
constexpr int kCcsBlockBits = 10;
constexpr int kCcsRowBits = 22;
struct CcsGeom {
    int nb, nb_bits;     // column blocks, bits of a block index
    int rows, tiles;     // rows per level-1 tile, tiles
    int waves;           // waves per level-1 workgroup
    int64_t table;       // tiles x blocks counts
    int64_t chunks;      // 4096-count chunks of the table scan
};
CcsGeom ccs_geom(int n);
hipError_t launch_ccs_bucketed(const CcsGeom& g, int n, int64_t nnz, const int* irp, const int* icol,
                               const void* val, int vbytes, int* table, int* csum, uint32_t* bkey, void* bval,
                               int* ccp, int* irow_t, void* val_t, ColSummary* sum, hipStream_t s);
// Radix CRS -> CCS: a least-significant-digit sort of the entries by column,
// 8 bits per pass, for matrices whose columns are scattered.  Buffers of
// the workspace: two sets of (column, row, value) arrays of nnz entries,
// the (digit, tile) count table and its scan's chunk sums.
struct RadixGeom {
    int passes;          // 8-bit digits of the largest column index
    int64_t tiles;       // 2048-entry tiles
    int64_t table;       // 256 x tiles counts
    int64_t chunks;      // 4096-count chunks of the table scan
};
RadixGeom radix_geom(int n, int64_t nnz);
struct RadixWs {
    int *xcol, *xrow, *ycol, *yrow;
    void *xval, *yval;
    int* table;
    int* csum;
};
hipError_t launch_ccs_radix(const RadixGeom& g, int n, int64_t nnz, const int* irp, const int* icol,
                            const void* val, int vbytes, const RadixWs& ws, int* ccp, int* irow_t, void* val_t,
                            ColSummary* sum, hipStream_t s);
// Banded CRS -> CCS for matrices of limited bandwidth (a two-level stable
// counting sort with coalesced stores): per-(tile, wave) counts over the
// 128-column blocks of each row tile's column window, a per-block walk over
// the tiles giving every stretch its start, the ordered distribution to the
// blocks, then a stable per-block placement by column staged in LDS.
struct WccsGeom {
    int rows, tiles;       // rows per tile, tiles
    int nb;                // 64-column blocks
    int nwbmax;            // window blocks of the widest window
    int wb_bits;           // bits of a window block index
    int64_t stretches;     // wave stretches: tiles x waves
    int64_t table;         // table counts: stretches x nwbmax
    bool usable;           // the window fits the kernels' LDS and n fits the packed key
};
constexpr uint32_t kWccsOutside = 1;    // an entry outside its tile's window (CRS changed since the plan)
struct WccsInfo {
    uint32_t flags;
    int32_t kmax;          // the longest column
};
WccsGeom wccs_geom(int n, int bw, int max_row);
// counts and the per-block walk; bcnt[b] receives the length of block b,
// sflag[stretches] the per-stretch flags of entries outside the window (info
// is cleared, then flagged, on the way)
hipError_t launch_wccs_front(const WccsGeom& g, int n, int bw, const int* irp, const int* icol, int* table,
                             int* bcnt, int* sflag, WccsInfo* info, hipStream_t s);
// bstart[nb + 1] = exclusive scan of bcnt, sum->total = the last start; bsum
// is the shared scan's scratch (col_scan_bsum_count(nb) x 2 ints) for block
// counts too many for one workgroup
hipError_t launch_wccs_scan(const WccsGeom& g, int* bcnt, int* bstart, int* bsum, ColSummary* sum, hipStream_t s);
// distribution (key[nnz], sval[nnz] staging) and placement; bstart[nb + 1]
// holds the scanned block lengths
hipError_t launch_wccs_back(const WccsGeom& g, int n, int bw, int vbytes, const int* irp, const int* icol,
                            const void* val, const int* table, const int* bstart, uint32_t* key, void* sval,
                            int* ccp, int* irow_t, void* val_t, WccsInfo* info, hipStream_t s);
hipError_t launch_ell_pack(int n, int width, const int* ptr, const int* idx, const void* val,
                           int vbytes, void* ell_val, int* ell_idx, hipStream_t s);

// ---- SpMV (dtype: 0 F64, 1 F32, 2 BF16, 3 F16).  The CRS and ELL-Row
// kernels store alpha * (A x)_i; spmv_exec passes alpha = 1, the server
// passes the power-of-two scale of a job's chain (exact either way).
hipError_t launch_fill_zero(void* y, int64_t bytes, hipStream_t s);
// out = 2^-shift in (dtype 0: binary64, else binary32)
hipError_t launch_scale_pow2(int dtype, int n, int shift, const void* in, void* out, hipStream_t s);
hipError_t launch_spmv_crs_scalar(int dtype, int n, const int* irp, const int* icol, const void* val,
                                  const void* x, void* y, double alpha, hipStream_t s);
int crs_stream_lanes(int n, int64_t nnz);   // lanes per row the stream kernel uses
hipError_t launch_spmv_crs_stream(int dtype, int n, int64_t nnz, const int* irp, const int* icol, const void* val,
                                  const void* x, void* y, double alpha, hipStream_t s);
hipError_t launch_spmv_crs_vector(int dtype, int width, int n, const int* irp, const int* icol,
                                  const void* val, const void* x, void* y, double alpha, hipStream_t s);
int ell_row_parts(int n, int width);   // threads per row ELL-Row uses (1: Fig. 3, more: Fig. 4)
hipError_t launch_spmv_ell_row(int dtype, int n, int width, const void* ev, const int* ec,
                               const void* x, void* y, double alpha, hipStream_t s);
hipError_t launch_spmv_ell_col(int dtype, int n, int width, const void* ev, const int* er,
                               const void* x, void* y, hipStream_t s);
hipError_t launch_spmv_coo_row(int dtype, int n, int64_t nnz, const int* irow, const int* icol,
                               const void* val, const void* x, void* y, void* carries, hipStream_t s);
hipError_t launch_spmv_coo_col(int dtype, int64_t nnz, const int* jcol, const int* irow_t,
                               const void* val_t, const void* x, void* y, hipStream_t s);
// Column SpMVs with y privatised in LDS by pages of 64 rows (bw = the
// matrix bandwidth, max |i - j|).  Both clear y first.  Correct for any bw;
// they pay off when col_paged_fits(n, bw): then every ELL-Column
// workgroup's row window fits the page table.
bool col_paged_fits(int n, int bw);
hipError_t launch_spmv_ell_col_paged(int dtype, int n, int width, int bw, const void* ev, const int* er,
                                     const void* x, void* y, hipStream_t s);
hipError_t launch_spmv_coo_col_paged(int dtype, int n, int64_t nnz, int bw, const int* jcol, const int* irow_t,
                                     const void* val_t, const void* x, void* y, hipStream_t s);
size_t coo_carry_bytes(int64_t nnz);
// COO-Row SpMV with its carries in a fixed per-device array (no workspace):
// y is cleared first, then the same kernels as launch_spmv_coo_row run.
int64_t coo_row_static_max_nnz();
hipError_t launch_spmv_coo_row_static(int dtype, int n, int64_t nnz, const int* irow, const int* icol,
                                      const void* val, const void* x, void* y, hipStream_t s);

// ---- serving: one batched chain step over every running job (binary32)
constexpr int kServeCrs = 0, kServeEll = 1;
constexpr int kServeCoarseBits = 6;   // the coarse map holds the job of every 64th work item
constexpr int kServeThreads = 256;    // threads of the step kernel: an ELL-Row item is 256 rows
struct ServeStep {
    const int* a0;            // CRS: row pointers; ELL-Row: slot-major column indices
    const int* a1;            // CRS: column indices
    const float* val;         // CRS values or ELL-Row slot-major values
    const float* x;           // input of this step
    float* y;                 // output of this step
    int32_t n, kind, param;   // param: lanes per row (CRS) or the ELL width
    int32_t item0;            // first work item of the job in this step
    int32_t rows_per_item;
    float alpha;              // y = alpha A x
};
int serve_crs_lanes(int n, int64_t nnz);
hipError_t launch_serve_step(const ServeStep* jobs, int njobs, const int* coarse, int items, hipStream_t s);

// ---- value conversion (to: 1 F32, 2 BF16, 3 F16)
hipError_t launch_convert(int to, int64_t m, const double* in, void* out, hipStream_t s);

}  // namespace spmvat
