/*
 * spmvat.h -- run-time CRS transformation and auto-tuned SpMV on AMD MI355X
 * (gfx950), after Katagiri & Sato, "An Auto-tuning Method for Run-time Data
 * Transformation for Sparse Matrix-Vector Multiplication" (arXiv:2407.00019).
 *
 * Conventions for every entry point
 *  - Matrices are square, n x n (section 2.1).  Indices are 0-based int32:
 *    the paper's 1-based IRP(1)=1 ... IRP(N+1)=NNZ+1 is irp[0]=0 ...
 *    irp[n]=nnz here.  1 <= n and 0 <= nnz <= SPMV_MAX_NNZ = 2^31 - 2^20:
 *    the kernels step through entry positions in 32-bit chunks of up to a
 *    few thousand, and the 2^20 of headroom keeps every such step in range.
 *  - "device" pointers are HIP device memory of the current device; every
 *    device array must be 16-byte aligned (SPMV_E_ARG otherwise).
 *  - `stream` is a hipStream_t passed as void* (NULL: the default stream).
 *    Work is enqueued on it; unless stated, calls return before it runs.
 *  - The caller owns every device buffer.  A plan *borrows* the CRS arrays
 *    and every buffer handed to a transformation: they must stay alive and
 *    unchanged while the plan may use them.  The plan itself is host memory.
 *  - Errors are returned as spmv_status; nothing aborts, prints or throws.
 *    On an error no device work has been enqueued unless stated, and formats
 *    built earlier on the plan stay usable.
 *  - Calls on different plans may run concurrently from different host
 *    threads and streams.  Calls on one plan that overlap in time (two
 *    streams, or two host threads) race on the plan's workspace.
 *  - Floating-point inputs must be finite (0 * Inf in ELL padding is NaN).
 */
#ifndef SPMVAT_H
#define SPMVAT_H

#include <stddef.h>
#include <stdint.h>

#define SPMV_MAX_NNZ 2146435072   /* 2^31 - 2^20 */

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPMV_OK = 0,
    SPMV_E_ARG = 1,        /* bad argument: null, size, enum, alignment, short buffer */
    SPMV_E_MATRIX = 2,     /* the CRS arrays break the contract (see spmv_plan_create) */
    SPMV_E_TOO_LARGE = 3,  /* the format would exceed the plan's memory limit */
    SPMV_E_NOT_READY = 4,  /* the format, or the CCS it needs, is not built yet */
    SPMV_E_HIP = 5         /* a HIP runtime error; see spmv_plan_last_error */
} spmv_status;

/* Storage formats of section 2.1.  CRS: VAL/ICOL/IRP.  COO_ROW: CRS VAL and
 * ICOL plus IROW.  CCS: column pointers, row numbers, values (Phase I of the
 * column-wise transformation).  COO_COL: the CCS arrays plus a column index
 * per entry (Phase II).  ELL_ROW / ELL_COL: VAL(n, nz) and the index array
 * of the same shape, zero padded. */
typedef enum {
    SPMV_CRS = 0, SPMV_COO_ROW = 1, SPMV_CCS = 2,
    SPMV_COO_COL = 3, SPMV_ELL_ROW = 4, SPMV_ELL_COL = 5
} spmv_format;

/* Value storage.  F64 values take F64 x and y; F32, BF16 and F16 values take
 * F32 x and y and accumulate in F32 (reduced-precision storage, an extension
 * beyond the paper).  Index arrays are int32 in every case. */
typedef enum { SPMV_F64 = 0, SPMV_F32 = 1, SPMV_BF16 = 2, SPMV_F16 = 3 } spmv_dtype;

typedef struct spmv_plan spmv_plan;

/* Row statistics behind D_mat, Eq. (4).  l_i = irp[i+1] - irp[i] counts every
 * stored entry of row i.  sum_len and sum_len2 are exact; mu = sum_len / n;
 * sigma is the population standard deviation; d_mat = sigma / mu (0 when
 * nnz = 0), each rounded once from the exact integers: with
 * num = n*sum_len2 - sum_len^2 rounded to binary64, sigma = sqrt(num) / n and
 * d_mat = sqrt(num) / sum_len.  max_col is the longest column (the ELL-Column
 * width), -1 until csr_to_ccs has run.  bandwidth is the matrix bandwidth
 * max |i - j| over every stored entry (0 for nnz = 0): the locality feature
 * of the cost model, not part of the paper. */
typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t sum_len, sum_len2;
    int32_t max_row, min_row, max_col, bandwidth;
    double mu, sigma, d_mat;
} spmv_stats;

/* Bytes of every device array a transformation writes (index order as in
 * spmv_buffers), the scratch workspace it needs, and the ELL width. */
typedef struct {
    size_t bytes[4];
    size_t workspace;
    int32_t width;
} spmv_sizes;

/* Output arrays of a transformation and their sizes in bytes.
 *   COO_ROW: ptr[0] irow[nnz] int32
 *   CCS:     ptr[0] ccp[n+1] int32, ptr[1] irow_t[nnz] int32, ptr[2] val_t[nnz]
 *   COO_COL: ptr[0] jcol[nnz] int32 (with the CCS arrays already built)
 *   ELL_ROW: ptr[0] ell_val[width*n], ptr[1] ell_col[width*n] int32
 *   ELL_COL: ptr[0] ell_val[width*n], ptr[1] ell_row[width*n] int32
 * ELL arrays are slot-major (the paper's Fortran VAL(1:n,1:nz)): slot k of
 * line i at k*n + i. */
typedef struct {
    void *ptr[4];
    size_t bytes[4];
} spmv_buffers;

/* Auto-tuning table: the off-line phase's result (section 2.2) plus a cost
 * model for the amortised (k-aware) decision, indexed by a locality class
 * (0: bandwidth <= AT_LOCAL_BAND, the x entries a row gathers lie close to
 * it; 1: scattered) and a D_mat bucket b = the number of the edges 1/16,
 * 1/8, 1/4, 1/2, 1, 2, 4 that D_mat reaches.  Rates are algorithmic bytes
 * per second; 0 marks a missing entry. */
#define AT_DBUCKETS 8
#define AT_LOCAL_BAND 65536
/* The k-aware rule transforms only when the estimated cost with the
 * transformation, times a margin m, stays below the cost of staying in CRS:
 * a predicted gain smaller than the model's typical error is not acted on.
 * m is the table's k_margin, measured by the off-line phase on the
 * machine; AT_K_MARGIN applies when the table carries none (0). */
#define AT_K_MARGIN 1.1
typedef struct {
    double c;                                 /* R_ell threshold (the paper uses 1.0) */
    double d_star;                            /* ELL-Row when D_mat < d_star; +inf: always */
    int32_t calibrated;                       /* 1 when the cost model is filled */
    double spmv_bps[2][6][2][AT_DBUCKETS];    /* [locality][format][variant][bucket] SpMV rate */
    double trans_bps[2][6][AT_DBUCKETS];      /* [locality][format][bucket] transformation rate */
    double launch_s;                          /* fixed cost added per kernel launch */
    double k_margin;                          /* the k-aware rule's margin; 0: AT_K_MARGIN */
} at_table;

typedef struct {
    int32_t rule;          /* 0: paper rule (D_mat vs D*), 1: k-aware cost model */
    int32_t feasible_ell;  /* ELL-Row fits the plan's memory limit */
    double d_mat;
    double t_crs_hat;      /* estimated CRS SpMV seconds (best CRS variant) */
    double t_fmt_hat;      /* estimated SpMV seconds in the chosen format */
    double t_trans_hat;    /* estimated transformation seconds into it */
    double k_break_even;   /* TT / (1 - 1/SP) for the chosen format (where its cost
                            * equals CRS's, before the margin); 0 for CRS */
} at_decision;

/* ------------------------------------------------------------- planning */

/* Bytes of the per-plan device workspace for an n x n matrix with nnz
 * entries (row-statistics partials and SpMV carries). */
size_t spmv_plan_workspace_bytes(int32_t n, int64_t nnz);

/* Creates a plan over a CRS matrix (section 2.1) and computes its row
 * statistics (Eq. (4)) on the GPU.
 *   irp[n+1], icol[nnz]: device int32; val[nnz]: device, of type val_type.
 *   plan_work: device, at least spmv_plan_workspace_bytes(n, nnz) bytes,
 *     owned by the caller, used by the plan until spmv_plan_destroy.
 * The CRS contract is checked on the GPU: irp[0] = 0, irp[n] = nnz, irp
 * non-decreasing, 0 <= icol[p] < n; rows may be empty, unsorted or hold
 * duplicates.  Violations return SPMV_E_MATRIX (no plan is made).
 * Synchronises `stream` once to read the statistics back: on return they are
 * final.  The plan's memory limit for transformed formats starts at
 * 8 x the CRS bytes (spmv_plan_set_limit changes it). */
spmv_status spmv_plan_create(spmv_plan **plan, int32_t n, int64_t nnz,
                             const int32_t *irp, const int32_t *icol, const void *val,
                             spmv_dtype val_type, void *plan_work, size_t plan_work_bytes,
                             void *stream);

/* Host only.  Copies the statistics out. */
spmv_status spmv_plan_stats(const spmv_plan *p, spmv_stats *out);

/* Host only.  The plan's value storage type (the val_type it was created
 * with), which fixes the element type of x and y in spmv_exec. */
spmv_status spmv_plan_value_type(const spmv_plan *p, spmv_dtype *out);

/* Host only.  Largest number of bytes one transformed format (its output
 * arrays) may take; a transformation past it returns SPMV_E_TOO_LARGE
 * before any device work.  This is the memory guard of section 4.2, where
 * ELL overflowed memory for torso1. */
spmv_status spmv_plan_set_limit(spmv_plan *p, size_t max_format_bytes);

/* Algorithms of the CRS -> CCS transformation (Phase I of section 2.1).
 * All give the same arrays bit for bit; they differ in speed by structure.
 *   AUTO      BANDED when it applies, else RADIX (the default)
 *   SORT      column counts, a scatter of (position, row) keys through
 *             per-column cursors, then a per-column sort of the keys
 *   BUCKETED  two-level stable counting sort over all 1024-column blocks
 *             (n <= 2^22)
 *   BANDED    two-level stable counting sort over the 64-column blocks of
 *             each row tile's column window (limited bandwidth)
 *   RADIX     least-significant-digit radix sort of the entries by column,
 *             8 bits per pass, each pass a stable counting sort over 2048-
 *             entry tiles (any n; the workspace holds two copies of the
 *             entries) */
typedef enum {
    SPMV_CCS_AUTO = 0, SPMV_CCS_SORT = 1, SPMV_CCS_BUCKETED = 2, SPMV_CCS_BANDED = 3,
    SPMV_CCS_RADIX = 4
} spmv_ccs_algorithm;

/* Host only.  Selects the algorithm csr_to_ccs (and spmv_buffer_sizes for
 * CCS) uses from now on.  SPMV_E_ARG for an unknown value or one that does
 * not apply to the matrix (BUCKETED with n > 2^22; BANDED when a row
 * tile's column window is too wide or n > 2^26). */
spmv_status spmv_plan_set_ccs_algorithm(spmv_plan *p, spmv_ccs_algorithm alg);

/* Host only.  Output and workspace sizes of the transformation into `f`
 * (COO_ROW, CCS, COO_COL, ELL_ROW, ELL_COL).  ELL_COL needs csr_to_ccs to
 * have run (its width is the longest column): SPMV_E_NOT_READY before.
 * SPMV_E_TOO_LARGE when the format exceeds the plan's limit (sizes are still
 * filled in). */
spmv_status spmv_buffer_sizes(const spmv_plan *p, spmv_format f, spmv_sizes *out);

/* ------------------------------------------------------- transformations */

/* CRS -> COO (section 2.1).  column_wise = 0: COO-Row, out->ptr[0] =
 * irow[nnz] with irow[p] = the row owning position p (VAL and ICOL are the
 * CRS arrays).  column_wise = 1: COO-Column (Phase II), out->ptr[0] =
 * jcol[nnz] with jcol[q] = the column owning CCS position q; needs
 * csr_to_ccs first (SPMV_E_NOT_READY).  work: unused (may be NULL).
 * Index arrays are bit-exact with the definition. */
spmv_status csr_to_coo(spmv_plan *p, int column_wise, const spmv_buffers *out,
                       void *work, size_t work_bytes, void *stream);

/* CRS -> CCS, Phase I of section 2.1: column pointers ccp[n+1] (exclusive
 * prefix of the column counts, ccp[n] = nnz), row numbers irow_t[nnz] and
 * values val_t[nnz] in the stable order of the paper's counting sort:
 * inside a column, by row, then by position within the row.  Bit-exact and
 * deterministic.  work: device scratch of spmv_sizes.workspace bytes.
 * Out-of-place: the CRS arrays are not modified.  Synchronises `stream`
 * once (after the column count) to size the column sort and to learn the
 * longest column. */
spmv_status csr_to_ccs(spmv_plan *p, const spmv_buffers *out, void *work, size_t work_bytes,
                       void *stream);

/* In-place CRS -> CCS: Phase I of section 2.1 with its final copy-back.
 * The CCS arrays are built in `work` (as csr_to_ccs builds them, bit-exact)
 * and then copied over the CRS arrays: the column pointers (n + 1) over
 * irp, the row numbers (nnz) over icol, the values (nnz) over val.  irp,
 * icol and val must be the arrays the plan was created with (SPMV_E_ARG
 * otherwise), handed back writable.  Afterwards the plan's CCS lives in
 * those arrays and its CRS is gone: COO-Column and ELL-Column can be built
 * and run from it; CRS SpMV, COO-Row, ELL-Row conversion and another CCS
 * give SPMV_E_NOT_READY (an ELL-Row built before is its own copy and stays
 * usable).  work: device scratch of spmv_ccs_inplace_workspace_bytes, only
 * during the call.  The memory guard does not apply: the result replaces
 * the CRS arrays.  Synchronises `stream` as csr_to_ccs does. */
spmv_status spmv_ccs_inplace_workspace_bytes(const spmv_plan *p, size_t *bytes);
spmv_status csr_to_ccs_inplace(spmv_plan *p, int32_t *irp, int32_t *icol, void *val,
                               void *work, size_t work_bytes, void *stream);

/* CRS -> ELL (section 2.1).  column_wise = 0: ELL-Row from the CRS rows,
 * width = longest row.  column_wise = 1: ELL-Column from the CCS columns
 * (needs csr_to_ccs), width = longest column.  Slot k of line i sits at
 * k*n + i; padding slots hold value +0.0 (all bits zero) and the line's own
 * index i.  SPMV_E_TOO_LARGE if width*n overflows or the arrays exceed the
 * plan's limit.  work: unused. */
spmv_status csr_to_ell(spmv_plan *p, int column_wise, const spmv_buffers *out,
                       void *work, size_t work_bytes, void *stream);

/* ----------------------------------------------------------------- SpMV */

/* y = A x (overwrites y; the paper's loops accumulate into a cleared Y) in
 * format f (section 3, Figs. 1-3, and CRS itself).  x[n] and y[n] are
 * device arrays: F64 for F64 values, else F32 (accumulation in F32).
 * variant, CRS: 0 one thread per row (the plain CRS loop); 1 the
 * library's CRS kernel, currently the stream kernel; 2..7 a group of
 * 2^(variant-1) lanes per row; 8 the stream kernel (a workgroup stages the
 * products of 256/G consecutive rows in LDS and G lanes sum each row, G from
 * the mean row length and n; with G = 1 a thread sums its row in storage
 * order; the workgroup reduces rows of more than 256 entries).
 * variant, COO_COL and ELL_COL (Fig. 1's private copies of Y): 1 one atomic
 * add into y per entry; 2 a workgroup sums its entries into LDS partial
 * sums for the rows it touches (pages of 64 rows of its window of rows,
 * [first column - bandwidth, last column + bandwidth]) and adds each sum
 * into y once; 0 takes 2 when every workgroup's window fits the page table
 * (matrix bandwidth at most 32,192, or 32,576 when n is not a multiple of
 * 4), else 1.
 * COO_ROW and ELL_ROW take variant 0; ELL_ROW splits a row's slots over
 * several threads (the outer-parallel form of Fig. 4) when n is too small to
 * fill the GPU with one thread per row.
 * Determinism: CRS, COO_ROW and ELL_ROW are deterministic run to run;
 * COO_COL and ELL_COL scatter with atomics and are not.  x and y must not
 * overlap.  SPMV_E_NOT_READY when the format has not been built. */
spmv_status spmv_exec(const spmv_plan *p, spmv_format f, int variant,
                      const void *x, void *y, void *stream);

/* COO-Row SpMV that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  No plan and no workspace: the
 * per-workgroup carries of the segmented reduction live in a fixed device
 * array of 1 MiB that the library holds on every GPU it runs on until the
 * process ends.  y = A x with A in COO-Row form: irow[nnz] (non-decreasing,
 * as csr_to_coo writes it), icol[nnz], val[nnz] of type val_type, x[n] and
 * y[n] as for spmv_exec; all device arrays, 16-byte aligned.  y is cleared
 * by a kernel and then written by the same kernels as
 * spmv_exec(COO_ROW), so the result is bitwise the same.
 * Errors: SPMV_E_ARG for n < 1, nnz < 0, an unknown type, a null or
 * misaligned array; SPMV_E_TOO_LARGE for nnz > SPMV_COO_ROW_NOALLOC_MAX_NNZ
 * (nothing is enqueued in either case); SPMV_E_HIP if a launch fails.
 * Indices are not checked: every irow and icol entry must lie in [0, n).
 * Calls that overlap in time on one GPU (two streams, or two host threads)
 * share the array and race; successive calls on one stream do not. */
#define SPMV_COO_ROW_NOALLOC_MAX_NNZ 134217728   /* 65,536 workgroups of 2048 entries */
spmv_status spmv_exec_coo_row_noalloc(int32_t n, int64_t nnz, const int32_t *irow, const int32_t *icol,
                                      const void *val, spmv_dtype val_type, const void *x, void *y,
                                      void *stream);

/* ---------------------------------------------------------- auto-tuning */

/* Host only.  Off-line phase step (4) of section 2.2: from m benchmark points
 * (d[i] = D_mat, r[i] = R_ell, feasible[i] = 0 when the format did not fit in
 * memory, which drops the point), D* is the smallest D_mat among feasible
 * points with R_ell < c (+inf when there is none).  Fills c and d_star and
 * clears the cost model. */
spmv_status at_table_build(const double *d, const double *r, const int32_t *feasible,
                           int32_t m, double c, at_table *out);

/* Host only.  On-line phase of section 2.2.  k_repeats <= 0: the paper's
 * rule, ELL_ROW when D_mat < D* and ELL-Row fits the plan's limit, else
 * CRS (variant 1, the library's CRS kernel, which D* is measured against).  k_repeats > 0 and a calibrated table: the option with
 * the least estimated transformation + k_repeats SpMVs among COO_ROW and
 * ELL_ROW (when it fits), if the margin times that cost is below
 * k_repeats SpMVs of the faster CRS variant; otherwise CRS. */
spmv_status at_choose_format(const spmv_plan *p, const at_table *t, int64_t k_repeats,
                             spmv_format *fmt, int *variant, at_decision *why);

/* Host only.  The same decision from statistics alone: `st` as filled by
 * spmv_plan_stats, val_type the value storage and max_format_bytes the
 * memory limit that the ELL-Row footprint is checked against. */
spmv_status at_choose_format_stats(const spmv_stats *st, spmv_dtype val_type, size_t max_format_bytes,
                                   const at_table *t, int64_t k_repeats,
                                   spmv_format *fmt, int *variant, at_decision *why);

/* ------------------------------------------------------------ utilities */

/* Rounds m binary64 values to `to` (F32, BF16 or F16), to nearest with
 * ties to even, straight from binary64; overflow gives +-inf.  in and out
 * are device arrays. */
spmv_status spmv_convert_values(const double *in, void *out, int64_t m, spmv_dtype to,
                                void *stream);

void spmv_plan_destroy(spmv_plan *p);
const char *spmv_status_string(spmv_status s);
const char *spmv_plan_last_error(const spmv_plan *p);

/* -------------------------------------------------------------- serving
 *
 * A continuous-batching SpMV server built on the calls above: the on-line
 * auto-tuning of section 2.2 applied per request, with the transformation
 * amortised over the request's declared number of SpMVs (the discussion of
 * iteration counts after the on-line phase).  Binary32 values, x and y.
 *
 * Jobs become visible at their arrival time and wait in FIFO order.  A job
 * is admitted when one of `slots` ingest streams is free and its CRS and
 * vector footprint fits in the server's device arena (one allocation of
 * hbm_cap bytes made at creation).  The slot copies it in, computes its
 * statistics, chooses the format (policy 0 and 2: at_choose_format_stats
 * with k = the job's k, among CRS and ELL-Row; policy 1: CRS), allocates
 * the converted format only if it fits right now (else the job stays in
 * CRS) and converts; under policy 2 a converted job then gives its CRS
 * arrays back to the arena (the memory policy that the transformation's
 * extra footprint calls for), so more jobs fit at once.  Every prepared job
 * joins the running batch: each batched launch advances the chain
 *     y_1 = A x_0,  x_t = 2^-shift y_t,  y_{t+1} = A x_t   (t < k)
 * of every running job by one SpMV, each in its own format, and jobs join
 * and leave between launches; y_k is copied to y_out.  A job's result does
 * not depend on the jobs beside it.  Host arrays must stay valid until the
 * job is reported; pinned host memory lets the copies run asynchronously. */

typedef struct spmv_server spmv_server;

typedef struct {
    int32_t slots;       /* jobs being copied in and prepared at once, one HIP stream each, 1..64 */
    int32_t policy;      /* 0: per-job k-aware choice, 1: always CRS, 2: as 0, and a converted
                          *    job gives back its CRS arrays */
    size_t hbm_cap;      /* device bytes the server owns */
    at_table table;      /* auto-tuning table for policy 0 */
} spmv_server_config;

typedef struct {
    int64_t id;
    double arrival_s;          /* seconds after spmv_server_start; < 0: at submission */
    int32_t n;
    int64_t nnz;
    const int32_t *irp;        /* host, n+1 */
    const int32_t *icol;       /* host, nnz */
    const float *val;          /* host, nnz, binary32 */
    const float *x0;           /* host, n */
    int32_t k;                 /* SpMVs in the chain, >= 1 */
    int32_t shift;             /* 0..126 */
    float *y_out;              /* host, n: receives y_k */
} spmv_job;

typedef struct {
    int64_t id;
    int32_t status;            /* spmv_status of the job */
    int32_t format, variant;   /* format used (-1 if never admitted) */
    /* seconds after start: arrival; admission (CRS and vector blocks
     * allocated); ready (format built, handed to the engine); done (result
     * copied back, the job's memory given back) */
    double arrival_s, admit_s, ready_s, done_s;
    double d_mat;
    size_t device_bytes;       /* arena bytes the job held */
} spmv_job_result;

/* Creates the server on the current device (allocates hbm_cap bytes and the
 * slots' streams).  SPMV_E_TOO_LARGE if the allocation fails. */
spmv_status spmv_server_create(const spmv_server_config *cfg, spmv_server **out);
/* Starts the dispatcher and the slots' worker threads; arrival times count
 * from here. */
spmv_status spmv_server_start(spmv_server *s);
/* Queues a job (thread-safe); SPMV_E_ARG for an invalid descriptor.  A job
 * whose CRS footprint exceeds hbm_cap is reported with SPMV_E_TOO_LARGE. */
spmv_status spmv_server_submit(spmv_server *s, const spmv_job *job);
/* Blocks until every submitted job is reported, or SPMV_E_NOT_READY after
 * timeout_s seconds. */
spmv_status spmv_server_wait(spmv_server *s, double timeout_s);
/* Copies up to cap results, in completion order; returns how many. */
int32_t spmv_server_results(spmv_server *s, spmv_job_result *out, int32_t cap);
/* Stops the scheduler (jobs in flight are drained) and frees everything. */
void spmv_server_destroy(spmv_server *s);

/* Host-only offset allocator of the server's arena, exported for callers
 * that sub-allocate one device block themselves: first fit, 256-byte
 * granularity, free neighbours coalesce.  Offsets, not pointers.  A size
 * too large for the arena gets -1; spmv_arena_free takes back exactly what
 * spmv_arena_alloc gave (same offset and size) and ignores a range outside
 * the arena or overlapping free space.  Not thread-safe. */
typedef struct spmv_arena spmv_arena;
spmv_arena *spmv_arena_create(size_t bytes);
int64_t spmv_arena_alloc(spmv_arena *a, size_t bytes);      /* offset, or -1 when no block fits */
void spmv_arena_free(spmv_arena *a, int64_t off, size_t bytes);
size_t spmv_arena_free_bytes(const spmv_arena *a);
size_t spmv_arena_largest(const spmv_arena *a);
void spmv_arena_destroy(spmv_arena *a);

#ifdef __cplusplus
}
#endif
#endif /* SPMVAT_H */
