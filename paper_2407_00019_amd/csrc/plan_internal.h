// Internal view of a plan, shared by the C ABI (api.cpp) and the serving
// loop (serve.cpp).  Not installed; not part of include/spmvat.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/spmvat.h"
#include "kernels.h"

struct spmv_plan {
    int32_t n = 0;
    int64_t nnz = 0;
    spmv_dtype dt = SPMV_F64;
    const int32_t* irp = nullptr;
    const int32_t* icol = nullptr;
    const void* val = nullptr;
    char* work = nullptr;
    size_t work_bytes = 0;
    spmv_stats st{};
    size_t limit = 0;
    int ccs_alg = 0;                  // spmv_ccs_algorithm; 0 lets the structure decide
    bool crs_consumed = false;        // csr_to_ccs_inplace overwrote the CRS arrays with CCS
    // formats built so far (borrowed caller buffers; arrays may be null when nnz = 0)
    bool has_coo_row = false, has_ccs = false, has_coo_col = false;
    const int32_t* irow = nullptr;                                            // COO-Row
    const int32_t* ccp = nullptr; const int32_t* irow_t = nullptr; const void* val_t = nullptr;  // CCS
    const int32_t* jcol = nullptr;                                            // COO-Col
    int32_t ell_w = -1; const void* ell_val = nullptr; const int32_t* ell_col = nullptr;        // ELL-Row
    int32_t ellc_w = -1; const void* ellc_val = nullptr; const int32_t* ellc_row = nullptr;     // ELL-Col
    std::string err;
};


namespace spmvat {

// Validates the arguments of a plan, fills *p and enqueues the row
// statistics on s; their last kernel also writes them to *host_stats, which
// must be pinned host memory (hipHostMalloc).  No synchronisation.
spmv_status plan_begin(spmv_plan* p, int32_t n, int64_t nnz, const int32_t* irp, const int32_t* icol,
                       const void* val, spmv_dtype dt, void* work, size_t work_bytes, RowStats* host_stats,
                       hipStream_t s);

// Completes the plan from the statistics read back: SPMV_E_MATRIX when the
// CRS contract is broken, else D_mat (Eq. (4)) and the memory limit.
spmv_status plan_finish(spmv_plan* p, const RowStats& rs);

// spmv_exec with the stored result scaled: y = alpha * A x.  alpha != 1 only
// for CRS and ELL-Row (SPMV_E_ARG otherwise).
spmv_status plan_exec(const spmv_plan* p, spmv_format f, int variant, const void* x, void* y, double alpha,
                      hipStream_t s);

}  // namespace spmvat
