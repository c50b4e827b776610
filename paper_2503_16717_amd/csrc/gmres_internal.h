// Internal declarations of the s-step GMRES kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sko_internal.h"

namespace sko {

// CSR operand: structure + FP64 values of A (explicit residual) and the values used by
// the matrix-powers kernel (A D^{-1} in double or float, or A itself).
struct CsrView {
    int64_t n;
    int64_t nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* val;     // A, double
    const void* val_op;    // MPK operator values (double or float)
};

// y = A x, or with a Newton step (na != null) y = A x - (*na) x + (*nb) z (na, nb: device
// scalars; z: the basis vector before x, read only where *nb != 0).
hipError_t launch_spmv(const CsrView& A, bool f32, const void* x, void* y, int grid_cap, hipStream_t st,
                       const double* na = nullptr, const double* nb = nullptr, const void* z = nullptr);
// Mixed precision: one matrix-powers step of the FP64 panel (FP32 operator values, FP64
// vectors), and the widening copy of an FP32 basis column into the panel.
hipError_t launch_spmv_panel(const CsrView& A, const double* x, double* y, int grid_cap, hipStream_t st,
                             const double* na = nullptr, const double* nb = nullptr, const double* z = nullptr);
hipError_t launch_widen(int64_t n, const float* x, double* y, int grid_cap, hipStream_t st);
int residual_grid(int64_t n, int grid_cap);
hipError_t launch_residual(const CsrView& A, const double* x, const double* b, bool f32, void* r, double* partials,
                           int grid, hipStream_t st);
hipError_t launch_update(int64_t n, bool f32, const void* Q, int64_t ldq, int k, const double* y,
                         const double* dinv, double* x, hipStream_t st);
hipError_t launch_csr_check(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind, int* bad,
                            hipStream_t st);
hipError_t launch_jacobi_setup(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                               const double* val, double* dinv, int* status, hipStream_t st);
hipError_t launch_scale_values(int64_t nnz, const int32_t* colind, const double* val, const double* dinv, bool f32,
                               void* out, hipStream_t st);

enum GmOp : int {
    GM_INIT = 0,      // T_in = T_out = 0, g = beta e_1
    GM_BLOCK = 1,     // rewrite the boundary vector kk, store an s-step block, optional LSQ
    GM_BIGCLOSE = 2,  // express the closed big panel in the final basis, then LSQ
};

struct GmSmallArgs {
    int op;
    int m, s;
    int kk;            // GM_BLOCK: basis index of the block's start vector
    int k0;            // two-stage: first column of the current big panel
    int two_stage;
    int do_lsq;
    int Wb, kend;      // GM_BIGCLOSE: big-panel width and the basis size after it
    double* Tin;       // (m+1) x m
    double* Tout;      // (m+1) x m
    double* g;         // m+1
    double* gw;        // m+1 scratch
    double* H;         // (m+1) x m scratch
    double* y;         // m
    double* res;       // 1: implicit residual norm
    const double* beta;  // GM_INIT
    double* coef;      // (m+1) x (s+1) block coefficients (ld m+1)
    const double* Cpan;  // two-stage: k0 x (s+1) projection coefficients of the panel
    const double* Rh;  // GM_BIGCLOSE: Wb x Wb
    const double* Rt;  // GM_BIGCLOSE: Wb x Wb or null (identity)
    const double* C2;  // GM_BIGCLOSE: k0 x Wb or null
    // GM_BLOCK with the Newton basis: recurrence coefficients a (s) then b (s); null: monomial
    const double* newton;
    // GM_BLOCK with least squares, one system: mapped host words that receive the implicit
    // residual ([0]) and the status word (int at [1]) when the step ends (null: none)
    double* host_res;
    const int* status_in;
};

hipError_t launch_gm_small(const GmSmallArgs& a, hipStream_t st, const BatchReloc* br = nullptr);
// Ritz values of the leading k x k Hessenberg matrix (k <= 64) -> Newton coefficients (2 s).
hipError_t launch_ritz(const GmSmallArgs& a, int k, double* newton, hipStream_t st);

// Batched forms (batch.h): one launch for every active system; x, y, r and Q are template
// basis addresses, partials and y template workspace addresses.
// Rows one workgroup iteration of the batched SpMV covers for this value type and mean row
// length; the flat launch's BatchReloc::chunk is a multiple of it.
int spmv_flat_unit(bool f32, double avg_nnz);
hipError_t launch_spmv_batched(bool f32, double avg_nnz, int64_t max_n, const void* x, void* y, int grid_cap,
                               hipStream_t st, const BatchReloc& br);
hipError_t launch_residual_batched(bool f32, double avg_nnz, void* r, double* partials, int grid, hipStream_t st,
                                   const BatchReloc& br);
hipError_t launch_update_batched(bool f32, int64_t max_n, const void* Q, int max_k, const double* y, hipStream_t st,
                                 const BatchReloc& br);

}  // namespace sko
