// Internal declarations shared by the HIP translation units of libsko.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>

#include "sko.h"

namespace sko {

struct BatchReloc;  // batched launches (batch.h)

// ---------------------------------------------------------------------------
// Row-strip pass: one streaming sweep over n rows of a tall-skinny block.
//
// Per row (phase A, one thread per row):
//   x = Y[row, 0:W]
//   x -= Qu[row, 0:pu] * Cu                  (UPD: BCGS update V - Q C, Fig. 2a)
//   x  = x * R1^{-1} [* R2^{-1}]             (NTRSM: row forward substitution, Fig. 4a)
//   X[row, 0:W] = x                          (WRITE)
// Per strip (phase B, lanes over rows, waves over reduction rows): one reduction
//   RED_PROJ          Qp^T x       (Q^T V of BCGS, Fig. 2a)
//   RED_GRAM          x^T x        (Gram of CholQR, Fig. 2b)
//   RED_SKETCH_SPARSE Theta^T x    (sparse-sign sketch, hashed, Section 5.2)
//   RED_SKETCH_DENSE  Theta^T x    (Gaussian sketch, stored Theta, Section 5.2)
// Each workgroup writes its partial reduction to partials[blockIdx.x * part_stride + e],
// e = row + col * part_rows_total; a reduce kernel sums the partials in a fixed order.
// ---------------------------------------------------------------------------
enum RedKind : int {
    RED_NONE = 0,
    RED_PROJ = 1,
    RED_GRAM = 2,
    RED_SKETCH_SPARSE = 3,
    RED_SKETCH_DENSE = 4,
};

struct PassArgs {
    int64_t n;
    const void* Y;            // input block, W columns
    int64_t ldy;
    const void* Qu;           // UPD operand (pu columns)
    int64_t ldqu;
    const double* Cu;         // UPD coefficients, pu x W column-major (ld pu)
    const double* R1;         // TRSM factors, W x W column-major, upper
    const double* R2;
    void* X;                  // WRITE target
    int64_t ldx;
    const void* Qp;           // PROJ operand, already offset to reduction row red_row0
    int64_t ldqp;
    const double* theta;      // dense sketch, n x k column-major, offset to red_row0
    int64_t ldtheta;
    double* partials;
    int64_t part_stride;      // doubles between consecutive workgroups' partials
    uint64_t sk_seed;
    int32_t pu;
    int32_t red_rows;         // reduction rows handled by this launch
    int32_t red_row0;         // global index of the first of them
    int32_t part_rows_total;  // rows of the whole reduction output
    int32_t sk_k;
    int32_t sk_zeta;
};

struct PassKey {
    int W;
    bool f32;          // storage type float (else double)
    int red;
    bool upd;
    int ntrsm;
    bool write;
    int tiles = 0;     // projection: 16-row MFMA tiles one launch needs (0: the maximum)
    // mixed-precision GMRES panel (f32 basis): 1 = FP64 panel Y read against the basis, FP64
    // X; 2 = FP64 panel Y, X written into the FP32 basis; 0 = one storage type throughout
    int panel = 0;
};

// Launch one pass over all n rows with `grid` workgroups (grid <= pass_grid_cap()).  With
// `br`, one launch serves every active system of a batch (grid workgroups each).
hipError_t launch_pass(const PassKey& key, const PassArgs& args, int grid, hipStream_t stream,
                       const BatchReloc* br = nullptr);
// Reduction rows one launch of reduction kind `red` can produce for panel width W.
int pass_rows_per_launch(int W, int red);
// Identity of the kernel a pass variant launches (null if the variant does not exist).
const void* pass_kernel_id(const PassKey& key);
// Rows per strip (= threads per workgroup) of a pass variant.
int pass_strip_rows(const PassKey& key);
// Largest useful grid for a pass variant on the current device (resident workgroups).
int pass_grid_cap(const PassKey& key);
// Workgroups of `threads` threads of `kernel` resident on the current device at once
// (cached per kernel and device; -1 if the runtime cannot tell).
int resident_grid(const void* kernel, int threads);
constexpr int kPassThreads = 256;
constexpr int kMaxPassW = 16;
constexpr int kMaxUpdCoef = 4096;   // pu * W update coefficients of one pass (p * w of one block step)

// ---------------------------------------------------------------------------
// Reduction of pass partials + the small dense step that consumes it.
// ---------------------------------------------------------------------------
enum SmallOp : int {
    OP_STORE = 0,        // reduced values are the result (e.g. C = Q^T V)
    OP_HH = 1,           // Householder R of the k x w sketch (Fig. 4a Line 4), diag >= 0
    OP_CHOL = 2,         // upper Cholesky factor of the w x w Gram matrix (Fig. 2b)
    OP_SKETCH_BCGS2 = 3, // sketch-space BCGS2 with Householder (Fig. 8a)
    OP_PIP = 4,          // BCGS-PIP step (Fig. 7): R = chol(G - P^T P)
};

struct SmallArgs {
    int op;
    int w;               // block width
    int k;               // sketch rows (OP_HH / OP_SKETCH_BCGS2)
    int col0;            // global 1-based column offset for breakdown reports
    double* out;         // reduced values (count doubles); OP_HH/OP_SKETCH_BCGS2: k x w sketch
    double* R;           // OP_HH / OP_CHOL / OP_SKETCH_BCGS2: w x w result (ld w)
    // OP_CHOL, optional: R packed for the wide row solve, w reciprocal diagonal entries then
    // the strictly upper part column by column (column c's c entries at w + c(c-1)/2)
    double* Rpk;
    int* status;         // first breakdown column (0 = none)
    // OP_SKETCH_BCGS2
    double* Yacc;        // k x cap, column-major (ld k): accumulated orthonormal sketches
    int nacc;            // columns of Yacc orthogonalised against (the first nacc)
    double* r;           // nacc x w coefficients (ld nacc), r1 + r2
    // OP_PIP: the reduced values are P (nacc x w) and `gram` holds G (w x w) from an earlier
    // reduction; with nacc = 0 the reduced values are G itself.  R = chol(G - P^T P), r = P.
    const double* gram;
    // OP_SKETCH_BCGS2 / OP_PIP: optional copy of [r; R] into columns rbar_col0.. of Rbar (ld ldrbar)
    double* Rbar;
    int ldrbar;
    int rbar_col0;
    // assembly after OP_CHOL (assemble != 0):
    //   Rhat = Ra * Rb (w x w), Rdiag = R * Rhat, Rproj = C1 + C2 * Rhat (p x w)
    // (r_identity != 0: the R of this reduction is replaced by the identity in Rdiag)
    int assemble;
    int r_identity;
    const double* Ra;
    const double* Rb;
    const double* C1;
    const double* C2;
    int p;
    double* Rout;        // destination of [Rproj; Rdiag] columns in a big R (ld ldr)
    int64_t ldr;
    // Count-Gauss sketch (theta_g != null): the reduced values in `out` are the kc x w Count
    // part; the step first forms theta_g^T out (k x w, theta_g kc x k with leading dimension
    // ld_g) and works on that.  OP_STORE then writes the k x w product to R (ld k).
    const double* theta_g;
    int64_t ld_g;
    int kc;
};

struct ReduceArgs {
    const double* partials;
    int64_t stride;
    int G;
    int count;
    double scale;
    // Arrival counter, zero when the launch starts: the workgroup that draws ticket
    // grid - 1 is the last one; it runs the small step and resets the counter to zero, so
    // the next launch on it (stream order, so never concurrent) counts from zero again and
    // no launch is needed to clear it (nor inside a captured graph).
    unsigned int* counter;
    // Placement of reduced element e (= r + c * rows): small.out[r + c * ldo].  OP_STORE
    // may write into a sub-block of a larger matrix; the other ops need ldo == rows.
    int rows;
    int64_t ldo;
    SmallArgs small;
    // Rows the producing launch assigns to each workgroup index (workgroup g has rows only
    // if g * unit_rows < n).  Batched launches size their grid for the largest system, so
    // a smaller system's trailing workgroups wrote zero partials; its reduction sums only
    // the first ceil(n / unit_rows).  0: all G.
    int unit_rows = 0;
};
// Rows per workgroup index of the wide Gram / projection kernel (16-row groups, 4 waves).
constexpr int kGemmUnitRows = 64;

// How a sketch is applied: the tall passes reduce `rows` sketch rows of kind `red` (the
// hashed sparse-sign Theta, or the stored Gaussian Theta), scaled by `scale`; a Count-Gauss
// sketch then multiplies the reduced rows by its Gaussian factor in the small step.
struct SketchPlan {
    int red;
    int rows;      // rows the passes produce: k, or k_count for Count-Gauss
    int k;         // rows of the final sketch
    double scale;
    const double* theta_g;
    int64_t ld_g;
};
SketchPlan sketch_plan(const sko_sketch& sk);
// Hand the Count-Gauss factor (if any) to a small step.
inline void sketch_small(SmallArgs& sm, const SketchPlan& sp) {
    sm.theta_g = sp.theta_g;
    sm.ld_g = sp.ld_g;
    sm.kc = sp.theta_g ? sp.rows : 0;
}

// Number of workgroups launch_reduce uses for `count` reduced values.
int reduce_grid(int count);

hipError_t launch_reduce(const ReduceArgs& args, hipStream_t stream, const BatchReloc* br = nullptr);

// Small dense kernels used outside a reduction.
// Big-panel helpers (two-stage): C = A^T B for tall A (n x ma), B (n x nb), ma, nb <= 64.
hipError_t launch_skinny_gemm_tn(int64_t n, const void* A, int64_t lda, int ma,
                                 const void* B, int64_t ldb, int nb, bool f32,
                                 double* partials, int grid, hipStream_t stream,
                                 const BatchReloc* br = nullptr);
int skinny_gemm_grid_cap();
// Workgroups of the one-system wide Gram (sym) / projection kernel for ma x nb outputs that
// are resident at once (-1 if the runtime cannot tell).
int skinny_gemm_resident(bool sym, bool f32, int ma, int nb);

// The wide row operation with the following reduction in the same sweep: X as
// launch_wide_rowop (W <= kFusedMaxW; the solve only, no update), plus the per-workgroup partials of E^T X (E: n x me tall, me <= 48; stride me * W)
// or, with E null, of the Gram X^T X (upper tiles; stride W * W).  One system: the grid
// (workgroups = partial blocks, at most skinny_gemm_grid_cap()) is returned in *grid_out.
// Batched (br): *grid_out workgroups per system are launched, and those past a system's
// ceil(n / kFusedUnitRows) write no partials.
constexpr int kFusedMaxW = 40;
constexpr int kFusedUnitRows = 256;
hipError_t launch_wide_rowop_reduce(int64_t n, int W, bool f32, const void* Y, int64_t ldy, const void* Qu,
                                    int64_t ldqu, int pu, const double* Cu, const double* Rpk, void* X, int64_t ldx,
                                    const void* E, int64_t lde, int me, double* partials, int* grid_out,
                                    hipStream_t st, const BatchReloc* br = nullptr);

// Row-wise X = (Y - Qu Cu) * R^{-1} for wide blocks (w <= 64); used by the big-panel
// close of the two-stage scheme.  Rpk is R in the packed form of SmallArgs::Rpk (null: no
// solve).
hipError_t launch_wide_rowop(int64_t n, int W, bool f32, const void* Y, int64_t ldy,
                             const void* Qu, int64_t ldqu, int pu, const double* Cu,
                             const double* Rpk, void* X, int64_t ldx, hipStream_t stream,
                             const BatchReloc* br = nullptr);

// Zero `rows` runs of `width` bytes, consecutive runs `pitch` bytes apart (pointer, pitch
// and width multiples of 4 bytes).  A kernel rather than hipMemsetAsync, so the work is an
// ordinary kernel node wherever a caller captures the stream into a graph.
hipError_t launch_zero_2d(void* p, size_t pitch, size_t width, size_t rows, hipStream_t stream);
inline hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
    return launch_zero_2d(p, bytes, bytes, 1, stream);
}

// The R assembly of a BCGS2 block step on its own (the assembly fields of SmallArgs: Rhat =
// Ra Rb into rh (w x w), Rdiag = R Rhat, Rproj = C1 + C2 Rhat into Rout); one workgroup.
hipError_t launch_assemble(const SmallArgs& s, double* rh, hipStream_t stream);

// Small matrix helpers on the device (single workgroup).
hipError_t launch_small_matmul_upper(int w, const double* A, const double* B, double* C,
                                     hipStream_t stream);

}  // namespace sko
