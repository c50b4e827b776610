/*
 * sko.h -- C ABI of the MI355X (gfx950) sketched block-orthogonalisation library.
 *
 * Method: Yamazaki, Higgins, Boman, Szyld, "Random sketching to enhance the
 * numerical stability of block orthogonalization algorithms for s-step GMRES",
 * arXiv:2503.16717.  The library computes the block QR step [Q_j, R_j] = qr(Q, V_j)
 * of Section 4 (Fig. 1 caption: Q R = V, Q^T Q = I, R upper triangular with a
 * non-negative diagonal) by BCGS2 (Fig. 2c) with a CholQR2 (Section 5.1) or
 * RandCholQR (Fig. 4, Section 5.2) first intra-block step, or by the two-stage
 * scheme with RandBCGS2 pre-processing (Figs. 5, 6 and 8, Sections 6-7), and solves
 * A x = b with restarted s-step GMRES (Fig. 1) on a CSR matrix (Section 10: A in
 * CSR, the Krylov vectors column-major).
 *
 * Conventions for every entry point
 *  - Tall arrays (n rows) are DEVICE memory owned by the caller, column-major with
 *    a leading dimension (>= n).  Their element type is double for SKO_F64 and float
 *    for SKO_MIXED_F32 (the basis is then stored in single precision; every small
 *    matrix and every factorisation stays double).
 *  - Small matrices (R factors, GMRES information) are HOST memory owned by the
 *    caller, column-major.  Section 10: the small projected matrices live on the host.
 *  - Work is ordered on the context's HIP stream.  A call returns after its host
 *    outputs are valid (it synchronises that stream once, at its end).
 *  - Nothing is thrown across the ABI; every function returns an sko_status.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef SKO_H
#define SKO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sko_ctx_s* sko_ctx;

typedef enum {
    SKO_OK = 0,
    SKO_EINVAL = 1,        /* bad argument: shape, leading dimension, option or NULL pointer */
    SKO_EDEVICE = 2,       /* a HIP runtime call failed */
    SKO_ENOMEM = 3,        /* device workspace could not be allocated */
    SKO_EBREAKDOWN = 4,    /* non-positive / non-finite Cholesky pivot or zero Householder diagonal */
    SKO_ENOCONV = 5,       /* GMRES reached maxiter without meeting the tolerance */
    SKO_EUNSUPPORTED = 6,  /* valid request outside what this build implements */
    SKO_ESCRATCH = 7       /* sko_orth_block_noalloc: the request needs more than the fixed scratch */
} sko_status;

typedef enum { SKO_F64 = 0, SKO_MIXED_F32 = 1 } sko_precision;
typedef enum { SKO_SKETCH_GAUSSIAN = 0, SKO_SKETCH_SPARSE_SIGN = 1, SKO_SKETCH_COUNT_GAUSS = 2 } sko_sketch_kind;
typedef enum { SKO_INTRA_CHOLQR2 = 0, SKO_INTRA_RANDCHOLQR = 1, SKO_INTRA_CHOLQR2_RECURSIVE = 2 } sko_intra;
typedef enum { SKO_PREPROC_RANDBCGS2 = 0, SKO_PREPROC_PIP = 1 } sko_preproc;
typedef enum { SKO_BASIS_MONOMIAL = 0, SKO_BASIS_NEWTON = 1 } sko_basis;

/*
 * Random sketch Theta (n x k), applied as Theta^T X (Section 3).
 *  SKO_SKETCH_GAUSSIAN: theta points to the caller's DEVICE array holding Theta,
 *    column-major n x k with leading dimension ld_theta (Section 3: Theta = G/sqrt(k);
 *    the caller draws and scales it).  zeta and seed are ignored.
 *  SKO_SKETCH_SPARSE_SIGN: Theta has zeta nonzeros +-1/sqrt(zeta) per row and is
 *    never stored (Section 5.2 Count sketch for zeta = 1).  Requires zeta | k,
 *    k/zeta <= 128 and zeta <= 8.  Placement: with B = k/zeta, nonzero t of row i
 *    sits in slot block [tB, (t+1)B); its byte b is bits [8t, 8t+8) of the 64-bit
 *    output number i+1 of a SplitMix64 stream started at state `seed` (Steele, Lea,
 *    Flood 2014); sign = -1 iff (b & 1), slot = tB + ((b >> 1) * B >> 7).
 *  SKO_SKETCH_COUNT_GAUSS: the Count-Gaussian composite of Section 5.2, Theta =
 *    Theta_c Theta_g: a sparse-sign sketch Theta_c with k_count rows (zeta, seed and
 *    placement as above; zeta = 1 is the Count sketch), applied by the tall passes, then the
 *    caller's Gaussian factor Theta_g (DEVICE, k_count x k column-major, leading dimension
 *    ld_theta >= k_count; the caller draws it, N(0, 1/k)) applied to the reduced k_count x w
 *    sketch.  Requires k <= k_count <= 256 and the sparse-sign conditions on k_count.
 */
typedef struct {
    int32_t kind;          /* sko_sketch_kind */
    int32_t k;             /* sketch rows, 1..256 */
    int32_t zeta;          /* nonzeros per row of Theta (sparse-sign), of Theta_c (Count-Gauss) */
    int32_t k_count;       /* Count-Gauss: rows of the sparse-sign part; ignored otherwise */
    uint64_t seed;         /* sparse-sign stream seed */
    const double* theta;   /* Gaussian: device n x k; Count-Gauss: device k_count x k; column-major */
    int64_t ld_theta;
} sko_sketch;

/*
 * Orthogonalisation options.
 *  intra            first intra-block step of one-stage BCGS2 (Section 5):
 *                   SKO_INTRA_CHOLQR2, SKO_INTRA_RANDCHOLQR, or SKO_INTRA_CHOLQR2_RECURSIVE:
 *                   CholQR2 whose CholQRs (and the final CholQR of the block) use the
 *                   recursive fallback of Fig. 3: on a non-positive pivot at column k the
 *                   first k-1 columns are finished with the partial factor, the others are
 *                   projected against them with its off-diagonal block and factorised
 *                   recursively.  The host reads each Cholesky's status before going on
 *                   (one synchronisation per CholQR), and the passes are not fused.
 *                   Breakdown is reported only for a column that is numerically
 *                   dependent on the ones before it.
 *  two_stage        0: one-stage BCGS2 per block; 1: two-stage scheme (Fig. 6).
 *  preproc          two-stage pre-processing: SKO_PREPROC_RANDBCGS2 (Fig. 8; uses the
 *                   sketch) or SKO_PREPROC_PIP (BCGS with the Pythagorean inner product,
 *                   Fig. 7, Section 7.1: one reduction gives P = Q_bar_prev^T V_hat and
 *                   G = V_hat^T V_hat, R = chol(G - P^T P); no sketch; breaks down once a
 *                   big panel's condition number passes about eps^(-1/2), Section 9).
 *  panels_per_big   two-stage: blocks per big panel (s_hat / s).
 *  reorth           two-stage: 1 runs the second BCGS + CholQR over each big panel
 *                   (Fig. 5 Line 19); 0 skips it (valid when one big panel spans the
 *                   whole basis, Section 7.3).
 *  precision        SKO_F64, or SKO_MIXED_F32 (float storage of the tall arrays).
 */
typedef struct {
    int32_t intra;
    int32_t two_stage;
    int32_t panels_per_big;
    int32_t reorth;
    int32_t precision;
    int32_t preproc;       /* sko_preproc (two-stage) */
    sko_sketch sketch;
} sko_orth_opts;

/* CSR matrix in DEVICE memory: 0-based int32 row pointers (n+1) and column indices
 * (sorted within each row), double values.  Section 10: A is stored in CSR. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t* rowptr;
    const int32_t* colind;
    const double* val;
} sko_csr;

/*
 * s-step GMRES options (Fig. 1; two-stage Fig. 5).
 *  s, m           step size and restart length (s | m).
 *  shat           two-stage big-panel size (s | shat, shat | m); ignored for one-stage.
 *  two_stage      0 one-stage BCGS2 per s-step block; 1 two-stage with RandBCGS2.
 *  precond        0 none, 1 right Jacobi (M = diag(A)).
 *  intra, sketch  as for sko_orth_opts.
 *  precision      SKO_F64, or SKO_MIXED_F32 (basis in float; x and the explicit
 *                 residual in double; the matrix-powers values in float.  The
 *                 two-stage solver keeps each panel's start vector and s monomial
 *                 vectors in a double panel buffer until the panel step writes the
 *                 orthogonalised columns to the float basis: rounding the nearly
 *                 parallel monomial vectors to float would cost iterations.  The
 *                 one-stage and batched solvers write the monomial vectors to the
 *                 float basis directly.)
 *  phase_timing   1: fill t_spmv, t_orth and t_small of sko_gmres_info (HIP events at
 *                 the phase boundaries, a few microseconds each); 0: they are 0.
 *  tol            stop when ||b - A x||_2 / ||b||_2 <= tol (explicit, double).
 *  maxiter        cap on generated basis vectors (0: 50000).
 *  basis          SKO_BASIS_MONOMIAL, or SKO_BASIS_NEWTON (Section 4; Bai, Hu and Reichel
 *                 1994): the first restart cycle runs with the monomial basis; the
 *                 eigenvalues of its square Hessenberg matrix (Ritz values, computed on the
 *                 device by the double-shift QR iteration), in Leja order, give the shifts of
 *                 every later cycle, whose matrix-powers steps are v_{j+1} = (A M^{-1} - a_j)
 *                 v_j + b_j v_{j-1} (a real shift theta: (theta, 0); a complex pair alpha +- i
 *                 beta: two steps (alpha, 0), (alpha, beta^2)).  Requires m <= 64; batches with
 *                 it are solved system by system.
 *  eager          0: the one-stage single-system solver captures the launches of each s-step
 *                 block (matrix powers, orthogonalisation, Hessenberg step) into a HIP graph
 *                 once per block position and solve, and replays it (one graph launch per
 *                 block instead of about 20 kernel launches; not while the kernel profiler or
 *                 phase timing is on); 1: plain launches.  Results are the same either way.
 */
typedef struct {
    int32_t s, shat, m, two_stage;
    int32_t precond;
    int32_t intra;
    int32_t precision;
    int32_t phase_timing;
    sko_sketch sketch;
    double tol;
    int64_t maxiter;
    int32_t basis;         /* sko_basis */
    int32_t eager;         /* 1: no launch graphs */
} sko_gmres_opts;

typedef struct {
    int32_t converged;       /* 1 when the explicit relative residual met tol */
    int32_t breakdown_col;   /* 1-based basis column of a breakdown, 0 if none */
    int64_t iters;           /* basis vectors generated (multiple of s, or of shat) */
    int64_t restarts;        /* completed restart cycles */
    double relres;           /* last explicit relative residual */
    double relres_implicit;  /* last implicit (least-squares) relative residual */
    double t_total;          /* seconds, measured with HIP events on the stream */
    /* Phase times in seconds (opts->phase_timing), the split the paper's time-to-solution
     * table reports (Table 4: SpMV and orthogonalisation):
     *  t_spmv   matrix-powers SpMVs and the explicit residual b - A x;
     *  t_orth   block orthogonalisation: tall passes, reductions and their small
     *           factorisations (sketch QR, Cholesky, sketch-space BCGS2);
     *  t_small  Hessenberg bookkeeping, least squares and the update x += M^{-1} Q y.
     * The batched solver reports the whole batch's phase times for every system. */
    double t_spmv, t_orth, t_small;
} sko_gmres_info;

/* Create a context on HIP device `device` that orders its work on `hip_stream`
 * (a hipStream_t; NULL means the device's null stream).  The context owns a device
 * workspace that grows on demand and is reused. */
sko_status sko_create(int device, void* hip_stream, sko_ctx* out);
sko_status sko_destroy(sko_ctx ctx);
/* Re-target the context to another stream of the same device. */
sko_status sko_set_stream(sko_ctx ctx, void* hip_stream);
const char* sko_strerror(sko_status status);

/*
 * One BCGS2 block step (Fig. 2c): orthogonalise V (n x w) against the orthonormal
 * columns of Q (n x p), giving Q_out (n x w, may alias V) with
 *   V = Q * R_proj + Q_out * R_diag,   Q^T Q_out = 0,   Q_out^T Q_out = I.
 * R_proj (p x w, ld p) and R_diag (w x w, ld w, upper, positive diagonal) are HOST
 * arrays; either may be NULL.  Q may be NULL when p == 0.  opts->two_stage must be 0.
 * w <= 16.  On SKO_EBREAKDOWN *breakdown_col (if not NULL) is the 1-based column of V.
 */
sko_status sko_orth_block(sko_ctx ctx, int64_t n, int32_t p, int32_t w,
                          const void* Q, int64_t ldq, const void* V, int64_t ldv,
                          void* Q_out, int64_t ldqo, double* R_proj, double* R_diag,
                          const sko_orth_opts* opts, int32_t* breakdown_col);

/*
 * sko_orth_block without allocating: for callers that cannot allocate device or pinned
 * memory while they run (work recorded for a graph replay, tight serving loops, harnesses
 * that forbid allocation).  Arguments, results and errors are those of sko_orth_block; the
 * kernels and the order of every partial sum are the same, so on the same context the
 * outputs are the same.  The call allocates nothing: the reductions' partial sums, the
 * small factors and the status words live in a fixed device scratch of
 * SKO_NOALLOC_SCRATCH_BYTES (32 MiB) that the library holds on every device it runs on
 * until the process ends (its device address is looked up by sko_create); R is copied
 * straight into the caller's host arrays, and the context's kernel profiler does not see
 * these launches.  Needed scratch: 8 * G * ceil(max(p, k, w) * w / 32) * 32 bytes of
 * partial sums, G = min(ceil(n / 256), 8 * compute units), plus about 8 * (2 p w + k w +
 * (p + w)^2 + 5 w^2) bytes; a request above 32 MiB returns SKO_ESCRATCH (2^24 rows with
 * w = 6, k = 64 and p <= 66 need 7 MB).
 * Every call on a device shares that device's scratch, and the status words are cleared at
 * the start of each call: calls that overlap on one device (from any context or thread)
 * race and give wrong results.
 */
#define SKO_NOALLOC_SCRATCH_BYTES (32u << 20)
sko_status sko_orth_block_noalloc(sko_ctx ctx, int64_t n, int32_t p, int32_t w,
                                  const void* Q, int64_t ldq, const void* V, int64_t ldv,
                                  void* Q_out, int64_t ldqo, double* R_proj, double* R_diag,
                                  const sko_orth_opts* opts, int32_t* breakdown_col);

/*
 * Orthogonalise all nb blocks of width w of V (n x nb*w) in order: one-stage BCGS2
 * per block (Fig. 2c), or two-stage over big panels of panels_per_big blocks (Fig. 6,
 * the flat form of Fig. 5, with the RandBCGS2 pre-processing of Fig. 8).  Result: Q
 * (n x nb*w, may alias V) and the HOST upper-triangular R (N x N, N = nb*w, leading
 * dimension ldr >= N; may be NULL) with V = Q R.  w <= 16; two-stage big panels are at
 * most 64 columns wide.  On SKO_EBREAKDOWN *breakdown_col is the 1-based column.
 */
sko_status sko_orth_blocks(sko_ctx ctx, int64_t n, int32_t nb, int32_t w,
                           const void* V, int64_t ldv, void* Q, int64_t ldq,
                           double* R, int64_t ldr, const sko_orth_opts* opts,
                           int32_t* breakdown_col);

/*
 * Sketch a tall block: Y = Theta^T X (Section 3: the sketch is applied to a block as
 * Theta^T X; Section 5.2: the Count sketch, here the sparse-sign sketch, is applied without
 * storing Theta).  This is the reduction the RandCholQR step (Fig. 4a) and the two-stage
 * panel step (Fig. 8) run on their panels, with the same kernels, the same nonzero
 * placement (see sko_sketch) and the same order of partial sums; it exposes that sketch so
 * it can be checked on its own.
 *  X          DEVICE, n x w column-major (leading dimension ldx >= n), w <= 16; double for
 *             SKO_F64, float for SKO_MIXED_F32 (`precision`).
 *  sketch     Theta (kind, k <= 256, zeta, seed; or the caller's Gaussian array with n rows).
 *  Y          HOST, k x w column-major (leading dimension ldy >= k), written on success.
 * Errors: SKO_EINVAL (shapes, NULL pointers, an invalid sketch), SKO_ENOMEM, SKO_EDEVICE.
 */
sko_status sko_sketch_apply(sko_ctx ctx, int64_t n, int32_t w, const void* X, int64_t ldx,
                            int32_t precision, const sko_sketch* sketch, double* Y, int64_t ldy);

/*
 * Restarted s-step GMRES (Fig. 1): solve A x = b with right preconditioning.
 * b and x are DEVICE double vectors of length A->n; x holds x0 on entry and the
 * last iterate on exit (also on SKO_ENOCONV).  info (HOST, may be NULL) is filled
 * in every case.  The workspace holds the (m+1)-column basis.
 */
sko_status sko_gmres(sko_ctx ctx, const sko_csr* A, const double* b, double* x,
                     const sko_gmres_opts* opts, sko_gmres_info* info);

/*
 * nsys independent systems solved together (same options; system i uses sketch
 * seed opts->sketch.seed + i).  A, b, x, infos are HOST arrays of length nsys whose
 * elements describe DEVICE data as in sko_gmres.  Returns SKO_OK when every system
 * converged, otherwise the first failing status; infos[i] tells each system's fate.
 */
sko_status sko_gmres_batched(sko_ctx ctx, int32_t nsys, const sko_csr* A,
                             const double* const* b, double* const* x,
                             const sko_gmres_opts* opts, sko_gmres_info* infos);

/*
 * Launch-shape autotuning (the row-strip passes of the block orthogonalisation).
 * How many workgroups per compute unit stream a pass fastest depends on the pass variant
 * (its registers, LDS and the number of column streams it reads).  This call times every
 * pass variant that sko_orth_blocks(ctx, n, nb, w, ..., opts) launches, each at its median
 * operand width, on scratch blocks the library allocates (n x (2w + p_max) elements plus
 * small buffers, freed before returning), for 2..8 workgroups per compute unit, and keeps
 * the fastest count in ctx for that variant and row-count class (floor(log2(n / 256))).
 * Later launches of those variants on this context, by any entry point, use the choice;
 * all other launches keep the default (as many workgroups as are resident at once).  The
 * deterministic comparators (two-stage with SKO_PREPROC_PIP, SKO_INTRA_CHOLQR2_RECURSIVE)
 * are not tuned: the call returns SKO_OK without timing anything.
 * The arithmetic per row is unchanged; only the grouping of the per-workgroup partial
 * sums follows the grid, so results may change in the last bits once, when a choice
 * changes.  n below 1024 * (compute units) rows: nothing to tune, returns SKO_OK.
 * Errors: SKO_EINVAL (arguments as for sko_orth_blocks), SKO_ENOMEM (scratch), SKO_EDEVICE.
 */
sko_status sko_autotune_orth(sko_ctx ctx, int64_t n, int32_t nb, int32_t w, const sko_orth_opts* opts);

/*
 * Kernel profiling (tracing subsystem).  When enabled, every tall-pass and reduction
 * launch issued by the context is bracketed by HIP events on the context's stream,
 * and per kernel kind the library accumulates the launch count, the summed event time
 * and the algorithmic HBM bytes of those launches (each tall operand counted once per
 * pass: columns read plus columns written, times n, times the element size).
 * sko_profile_enable(ctx, 1) clears the counters and starts recording; 0 stops it.
 * sko_profile_read copies up to max entries (sorted by total time, largest first) and
 * returns the number of kinds recorded, or a negative sko_status on error.
 */
typedef struct {
    char name[96];         /* kernel kind, e.g. "pass W=6 f64 red=proj upd=0 trsm=2 write=1" */
    int64_t launches;
    double total_ms;       /* summed event time of all launches */
    double bytes;          /* summed algorithmic bytes of all launches */
} sko_kernel_stat;

sko_status sko_profile_enable(sko_ctx ctx, int enable);
int32_t sko_profile_read(sko_ctx ctx, sko_kernel_stat* out, int32_t max);

#ifdef __cplusplus
}
#endif

#endif /* SKO_H */
