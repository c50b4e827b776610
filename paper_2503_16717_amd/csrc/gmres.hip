// Restarted s-step GMRES on the device (Fig. 1) and its two-stage form (Fig. 5).
//
// Per restart cycle:
//   r = b - A x (FP64 A, x, b) written into basis column 0, beta = ||r|| (reduction +
//   1 x 1 Cholesky), the host checks ||r|| / ||b|| <= tol (explicit, the convergence test),
//   q_1 = r / beta.
// One-stage block (basis size k): the matrix-powers kernel writes (A M^{-1})^i q_k into basis
//   columns k+1..k+s, so V_j = Q[:, k:k+s+1] in place; BCGS2 against Q[:, 0:k] replaces the
//   boundary column k and the s new ones (Table 1: V_j includes its start vector).  The
//   block's R columns update T_in / T_out (device), H = T_out T_in^{-1}, and Givens rotations
//   give the implicit residual, read by the host after every block.
// Two-stage: per panel the MPK starts from the last pre-processed vector; BCGS against the
//   previous big panels, sketch, sketch-space BCGS2-HH, forward substitution (Fig. 5 Lines
//   10, 12); at the big-panel end CholQR (Line 15) and, when s_hat < m, BCGS + CholQR
//   (Line 19); the implicit check runs once per big panel.
// Cycle end: x += M^{-1} Q y with M = diag(A) for Jacobi (right preconditioning).
//
// Batched form (many independent systems, two-stage): the systems advance in lock step and
// every launch serves all systems still active (batch.h); the host reads all systems'
// residuals with one strided copy per check and drops converged systems from the launches.
#include <algorithm>
#include <chrono>
#include <numeric>
#include <vector>

#include "engine.h"
#include "gmres_internal.h"

namespace sko {
namespace {

struct GmCtx {
    sko_ctx c;
    hipStream_t st;
    int64_t n, ld;
    int s, m, W, shat, Wb;
    bool f32, two, jacobi, reorth;
    int intra;
    sko_sketch sk;
    // device
    void* Q;
    // mixed precision, two-stage: the FP64 panel (s + 1 columns, leading dimension ld) that
    // holds a panel's start vector and its matrix-powers vectors until the panel step writes
    // the orthogonalised columns into the FP32 basis (null otherwise)
    double* P = nullptr;
    double* dinv;
    CsrView A;
    double *Tin, *Tout, *g, *gw, *H, *y, *res, *beta, *bnorm, *coef;
    double *Cpan, *Yacc, *rt, *rho, *Gb, *Rh, *Rt, *C2b;
    double* Rpk;  // packed copy of Rh, then of Rt, for the row solves
    // Newton basis: recurrence coefficients a (s) then b (s) on the device, set from the first
    // cycle's Ritz values (newton_on from then on)
    double* newton = nullptr;
    bool newton_on = false;
    // launch graphs of the one-stage blocks, one per block position (null: eager launches);
    // cap_st: the private stream the launches are captured on
    std::vector<hipGraphExec_t>* graphs = nullptr;
    hipStream_t cap_st = nullptr;
    unsigned* counter = nullptr;  // reduction arrival counter (each reduction leaves it at zero)
    BlockBufs bb;
    int* status;
    int grid_cap;
    // host (pinned)
    double* host;  // [0] res, [1] beta, [2] bnorm; status at host+4 as int
    // batched mode: template addresses are system 0's; launches go to every active system
    const BatchReloc* br = nullptr;
    double avg_nnz = 0.0;
    int64_t max_n = 0;
    double rows_bytes = 0.0, nnz_bytes = 0.0;  // active totals for the byte accounting
    int spmv_cap = 0;
    PhaseTimer* pt = nullptr;  // phase times (sko_gmres_opts::phase_timing)
    void phase(int ph) const {
        if (pt) pt->phase(ph, st);
    }
};

// Small per-solve device buffers, one contiguous block (offsets in bytes).
struct SmallLayout {
    size_t bb, gm, ts, st, bytes;
};

// kr: sketch rows the passes reduce; k: rows of the (final) sketch.
SmallLayout small_layout(int m, int W, int kr, int k, int Wb, bool two) {
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t mW = (size_t)m * W;
    SmallLayout L{};
    L.bb = 0;
    L.gm = up(L.bb + sizeof(double) * (2 * mW + (size_t)std::max(kr, W) * W + 7 * (size_t)W * W));
    L.ts = up(L.gm + sizeof(double) * (3 * (size_t)(m + 1) * m + 3 * (size_t)(m + 1) + 8 + (size_t)(m + 1) * W));
    L.st = up(L.ts + (two ? sizeof(double) * (mW + (size_t)k * Wb + (size_t)Wb * W + (size_t)W * W +
                                              3 * (size_t)Wb * Wb + (size_t)m * Wb + (size_t)Wb * (Wb + 1) / 2)
                          : 0));
    L.bytes = up(L.st + 256);
    return L;
}

// Point g's small buffers into the block at `base`.
void carve_small(GmCtx& g, char* base, const SmallLayout& L, int kr, int k) {
    const int m = g.m, W = g.W;
    const int64_t mW = (int64_t)m * W;
    double* p = reinterpret_cast<double*>(base + L.bb);
    g.bb.C1 = p;
    g.bb.C2 = p + mW;
    g.bb.Ysk = g.bb.C2 + mW;
    g.bb.G2 = g.bb.Ysk + (int64_t)std::max(kr, W) * W;
    g.bb.G3 = g.bb.G2 + W * W;
    g.bb.R1 = g.bb.G3 + W * W;
    g.bb.R2 = g.bb.R1 + W * W;
    g.bb.R3 = g.bb.R2 + W * W;
    g.bb.S1 = g.bb.R3 + W * W;
    g.bb.S2 = g.bb.S1 + W * W;
    double* q = reinterpret_cast<double*>(base + L.gm);
    const int64_t big = (int64_t)(m + 1) * m;
    g.Tin = q;
    g.Tout = q + big;
    g.H = q + 2 * big;
    g.g = q + 3 * big;
    g.gw = g.g + (m + 1);
    g.y = g.gw + (m + 1);
    g.res = g.y + (m + 1);
    g.beta = g.res + 2;
    g.bnorm = g.beta + 2;
    g.coef = g.res + 8;
    if (g.two) {
        double* t = reinterpret_cast<double*>(base + L.ts);
        g.Cpan = t;
        g.Yacc = g.Cpan + mW;
        g.rt = g.Yacc + (int64_t)k * g.Wb;
        g.rho = g.rt + (int64_t)g.Wb * W;
        g.Gb = g.rho + W * W;
        g.Rh = g.Gb + g.Wb * g.Wb;
        g.Rt = g.Rh + g.Wb * g.Wb;
        g.C2b = g.Rt + g.Wb * g.Wb;
        g.Rpk = g.C2b + (int64_t)m * g.Wb;
    }
    g.status = reinterpret_cast<int*>(base + L.st);
}

void* col_ptr(const GmCtx& g, int col) {
    return static_cast<char*>(g.Q) + (int64_t)col * g.ld * (g.f32 ? 4 : 8);
}

sko_status read_scalars(GmCtx& g, const double* dev, int count, int* status_out) {
    if (g.pt) g.pt->stop(g.st);
    SKO_HIP(hipMemcpyAsync(g.host, dev, sizeof(double) * count, hipMemcpyDeviceToHost, g.st));
    SKO_HIP(hipMemcpyAsync(reinterpret_cast<int*>(g.host + 4), g.status, sizeof(int), hipMemcpyDeviceToHost, g.st));
    SKO_HIP(hipStreamSynchronize(g.st));
    g.c->prof.flush();
    if (g.pt) g.pt->flush();
    if (status_out) *status_out = *reinterpret_cast<int*>(g.host + 4);
    return SKO_OK;
}

// ||v||_2 of a device double vector via a 1-column Gram pass and a 1 x 1 Cholesky.
sko_status norm2(GmCtx& g, Engine& e1, const double* v, double* out) {
    PassArgs a{};
    a.Y = v;
    a.ldy = g.n;
    SmallArgs sm{};
    sm.op = OP_CHOL;
    sm.w = 1;
    sm.out = g.gw;  // scratch for the reduced value
    sm.R = out;
    return e1.reduction({1, false, RED_GRAM, false, 0, false}, a, 1, nullptr, 0, nullptr, 0, sm, 1.0);
}

sko_status mpk(GmCtx& g, int from, int s) {
    const double nnz = g.br ? g.nnz_bytes : (double)g.A.nnz;
    const double rows = g.br ? g.rows_bytes : (double)g.n;
    g.phase(PhaseTimer::SPMV);
    for (int i = 1; i <= s; ++i) {
        const int ev = g.c->prof.begin(std::string("spmv ") + (g.f32 ? "f32" : "f64"),
                                       nnz * (g.f32 ? 8.0 : 12.0) + rows * (g.f32 ? 12.0 : 20.0), g.st);
        if (g.br)
            SKO_HIP(launch_spmv_batched(g.f32, g.avg_nnz, g.max_n, col_ptr(g, from + i - 1), col_ptr(g, from + i),
                                        g.spmv_cap, g.st, *g.br));
        else if (g.newton_on)  // step i - 1 of the Newton recurrence
            SKO_HIP(launch_spmv(g.A, g.f32, col_ptr(g, from + i - 1), col_ptr(g, from + i), g.grid_cap, g.st,
                                g.newton + (i - 1), g.newton + g.s + (i - 1), col_ptr(g, from + (i >= 2 ? i - 2 : 0))));
        else
            SKO_HIP(launch_spmv(g.A, g.f32, col_ptr(g, from + i - 1), col_ptr(g, from + i), g.grid_cap, g.st));
        g.c->prof.end(ev, g.st);
    }
    return SKO_OK;
}

// Mixed precision, two-stage: the start vector (FP32 basis column `from`) widened into
// column 0 of the FP64 panel and the s monomial vectors computed in FP64 from it.  Rounding
// the nearly parallel monomial vectors to FP32 before they are orthogonalised would lose the
// small components that carry the new Krylov directions; the panel step rounds only the
// orthogonalised columns.
sko_status mpk_panel(GmCtx& g, int from, int s) {
    double* P = g.P;
    g.phase(PhaseTimer::SPMV);
    SKO_HIP(launch_widen(g.n, static_cast<const float*>(col_ptr(g, from)), P, g.grid_cap, g.st));
    for (int i = 1; i <= s; ++i) {
        const int ev = g.c->prof.begin("spmv f32 values, f64 vectors",
                                       (double)g.A.nnz * 8.0 + (double)g.n * 20.0, g.st);
        if (g.newton_on)
            SKO_HIP(launch_spmv_panel(g.A, P + (int64_t)(i - 1) * g.ld, P + (int64_t)i * g.ld, g.grid_cap, g.st,
                                      g.newton + (i - 1), g.newton + g.s + (i - 1),
                                      P + (int64_t)(i >= 2 ? i - 2 : 0) * g.ld));
        else
            SKO_HIP(launch_spmv_panel(g.A, P + (int64_t)(i - 1) * g.ld, P + (int64_t)i * g.ld, g.grid_cap, g.st));
        g.c->prof.end(ev, g.st);
    }
    return SKO_OK;
}

sko_status gm_op(GmCtx& g, GmSmallArgs a) {
    a.m = g.m;
    a.s = g.s;
    a.Tin = g.Tin;
    a.Tout = g.Tout;
    a.g = g.g;
    a.gw = g.gw;
    a.H = g.H;
    a.y = g.y;
    a.res = g.res;
    a.beta = g.beta;
    a.coef = g.coef;
    if (a.op == GM_BLOCK && g.newton_on) a.newton = g.newton;
    g.phase(PhaseTimer::SMALL);
    const int ev = g.c->prof.begin("gmres small", 0.0, g.st);
    SKO_HIP(launch_gm_small(a, g.st, g.br));
    g.c->prof.end(ev, g.st);
    return SKO_OK;
}

// The launches of one one-stage block at basis position k: matrix powers, BCGS2, the
// Hessenberg step, which also writes the implicit residual and the status word into the
// context's mapped host words.
sko_status one_stage_block_launches(GmCtx& g, Engine& e, int k) {
    sko_status s;
    if ((s = mpk(g, k, g.s))) return s;
    void* Vk = col_ptr(g, k);
    g.phase(PhaseTimer::ORTH);
    if ((s = one_stage_block(e, g.bb, g.intra, k, g.Q, g.ld, Vk, g.ld, Vk, g.ld, g.coef, g.m + 1, k))) return s;
    GmSmallArgs a{};
    a.op = GM_BLOCK;
    a.kk = k;
    a.do_lsq = 1;
    // the step itself writes the residual and the status word into the mapped host words
    a.host_res = g.c->zc_dev;
    a.status_in = g.status;
    if ((s = gm_op(g, a))) return s;
    if (g.pt) g.pt->stop(g.st);
    return SKO_OK;
}

// Ends a stream capture on every return path (a failed capture leaves no stream capturing).
struct CaptureGuard {
    hipStream_t st;
    bool active = false;
    hipGraph_t graph = nullptr;
    explicit CaptureGuard(hipStream_t s) : st(s) {}
    hipError_t begin() {
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        active = e == hipSuccess;
        return e;
    }
    hipError_t end() {
        active = false;
        return hipStreamEndCapture(st, &graph);
    }
    ~CaptureGuard() {
        if (active) (void)hipStreamEndCapture(st, &graph);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Block at position k through its launch graph: captured (on the private stream) the first
// time the position is reached in this solve, replayed on the solve's stream after that.  Every
// reduction leaves its arrival counter at zero, so a replay needs no clearing launch.
sko_status one_stage_block_graph(GmCtx& g, Engine& e, int k) {
    hipGraphExec_t& ge = (*g.graphs)[k / g.s];
    if (!ge) {
        const hipStream_t st0 = g.st;
        CaptureGuard cap(g.cap_st);
        SKO_HIP(cap.begin());
        g.st = e.st = g.cap_st;
        const sko_status s = one_stage_block_launches(g, e, k);
        g.st = e.st = st0;
        const hipError_t ce = cap.end();
        if (s) return s;
        if (ce != hipSuccess) return SKO_EDEVICE;
        SKO_HIP(hipGraphInstantiate(&ge, cap.graph, nullptr, nullptr, 0));
    }
    SKO_HIP(hipGraphLaunch(ge, g.st));
    return SKO_OK;
}

// One cycle; returns the basis size k reached (y[0:k] on the device), or 0 on breakdown.
sko_status cycle_one_stage(GmCtx& g, Engine& e, double bnorm, double tol, sko_gmres_info& inf, int64_t maxiter,
                           int* k_out) {
    int k = 0;
    sko_status s;
    while (k < g.m) {
        if ((s = g.graphs ? one_stage_block_graph(g, e, k) : one_stage_block_launches(g, e, k))) return s;
        SKO_HIP(hipStreamSynchronize(g.st));
        g.c->prof.flush();
        if (g.pt) g.pt->flush();
        const volatile double* zc = g.c->zc_host;
        const int status = reinterpret_cast<const volatile int*>(zc + 1)[0];
        inf.iters += g.s;
        k += g.s;
        if (status) {
            inf.breakdown_col = status;
            *k_out = 0;
            return SKO_EBREAKDOWN;
        }
        inf.relres_implicit = zc[0] / bnorm;
        if (inf.relres_implicit <= tol || inf.iters >= maxiter) break;
    }
    *k_out = k;
    return SKO_OK;
}

// One s-step panel of a two-stage big panel (Fig. 5): MPK from the last pre-processed
// vector, BCGS against the previous big panels, sketch with sketch-space BCGS2-HH, forward
// substitution, and the block's Hessenberg columns.
sko_status two_stage_panel(GmCtx& g, Engine& e, int k0, int i) {
    sko_status s;
    const int S = g.s, W = g.W, ld = (int)g.m + 1;
    const SketchPlan sp = sketch_plan(g.sk);
    const int red_sk = sp.red;
    const double sk_scale = sp.scale;
    void* Qb = col_ptr(g, k0);
    const int loc = i * S, kk = k0 + loc;
    // the panel V: in the basis itself, or (mixed precision) in the FP64 panel buffer
    const bool p64 = g.P != nullptr;
    if ((s = p64 ? mpk_panel(g, kk, S) : mpk(g, kk, S))) return s;
    void* V = p64 ? static_cast<void*>(g.P) : col_ptr(g, kk);
    g.phase(PhaseTimer::ORTH);
    PassKey key{W, g.f32 && !p64, red_sk, false, 0, false};
    PassArgs a{};
    a.Y = V;
    a.ldy = g.ld;
    if (k0 > 0) {
        PassArgs pa{};
        pa.Y = V;
        pa.ldy = g.ld;
        SmallArgs sm{};
        sm.op = OP_STORE;
        sm.w = W;
        sm.out = g.Cpan;
        PassKey pkey{W, g.f32, RED_PROJ, false, 0, false};
        pkey.panel = p64 ? 1 : 0;
        if ((s = e.reduction(pkey, pa, k0, V, g.ld, g.Q, g.ld, sm, 1.0))) return s;
        key.f32 = g.f32;
        key.panel = p64 ? 1 : 0;
        key.upd = true;
        key.write = true;
        a.Qu = g.Q;
        a.ldqu = g.ld;
        a.pu = k0;
        a.Cu = g.Cpan;
        a.X = V;
        a.ldx = g.ld;
    }
    SmallArgs sm{};
    sm.op = OP_SKETCH_BCGS2;
    sm.w = W;
    sm.k = sp.k;
    sketch_small(sm, sp);
    sm.col0 = kk;
    sm.out = g.bb.Ysk;
    sm.R = g.rho;
    sm.Yacc = g.Yacc;
    sm.nacc = loc;
    sm.r = g.rt;
    sm.Rbar = g.coef + k0;
    sm.ldrbar = ld;
    sm.rbar_col0 = 0;
    if ((s = e.reduction(key, a, sp.rows, V, g.ld, nullptr, 0, sm, sk_scale))) return s;
    PassArgs fa{};
    fa.Y = V;
    fa.ldy = g.ld;
    fa.R1 = g.rho;
    fa.X = col_ptr(g, kk);
    fa.ldx = g.ld;
    PassKey fkey{W, g.f32, RED_NONE, false, 1, true};
    fkey.panel = p64 ? 2 : 0;
    if (loc > 0) {
        fkey.upd = true;
        fa.Qu = Qb;
        fa.ldqu = g.ld;
        fa.pu = loc;
        fa.Cu = g.rt;
    }
    if ((s = e.plain(fkey, fa))) return s;
    GmSmallArgs ga{};
    ga.op = GM_BLOCK;
    ga.kk = kk;
    ga.k0 = k0;
    ga.two_stage = 1;
    ga.Cpan = k0 > 0 ? g.Cpan : nullptr;
    return gm_op(g, ga);
}

// Big-panel close (Fig. 5 Line 15, Fig. 6 Line 19): CholQR of the pre-processed big panel,
// then (s_hat < m) BCGS against the previous big panels and a second CholQR; the stored
// Hessenberg columns are re-expressed in the final basis and the least squares solved.
sko_status two_stage_bigclose(GmCtx& g, Engine& e, int k0) {
    sko_status s;
    const int Wb = g.Wb;
    void* Qb = col_ptr(g, k0);
    g.phase(PhaseTimer::ORTH);
    {
        SmallArgs sm{};
        sm.op = OP_CHOL;
        sm.w = Wb;
        sm.col0 = k0;
        sm.out = g.Gb;
        sm.R = g.Rh;
        sm.Rpk = g.Rpk;
        if ((s = e.gemm_reduction(Qb, g.ld, Wb, Qb, g.ld, Wb, sm, Wb))) return s;
    }
    // With the second pass, each row operation also accumulates the reduction that follows
    // it (the projection on the previous big panels, or the second Gram matrix).
    const bool proj2 = g.reorth && k0 > 0;
    const bool fuse_proj = proj2 && k0 <= 64;
    SmallArgs chol2{};
    chol2.op = OP_CHOL;
    chol2.w = Wb;
    chol2.col0 = k0;
    chol2.out = g.Gb;
    chol2.R = g.Rt;
    chol2.Rpk = g.Rpk;
    if (g.reorth && !proj2) {
        if ((s = e.rowop_reduction(Wb, Qb, g.ld, nullptr, 0, 0, nullptr, g.Rpk, Qb, g.ld, nullptr, 0, 0, chol2, Wb)))
            return s;
    } else if (fuse_proj) {
        SmallArgs sp2{};
        sp2.op = OP_STORE;
        sp2.w = Wb;
        sp2.out = g.C2b;
        if ((s = e.rowop_reduction(Wb, Qb, g.ld, nullptr, 0, 0, nullptr, g.Rpk, Qb, g.ld, col_ptr(g, 0), g.ld, k0, sp2,
                                   k0)))
            return s;
    } else {
        if ((s = e.rowop(Wb, Qb, g.ld, nullptr, 0, 0, nullptr, g.Rpk, Qb, g.ld))) return s;
    }
    if (g.reorth) {
        if (proj2) {
            if (!fuse_proj) {
                for (int a0 = 0; a0 < k0; a0 += 64) {
                    const int ma = std::min(64, k0 - a0);
                    SmallArgs sm{};
                    sm.op = OP_STORE;
                    sm.w = Wb;
                    sm.out = g.C2b + a0;
                    if ((s = e.gemm_reduction(col_ptr(g, a0), g.ld, ma, Qb, g.ld, Wb, sm, k0))) return s;
                }
            }
            if ((s = e.rowop_reduction(Wb, Qb, g.ld, g.Q, g.ld, k0, g.C2b, nullptr, Qb, g.ld, nullptr, 0, 0, chol2,
                                       Wb)))
                return s;
        }
        if ((s = e.rowop(Wb, Qb, g.ld, nullptr, 0, 0, nullptr, g.Rpk, Qb, g.ld))) return s;
    }
    GmSmallArgs ga{};
    ga.op = GM_BIGCLOSE;
    ga.k0 = k0;
    ga.Wb = Wb;
    ga.kend = k0 + g.shat;
    ga.two_stage = 1;
    ga.Rh = g.Rh;
    ga.Rt = g.reorth ? g.Rt : nullptr;
    ga.C2 = proj2 ? g.C2b : nullptr;
    return gm_op(g, ga);
}

sko_status cycle_two_stage(GmCtx& g, Engine& e, double bnorm, double tol, sko_gmres_info& inf, int64_t maxiter,
                           int* k_out) {
    sko_status s;
    int k0 = 0, k = 0;
    while (k0 < g.m) {
        for (int i = 0; i < g.shat / g.s; ++i) {
            if ((s = two_stage_panel(g, e, k0, i))) return s;
            inf.iters += g.s;
        }
        if ((s = two_stage_bigclose(g, e, k0))) return s;
        const int kend = k0 + g.shat;
        int status = 0;
        if ((s = read_scalars(g, g.res, 1, &status))) return s;
        k = kend;
        if (status) {
            inf.breakdown_col = status;
            *k_out = 0;
            return SKO_EBREAKDOWN;
        }
        inf.relres_implicit = g.host[0] / bnorm;
        if (inf.relres_implicit <= tol || inf.iters >= maxiter) break;
        k0 = kend;
    }
    *k_out = k;
    return SKO_OK;
}

}  // namespace

namespace {

// Option checks shared by the single and batched solvers; fills the shape fields of g.
sko_status check_opts(const sko_csr* A, const sko_gmres_opts* o, GmCtx& g) {
    if (!A || !o || !A->rowptr || !A->colind || !A->val || A->n < 1 || A->nnz < 1) return SKO_EINVAL;
    const int S = o->s, m = o->m;
    if (S < 1 || m < S || m % S) return SKO_EINVAL;
    if (S + 1 > kMaxPassW || m + 1 > 255) return SKO_EUNSUPPORTED;
    const bool two = o->two_stage != 0;
    const int shat = two ? (o->shat > 0 ? o->shat : m) : S;
    if (two && (shat % S || m % shat)) return SKO_EINVAL;
    if (two && shat + 1 > 64) return SKO_EUNSUPPORTED;
    if (o->precision != SKO_F64 && o->precision != SKO_MIXED_F32) return SKO_EINVAL;
    if (o->precond != 0 && o->precond != 1) return SKO_EINVAL;
    if (!two && o->intra != SKO_INTRA_CHOLQR2 && o->intra != SKO_INTRA_RANDCHOLQR) return SKO_EINVAL;
    const bool need_sketch = two || o->intra == SKO_INTRA_RANDCHOLQR;
    if (need_sketch && !sketch_ok(o->sketch, A->n)) return SKO_EINVAL;
    if (need_sketch && o->sketch.k < (two ? shat + 1 : S + 1)) return SKO_EINVAL;
    if (!(o->tol > 0.0)) return SKO_EINVAL;
    if (o->basis != SKO_BASIS_MONOMIAL && o->basis != SKO_BASIS_NEWTON) return SKO_EINVAL;
    if (o->basis == SKO_BASIS_NEWTON && m > 64) return SKO_EUNSUPPORTED;
    g.n = A->n;
    g.ld = ((A->n + 63) / 64) * 64;
    g.s = S;
    g.m = m;
    g.W = S + 1;
    g.shat = shat;
    g.Wb = shat + 1;
    g.f32 = o->precision == SKO_MIXED_F32;
    g.two = two;
    g.jacobi = o->precond == 1;
    g.reorth = two && shat < m;
    g.intra = o->intra;
    g.sk = o->sketch;
    return SKO_OK;
}

// Rows of the sketch (final = false: the rows the passes reduce, k_count for Count-Gauss).
int sketch_rows(const GmCtx& g, bool final = true) {
    const bool need_sketch = g.two || g.intra == SKO_INTRA_RANDCHOLQR;
    return need_sketch ? (final ? g.sk.k : sketch_plan(g.sk).rows) : g.W;
}

}  // namespace

sko_status gmres_impl(sko_ctx c, const sko_csr* A, const double* b, double* x, const sko_gmres_opts* o,
                      sko_gmres_info* info) {
    sko_gmres_info inf{};
    if (info) *info = inf;
    GmCtx g{};
    if (!b || !x) return SKO_EINVAL;
    if (sko_status cs = check_opts(A, o, g)) return cs;
    const int m = g.m;
    const int64_t maxiter = o->maxiter > 0 ? o->maxiter : 50000;
    g.c = c;
    g.st = c->stream;
    const int eb = g.f32 ? 4 : 8;
    const int k = sketch_rows(g), kr = sketch_rows(g, false);

    // ---- workspace
    Arena ar(c);
    const size_t o_Q = ar.reserve((size_t)eb * g.ld * (m + 1));
    const bool panel64 = g.f32 && g.two;
    const size_t o_P = panel64 ? ar.reserve(sizeof(double) * g.ld * g.W) : 0;
    const bool own_vals = g.jacobi || g.f32;
    const size_t o_val = own_vals ? ar.reserve((size_t)eb * A->nnz) : 0;
    const size_t o_dinv = g.jacobi ? ar.reserve(sizeof(double) * A->n) : 0;
    const int64_t nstrips = (A->n + kPassThreads - 1) / kPassThreads;
    const int gmax = (int)std::min<int64_t>(nstrips, (int64_t)std::max(1, c->cus) * 8);
    const int64_t rows = std::max({(int64_t)m, (int64_t)kr, (int64_t)g.W});
    const int64_t part_stride = ((rows * g.W + 31) / 32) * 32;
    g.grid_cap = std::max(1, c->cus) * 8;
    const size_t part_doubles = std::max({(size_t)part_stride * gmax, (size_t)64 * 64 * std::max(1, skinny_gemm_grid_cap()),
                                          (size_t)g.grid_cap});
    const size_t o_part = ar.reserve(sizeof(double) * part_doubles);
    const SmallLayout L = small_layout(m, g.W, kr, k, g.Wb, g.two);
    const size_t o_small = ar.reserve(L.bytes);
    const size_t o_newton = ar.reserve(sizeof(double) * 2 * g.s);
    sko_status s = ensure_workspace(c, ar.used());
    if (s) return s;
    if ((s = ensure_pinned(c, 64))) return s;
    if ((s = ensure_zerocopy(c))) return s;
    g.host = static_cast<double*>(c->pinned);
    g.newton = ar.at<double>(o_newton);
    g.Q = ar.at<void>(o_Q);
    g.P = panel64 ? ar.at<double>(o_P) : nullptr;
    g.dinv = g.jacobi ? ar.at<double>(o_dinv) : nullptr;
    carve_small(g, ar.at<char>(o_small), L, kr, k);

    EventPair ev_total;
    SKO_HIP(ev_total.create());
    PhaseTimer pt;
    pt.on = o->phase_timing != 0;
    g.pt = &pt;
    SKO_HIP(hipEventRecord(ev_total.a, g.st));
    SKO_HIP(launch_zero(g.status, 256, g.st));

    // ---- CSR structure check before any kernel indexes through it
    {
        int bad = 0;
        SKO_HIP(launch_csr_check(A->n, A->nnz, A->rowptr, A->colind, g.status + 32, g.st));
        SKO_HIP(hipMemcpyAsync(reinterpret_cast<int*>(g.host + 4), g.status + 32, sizeof(int), hipMemcpyDeviceToHost,
                               g.st));
        SKO_HIP(hipStreamSynchronize(g.st));
        bad = *reinterpret_cast<int*>(g.host + 4);
        if (bad) return SKO_EINVAL;
    }
    // ---- operator set-up: Jacobi scaling / float copy of the MPK values
    g.A = CsrView{A->n, A->nnz, A->rowptr, A->colind, A->val, A->val};
    if (g.jacobi) SKO_HIP(launch_jacobi_setup(A->n, A->nnz, A->rowptr, A->colind, A->val, g.dinv, g.status, g.st));
    if (own_vals) {
        void* vo = ar.at<void>(o_val);
        SKO_HIP(launch_scale_values(A->nnz, A->colind, A->val, g.dinv, g.f32, vo, g.st));
        g.A.val_op = vo;
    }

    Engine e(c, A->n, g.W, g.f32, g.sk);
    e.partials = ar.at<double>(o_part);
    e.part_stride = part_stride;
    e.gmax = gmax;
    e.status = g.status;
    e.counter = reinterpret_cast<unsigned*>(g.status + 16);
    g.counter = e.counter;
    // launch graphs for the one-stage blocks (not while launches are timed one by one)
    std::vector<hipGraphExec_t> graphs;
    struct GraphsGuard {
        std::vector<hipGraphExec_t>& v;
        ~GraphsGuard() {
            for (hipGraphExec_t ge : v)
                if (ge) (void)hipGraphExecDestroy(ge);
        }
    } graphs_guard{graphs};
    if (!g.two && !o->eager && !c->prof.on && !pt.on) {
        if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return SKO_EDEVICE;
        graphs.assign(g.m / g.s, nullptr);
        g.graphs = &graphs;
        g.cap_st = c->cap_stream;
    }
    Engine e1(c, A->n, 1, false, g.sk);
    e1.partials = e.partials;
    e1.part_stride = part_stride;
    e1.gmax = gmax;
    e1.status = g.status;
    e1.counter = e.counter;
    Engine e1f(c, A->n, 1, g.f32, g.sk);
    e1f.partials = e.partials;
    e1f.part_stride = part_stride;
    e1f.gmax = gmax;
    e1f.status = g.status;
    e1f.counter = e.counter;

    if ((s = norm2(g, e1, b, g.bnorm))) return s;
    int status = 0;
    if ((s = read_scalars(g, g.bnorm, 1, &status))) return s;
    if (status == -1) return SKO_EINVAL;  // zero diagonal with Jacobi
    const double bnorm = g.host[0];
    sko_status result = SKO_OK;
    if (!(bnorm > 0.0) || !std::isfinite(bnorm)) {
        result = bnorm == 0.0 ? SKO_OK : SKO_EINVAL;
    } else {
        while (true) {
            // explicit residual r = b - A x into basis column 0, beta = ||r||
            const int rg = residual_grid(A->n, g.grid_cap);
            g.phase(PhaseTimer::SPMV);
            const int ev = c->prof.begin("residual f64", (double)A->nnz * 12.0 + (double)A->n * 24.0, g.st);
            SKO_HIP(launch_residual(g.A, x, b, g.f32, g.Q, e.partials, rg, g.st));
            c->prof.end(ev, g.st);
            {
                ReduceArgs ra{};
                ra.partials = e.partials;
                ra.stride = 1;
                ra.G = rg;
                ra.count = 1;
                ra.scale = 1.0;
                ra.counter = e.counter;
                ra.rows = 1;
                ra.ldo = 1;
                ra.small.op = OP_CHOL;
                ra.small.w = 1;
                ra.small.out = g.gw;
                ra.small.R = g.beta;
                ra.small.status = nullptr;
                SKO_HIP(launch_reduce(ra, g.st));
            }
            if ((s = read_scalars(g, g.beta, 1, &status))) return s;
            const double beta = g.host[0];
            inf.relres = beta / bnorm;
            if (inf.relres <= o->tol) {
                inf.converged = 1;
                break;
            }
            if (inf.iters >= maxiter) {
                result = SKO_ENOCONV;
                break;
            }
            {   // q_1 = r / beta
                PassArgs a{};
                a.Y = g.Q;
                a.ldy = g.ld;
                a.R1 = g.beta;
                a.X = g.Q;
                a.ldx = g.ld;
                g.phase(PhaseTimer::ORTH);
                if ((s = e1f.plain({1, g.f32, RED_NONE, false, 1, true}, a))) return s;
            }
            GmSmallArgs ia{};
            ia.op = GM_INIT;
            if ((s = gm_op(g, ia))) return s;
            int kreached = 0;
            s = g.two ? cycle_two_stage(g, e, bnorm, o->tol, inf, maxiter, &kreached)
                    : cycle_one_stage(g, e, bnorm, o->tol, inf, maxiter, &kreached);
            if (s == SKO_EBREAKDOWN) {
                result = s;
                break;
            }
            if (s) return s;
            if (o->basis == SKO_BASIS_NEWTON && !g.newton_on && kreached > 0) {
                // shifts for the later cycles: Leja-ordered Ritz values of this cycle
                GmSmallArgs ra{};
                ra.m = g.m;
                ra.s = g.s;
                ra.Tin = g.Tin;
                ra.Tout = g.Tout;
                g.phase(PhaseTimer::SMALL);
                SKO_HIP(launch_ritz(ra, kreached, g.newton, g.st));
                g.newton_on = true;
                // the captured blocks ran the monomial steps: capture again
                for (hipGraphExec_t& ge : graphs)
                    if (ge) {
                        SKO_HIP(hipGraphExecDestroy(ge));
                        ge = nullptr;
                    }
            }
            {
                g.phase(PhaseTimer::SMALL);
                const int ev2 = c->prof.begin("update x", (double)A->n * (kreached * eb + 16.0), g.st);
                SKO_HIP(launch_update(A->n, g.f32, g.Q, g.ld, kreached, g.y, g.dinv, x, g.st));
                c->prof.end(ev2, g.st);
            }
            inf.restarts += 1;
        }
    }
    pt.stop(g.st);
    SKO_HIP(hipEventRecord(ev_total.b, g.st));
    SKO_HIP(hipEventSynchronize(ev_total.b));
    c->prof.flush();
    pt.flush();
    inf.t_total = ev_total.ms() * 1e-3;
    inf.t_spmv = pt.ms[PhaseTimer::SPMV] * 1e-3;
    inf.t_orth = pt.ms[PhaseTimer::ORTH] * 1e-3;
    inf.t_small = pt.ms[PhaseTimer::SMALL] * 1e-3;
    if (info) *info = inf;
    return result;
}

namespace {

sko_status gmres_sequential(sko_ctx c, int32_t nsys, const sko_csr* A, const double* const* b, double* const* x,
                            const sko_gmres_opts* o, sko_gmres_info* infos) {
    sko_status first = SKO_OK;
    for (int32_t i = 0; i < nsys; ++i) {
        sko_gmres_opts oi = *o;
        oi.sketch.seed = o->sketch.seed + (uint64_t)i;
        sko_gmres_info inf{};
        const sko_status s = gmres_impl(c, &A[i], b[i], x[i], &oi, &inf);
        if (infos) infos[i] = inf;
        if (s != SKO_OK && first == SKO_OK) first = s;
    }
    return first;
}

struct SysState {
    double bnorm = 0.0;
    bool finished = false;
    bool in_cycle = false;
    sko_status result = SKO_OK;
    sko_gmres_info inf{};
};

}  // namespace

// Many independent two-stage solves in lock step: one launch per step serves every system
// still active.  Systems share (s, s_hat, m, precision, preconditioner, sketch size); system i
// draws its sparse-sign sketch from seed + i, as a one-by-one solve of it would.
sko_status gmres_batched_impl(sko_ctx c, int32_t nsys, const sko_csr* A, const double* const* b, double* const* x,
                              const sko_gmres_opts* o, sko_gmres_info* infos) {
    if (nsys < 0 || (nsys > 0 && (!A || !b || !x || !o))) return SKO_EINVAL;
    if (nsys == 0) return SKO_OK;
    if (infos)
        for (int32_t i = 0; i < nsys; ++i) infos[i] = sko_gmres_info{};
    // lock step needs the two-stage scheme with the hashed sketch (no per-system Theta) and
    // the monomial basis (Newton shifts are per system)
    if (nsys == 1 || !o->two_stage || o->sketch.kind == SKO_SKETCH_GAUSSIAN || o->basis != SKO_BASIS_MONOMIAL)
        return gmres_sequential(c, nsys, A, b, x, o, infos);

    GmCtx g{};
    std::vector<SysState> S(nsys);
    for (int32_t i = 0; i < nsys; ++i) {
        GmCtx gi{};
        if (!b[i] || !x[i]) return SKO_EINVAL;
        if (sko_status cs = check_opts(&A[i], o, gi)) return cs;
        if (i == 0) g = gi;
    }
    const int m = g.m;
    const int64_t maxiter = o->maxiter > 0 ? o->maxiter : 50000;
    g.c = c;
    g.st = c->stream;
    const int eb = g.f32 ? 4 : 8;
    const int k = sketch_rows(g), kr = sketch_rows(g, false);
    const bool own_vals = g.jacobi || g.f32;
    int64_t max_n = 0;
    double nnz_sum = 0.0, n_sum = 0.0;
    for (int32_t i = 0; i < nsys; ++i) {
        max_n = std::max<int64_t>(max_n, A[i].n);
        nnz_sum += (double)A[i].nnz;
        n_sum += (double)A[i].n;
    }

    // ---- launch shapes: per system a fraction of the one-system grid, since one launch
    // holds every system
    const int cap = std::max(1, c->cus) * 8;
    const int64_t strips_max = (max_n + kPassThreads - 1) / kPassThreads;
    const int Gp = (int)std::max<int64_t>(1, std::min<int64_t>((strips_max + 7) / 8, cap));
    const int64_t rows = std::max({(int64_t)m, (int64_t)kr, (int64_t)g.W});
    const int64_t part_stride = ((rows * g.W + 31) / 32) * 32;
    const int64_t ns32 = (max_n + 31) / 32;
    const int Gg = (int)std::max<int64_t>(1, std::min<int64_t>((ns32 + 63) / 64, skinny_gemm_grid_cap()));
    const int64_t gemm_cells = std::max<int64_t>((int64_t)g.Wb * g.Wb, (int64_t)std::min(64, m) * g.Wb);
    const int64_t groups8 = (max_n + 256 / 8 - 1) / (256 / 8);
    const int Gr = (int)std::max<int64_t>(1, std::min<int64_t>((groups8 + 15) / 16, cap));
    const size_t part_doubles = std::max({(size_t)part_stride * Gp, (size_t)gemm_cells * Gg, (size_t)Gr});
    const size_t part_bytes = ((sizeof(double) * part_doubles + 255) / 256) * 256;
    const SmallLayout L = small_layout(m, g.W, kr, k, g.Wb, g.two);

    // ---- workspace: per-system basis / operator values / D^{-1}, then the equal-sized small
    // blocks, partial sums, the system table and the active list
    Arena ar(c);
    std::vector<size_t> o_Q(nsys), o_val(nsys, 0), o_dinv(nsys, 0);
    for (int32_t i = 0; i < nsys; ++i) {
        const int64_t ldi = ((A[i].n + 63) / 64) * 64;
        o_Q[i] = ar.reserve((size_t)eb * ldi * (m + 1));
        if (own_vals) o_val[i] = ar.reserve((size_t)eb * A[i].nnz);
        if (g.jacobi) o_dinv[i] = ar.reserve(sizeof(double) * A[i].n);
    }
    const size_t o_small = ar.reserve(L.bytes * nsys);
    const size_t o_part = ar.reserve(part_bytes * nsys);
    const size_t o_tbl = ar.reserve(sizeof(BatchSys) * nsys);
    const size_t o_act = ar.reserve(sizeof(int) * nsys);
    const size_t o_blk = ar.reserve(sizeof(int) * (nsys + 1));
    sko_status s = ensure_workspace(c, ar.used());
    if (s) return s;
    const size_t pin_tbl = 0, pin_act = sizeof(BatchSys) * nsys, pin_dbl = pin_act + ((sizeof(int) * nsys + 63) / 64) * 64,
                 pin_int = pin_dbl + sizeof(double) * nsys, pin_blk = pin_int + ((sizeof(int) * nsys + 63) / 64) * 64,
                 pin_end = pin_blk + sizeof(int) * (nsys + 1) + 64;
    if ((s = ensure_pinned(c, pin_end))) return s;
    char* pin = static_cast<char*>(c->pinned);
    BatchSys* tbl_h = reinterpret_cast<BatchSys*>(pin + pin_tbl);
    int* act_h = reinterpret_cast<int*>(pin + pin_act);
    double* dbl_h = reinterpret_cast<double*>(pin + pin_dbl);
    int* int_h = reinterpret_cast<int*>(pin + pin_int);
    int* blk_h = reinterpret_cast<int*>(pin + pin_blk);
    g.host = dbl_h;

    char* small0 = ar.at<char>(o_small);
    double* part0 = ar.at<double>(o_part);
    BatchSys* tbl_d = ar.at<BatchSys>(o_tbl);
    int* act_d = ar.at<int>(o_act);
    int* blk_d = ar.at<int>(o_blk);
    auto small_of = [&](int i) { return small0 + (size_t)i * L.bytes; };
    auto part_of = [&](int i) { return reinterpret_cast<double*>(reinterpret_cast<char*>(part0) + (size_t)i * part_bytes); };

    // template = system 0
    g.ld = ((A[0].n + 63) / 64) * 64;
    g.n = A[0].n;
    g.Q = ar.at<void>(o_Q[0]);
    carve_small(g, small_of(0), L, kr, k);
    g.grid_cap = cap;
    g.avg_nnz = nnz_sum / std::max(1.0, n_sum);
    g.max_n = max_n;
    g.spmv_cap = (int)std::max<int64_t>(1, std::min<int64_t>((groups8 + 7) / 8, cap));
    const size_t st_off = (size_t)(reinterpret_cast<char*>(g.status) - small_of(0));

    EventPair ev_total;
    SKO_HIP(ev_total.create());
    PhaseTimer pt;
    pt.on = o->phase_timing != 0;
    g.pt = &pt;
    SKO_HIP(hipEventRecord(ev_total.a, g.st));
    SKO_HIP(launch_zero_2d(small0 + st_off, L.bytes, 256, nsys, g.st));

    // strided reads of one double / one int of every system's small block
    auto read_dbl = [&](const double* tmpl) -> sko_status {
        pt.stop(g.st);
        SKO_HIP(hipMemcpy2DAsync(dbl_h, sizeof(double), tmpl, L.bytes, sizeof(double), nsys, hipMemcpyDeviceToHost,
                                 g.st));
        SKO_HIP(hipMemcpy2DAsync(int_h, sizeof(int), g.status, L.bytes, sizeof(int), nsys, hipMemcpyDeviceToHost,
                                 g.st));
        SKO_HIP(hipStreamSynchronize(g.st));
        c->prof.flush();
        pt.flush();
        return SKO_OK;
    };

    // ---- per system: CSR check, operator set-up, ||b|| (single-system launches)
    for (int32_t i = 0; i < nsys; ++i) {
        int* st_i = reinterpret_cast<int*>(small_of(i) + st_off);
        SKO_HIP(launch_csr_check(A[i].n, A[i].nnz, A[i].rowptr, A[i].colind, st_i + 32, g.st));
    }
    SKO_HIP(hipMemcpy2DAsync(int_h, sizeof(int), g.status + 32, L.bytes, sizeof(int), nsys, hipMemcpyDeviceToHost,
                             g.st));
    SKO_HIP(hipStreamSynchronize(g.st));
    for (int32_t i = 0; i < nsys; ++i)
        if (int_h[i]) {
            S[i].finished = true;
            S[i].result = SKO_EINVAL;
        }
    for (int32_t i = 0; i < nsys; ++i) {
        const int64_t ldi = ((A[i].n + 63) / 64) * 64;
        BatchSys& d = tbl_h[i];
        d = BatchSys{};
        d.n = A[i].n;
        d.ld = ldi;
        d.nnz = A[i].nnz;
        d.Q = ar.at<char>(o_Q[i]);
        d.rowptr = A[i].rowptr;
        d.colind = A[i].colind;
        d.val = A[i].val;
        d.val_op = A[i].val;
        d.b = b[i];
        d.x = x[i];
        d.dinv = g.jacobi ? ar.at<double>(o_dinv[i]) : nullptr;
        d.seed = o->sketch.seed + (uint64_t)i;
        d.kupd = 0;
        if (S[i].finished) continue;
        int* st_i = reinterpret_cast<int*>(small_of(i) + st_off);
        if (g.jacobi)
            SKO_HIP(launch_jacobi_setup(A[i].n, A[i].nnz, A[i].rowptr, A[i].colind, A[i].val,
                                        const_cast<double*>(d.dinv), st_i, g.st));
        if (own_vals) {
            void* vo = ar.at<void>(o_val[i]);
            SKO_HIP(launch_scale_values(A[i].nnz, A[i].colind, A[i].val, d.dinv, g.f32, vo, g.st));
            d.val_op = vo;
        }
        GmCtx gi = g;
        gi.n = A[i].n;
        carve_small(gi, small_of(i), L, kr, k);
        Engine e1(c, A[i].n, 1, false, g.sk);
        e1.partials = part_of(i);
        e1.part_stride = part_stride;
        e1.gmax = Gp;
        e1.status = gi.status;
        e1.counter = reinterpret_cast<unsigned*>(gi.status + 16);
        if ((s = norm2(gi, e1, b[i], gi.bnorm))) return s;
    }
    if ((s = read_dbl(g.bnorm))) return s;
    for (int32_t i = 0; i < nsys; ++i) {
        if (S[i].finished) continue;
        if (int_h[i] == -1) {  // zero diagonal with Jacobi
            S[i].finished = true;
            S[i].result = SKO_EINVAL;
            continue;
        }
        S[i].bnorm = dbl_h[i];
        if (!(S[i].bnorm > 0.0) || !std::isfinite(S[i].bnorm)) {
            S[i].finished = true;
            S[i].result = S[i].bnorm == 0.0 ? SKO_OK : SKO_EINVAL;
        }
    }
    SKO_HIP(hipMemcpyAsync(tbl_d, tbl_h, sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, g.st));
    SKO_HIP(hipStreamSynchronize(g.st));

    BatchReloc br{};
    br.sys = tbl_d;
    br.active = act_d;
    br.nact = 0;
    br.eb = eb;
    br.q0 = static_cast<const char*>(g.Q);
    br.q0_bytes = (int64_t)eb * g.ld * (m + 1);
    br.ld0 = g.ld;
    br.ws0 = small0;
    br.ws_bytes = (int64_t)L.bytes;
    br.part0 = reinterpret_cast<const char*>(part0);
    br.part_bytes = (int64_t)part_bytes;
    br.cnt0 = nullptr;
    br.cnt_bytes = 0;
    br.blk0 = blk_d;
    {
        // the arena carves every region one after another, so this holds by construction
        const void* shared[3] = {tbl_d, act_d, blk_d};
        const int64_t shared_bytes[3] = {(int64_t)sizeof(BatchSys) * nsys, (int64_t)sizeof(int) * nsys,
                                         (int64_t)sizeof(int) * (nsys + 1)};
        if (!batch_regions_disjoint(br, shared, shared_bytes, 3)) return SKO_EINVAL;
    }
    const int flat_unit = spmv_flat_unit(g.f32, g.avg_nnz);
    g.br = &br;

    Engine e(c, max_n, g.W, g.f32, g.sk);
    e.partials = part0;
    e.part_stride = part_stride;
    e.gmax = Gp;
    e.status = g.status;
    e.counter = reinterpret_cast<unsigned*>(g.status + 16);
    e.br = &br;
    Engine e1f(c, max_n, 1, g.f32, g.sk);
    e1f.partials = part0;
    e1f.part_stride = part_stride;
    e1f.gmax = Gp;
    e1f.status = g.status;
    e1f.counter = e.counter;
    e1f.br = &br;

    // New active list (largest systems first, so their workgroups are dispatched first).
    auto set_active = [&](std::vector<int> list) -> sko_status {
        std::sort(list.begin(), list.end(), [&](int a, int q) { return A[a].n > A[q].n || (A[a].n == A[q].n && a < q); });
        double nr = 0.0, nz = 0.0;
        for (size_t j = 0; j < list.size(); ++j) {
            act_h[j] = list[j];
            nr += (double)A[list[j]].n;
            nz += (double)A[list[j]].nnz;
        }
        // flat SpMV: about 16 workgroups per CU over the active rows, each 1 to 8 iterations
        // (fewer rows per workgroup once only a few large systems are left)
        const int64_t want = (int64_t)std::max(1, c->cus) * 16;
        const int64_t iters = std::min<int64_t>(8, std::max<int64_t>(1, ((int64_t)nr / want + flat_unit - 1) / flat_unit));
        br.chunk = (int)(iters * flat_unit);
        blk_h[0] = 0;
        for (size_t j = 0; j < list.size(); ++j)
            blk_h[j + 1] = blk_h[j] + (int)((A[list[j]].n + br.chunk - 1) / br.chunk);
        br.nact = (int)list.size();
        br.nblk = blk_h[list.size()];
        e.rows_bytes = e1f.rows_bytes = g.rows_bytes = nr;
        g.nnz_bytes = nz;
        if (list.empty()) return SKO_OK;
        pt.stop(g.st);
        SKO_HIP(hipMemcpyAsync(act_d, act_h, sizeof(int) * list.size(), hipMemcpyHostToDevice, g.st));
        SKO_HIP(hipMemcpyAsync(blk_d, blk_h, sizeof(int) * (list.size() + 1), hipMemcpyHostToDevice, g.st));
        SKO_HIP(launch_zero_2d(small0 + st_off + 16 * sizeof(int), L.bytes, sizeof(unsigned), nsys, g.st));
        SKO_HIP(hipStreamSynchronize(g.st));
            return SKO_OK;
    };

    while (true) {
        std::vector<int> live;
        for (int32_t i = 0; i < nsys; ++i)
            if (!S[i].finished) live.push_back(i);
        if (live.empty()) break;
        if ((s = set_active(live))) return s;
        // explicit residuals r = b - A x into basis column 0, beta = ||r||
        {
            g.phase(PhaseTimer::SPMV);
            const int ev = c->prof.begin("residual f64", g.nnz_bytes * 12.0 + g.rows_bytes * 24.0,
                                         g.st);
            SKO_HIP(launch_residual_batched(g.f32, g.avg_nnz, g.Q, part0, Gr, g.st, br));
            c->prof.end(ev, g.st);
            ReduceArgs ra{};
            ra.partials = part0;
            ra.stride = 1;
            ra.G = Gr;
            ra.count = 1;
            ra.scale = 1.0;
            ra.counter = e.counter;
            ra.rows = 1;
            ra.ldo = 1;
            ra.small.op = OP_CHOL;
            ra.small.w = 1;
            ra.small.out = g.gw;
            ra.small.R = g.beta;
            ra.small.status = nullptr;
            SKO_HIP(launch_reduce(ra, g.st, &br));
        }
        if ((s = read_dbl(g.beta))) return s;
        std::vector<int> cyc;
        for (int i : live) {
            SysState& q = S[i];
            q.inf.relres = dbl_h[i] / q.bnorm;
            if (q.inf.relres <= o->tol) {
                q.inf.converged = 1;
                q.finished = true;
            } else if (q.inf.iters >= maxiter) {
                q.result = SKO_ENOCONV;
                q.finished = true;
            } else {
                cyc.push_back(i);
            }
        }
        if (cyc.empty()) break;
        if (cyc.size() != live.size() && (s = set_active(cyc))) return s;
        for (int i : cyc) S[i].in_cycle = true;
        {   // q_1 = r / beta
            PassArgs a{};
            a.Y = g.Q;
            a.ldy = g.ld;
            a.R1 = g.beta;
            a.X = g.Q;
            a.ldx = g.ld;
            g.phase(PhaseTimer::ORTH);
            if ((s = e1f.plain({1, g.f32, RED_NONE, false, 1, true}, a))) return s;
        }
        GmSmallArgs ia{};
        ia.op = GM_INIT;
        if ((s = gm_op(g, ia))) return s;
        std::vector<int> kreached(nsys, 0);
        std::vector<int> running = cyc;
        for (int k0 = 0; k0 < m && !running.empty(); k0 += g.shat) {
            for (int i = 0; i < g.shat / g.s; ++i) {
                if ((s = two_stage_panel(g, e, k0, i))) return s;
                for (int j : running) S[j].inf.iters += g.s;
            }
            if ((s = two_stage_bigclose(g, e, k0))) return s;
            if ((s = read_dbl(g.res))) return s;
            const int kend = k0 + g.shat;
            std::vector<int> next;
            for (int j : running) {
                SysState& q = S[j];
                if (int_h[j]) {  // breakdown: no update from this cycle
                    q.inf.breakdown_col = int_h[j];
                    q.result = SKO_EBREAKDOWN;
                    q.finished = true;
                    q.in_cycle = false;
                    kreached[j] = 0;
                    continue;
                }
                kreached[j] = kend;
                q.inf.relres_implicit = dbl_h[j] / q.bnorm;
                if (q.inf.relres_implicit <= o->tol || q.inf.iters >= maxiter || kend >= m) continue;
                next.push_back(j);
            }
            if (next.size() != running.size() && !next.empty() && (s = set_active(next))) return s;
            running.swap(next);
        }
        // x += M^{-1} Q y for every system of this cycle
        std::vector<int> upd;
        for (int i : cyc) {
            tbl_h[i].kupd = S[i].in_cycle ? kreached[i] : 0;
            if (S[i].in_cycle && kreached[i] > 0) upd.push_back(i);
            if (S[i].in_cycle) S[i].inf.restarts += 1;
            S[i].in_cycle = false;
        }
        if (!upd.empty()) {
            SKO_HIP(hipMemcpyAsync(tbl_d, tbl_h, sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, g.st));
            if ((s = set_active(upd))) return s;
            g.phase(PhaseTimer::SMALL);
            const int ev2 = c->prof.begin("update x", g.rows_bytes * (m * eb + 16.0), g.st);
            SKO_HIP(launch_update_batched(g.f32, max_n, g.Q, m, g.y, g.st, br));
            c->prof.end(ev2, g.st);
        }
    }
    pt.stop(g.st);
    SKO_HIP(hipEventRecord(ev_total.b, g.st));
    SKO_HIP(hipEventSynchronize(ev_total.b));
    c->prof.flush();
    pt.flush();
    const double total_ms = ev_total.ms();
    sko_status first = SKO_OK;
    for (int32_t i = 0; i < nsys; ++i) {
        S[i].inf.t_total = total_ms * 1e-3;
        S[i].inf.t_spmv = pt.ms[PhaseTimer::SPMV] * 1e-3;
        S[i].inf.t_orth = pt.ms[PhaseTimer::ORTH] * 1e-3;
        S[i].inf.t_small = pt.ms[PhaseTimer::SMALL] * 1e-3;
        if (infos) infos[i] = S[i].inf;
        if (S[i].result != SKO_OK && first == SKO_OK) first = S[i].result;
    }
    return first;
}

}  // namespace sko
