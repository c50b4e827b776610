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
#include <chrono>
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
    double* dinv;
    CsrView A;
    double *Tin, *Tout, *g, *gw, *H, *y, *res, *beta, *bnorm, *coef;
    double *Cpan, *Yacc, *rt, *rho, *Gb, *Rh, *Rt, *C2b;
    BlockBufs bb;
    int* status;
    int grid_cap;
    // host (pinned)
    double* host;  // [0] res, [1] beta, [2] bnorm; status at host+4 as int
};

void* col_ptr(const GmCtx& g, int col) {
    return static_cast<char*>(g.Q) + (int64_t)col * g.ld * (g.f32 ? 4 : 8);
}

sko_status read_scalars(GmCtx& g, const double* dev, int count, int* status_out) {
    SKO_HIP(hipMemcpyAsync(g.host, dev, sizeof(double) * count, hipMemcpyDeviceToHost, g.st));
    SKO_HIP(hipMemcpyAsync(reinterpret_cast<int*>(g.host + 4), g.status, sizeof(int), hipMemcpyDeviceToHost, g.st));
    SKO_HIP(hipStreamSynchronize(g.st));
    g.c->prof.flush();
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
    for (int i = 1; i <= s; ++i) {
        const int ev = g.c->prof.begin(std::string("spmv ") + (g.f32 ? "f32" : "f64"),
                                       (double)g.A.nnz * (g.f32 ? 8.0 : 12.0) + (double)g.n * (g.f32 ? 12.0 : 20.0),
                                       g.st);
        SKO_HIP(launch_spmv(g.A, g.f32, col_ptr(g, from + i - 1), col_ptr(g, from + i), g.grid_cap, g.st));
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
    const int ev = g.c->prof.begin("gmres small", 0.0, g.st);
    SKO_HIP(launch_gm_small(a, g.st));
    g.c->prof.end(ev, g.st);
    return SKO_OK;
}

// One cycle; returns the basis size k reached (y[0:k] on the device), or 0 on breakdown.
sko_status cycle_one_stage(GmCtx& g, Engine& e, double bnorm, double tol, sko_gmres_info& inf, int64_t maxiter,
                           int* k_out) {
    int k = 0;
    sko_status s;
    while (k < g.m) {
        if ((s = mpk(g, k, g.s))) return s;
        void* Vk = col_ptr(g, k);
        if ((s = one_stage_block(e, g.bb, g.intra, k, g.Q, g.ld, Vk, g.ld, Vk, g.ld, g.coef, g.m + 1, k))) return s;
        GmSmallArgs a{};
        a.op = GM_BLOCK;
        a.kk = k;
        a.do_lsq = 1;
        if ((s = gm_op(g, a))) return s;
        int status = 0;
        if ((s = read_scalars(g, g.res, 1, &status))) return s;
        inf.iters += g.s;
        k += g.s;
        if (status) {
            inf.breakdown_col = status;
            *k_out = 0;
            return SKO_EBREAKDOWN;
        }
        inf.relres_implicit = g.host[0] / bnorm;
        if (inf.relres_implicit <= tol || inf.iters >= maxiter) break;
    }
    *k_out = k;
    return SKO_OK;
}

sko_status cycle_two_stage(GmCtx& g, Engine& e, double bnorm, double tol, sko_gmres_info& inf, int64_t maxiter,
                           int* k_out) {
    sko_status s;
    const int S = g.s, W = g.W, Wb = g.Wb, ld = (int)g.m + 1;
    const int red_sk = g.sk.kind == SKO_SKETCH_SPARSE_SIGN ? RED_SKETCH_SPARSE : RED_SKETCH_DENSE;
    const double sk_scale = g.sk.kind == SKO_SKETCH_SPARSE_SIGN ? 1.0 / std::sqrt((double)g.sk.zeta) : 1.0;
    int k0 = 0, k = 0;
    while (k0 < g.m) {
        void* Qb = col_ptr(g, k0);
        for (int i = 0; i < g.shat / S; ++i) {
            const int loc = i * S, kk = k0 + loc;
            if ((s = mpk(g, kk, S))) return s;
            void* V = col_ptr(g, kk);
            PassKey key{W, g.f32, red_sk, false, 0, false};
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
                if ((s = e.reduction({W, g.f32, RED_PROJ, false, 0, false}, pa, k0, V, g.ld, g.Q, g.ld, sm, 1.0)))
                    return s;
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
            sm.k = g.sk.k;
            sm.col0 = kk;
            sm.out = g.bb.Ysk;
            sm.R = g.rho;
            sm.Yacc = g.Yacc;
            sm.nacc = loc;
            sm.r = g.rt;
            sm.Rbar = g.coef + k0;
            sm.ldrbar = ld;
            sm.rbar_col0 = 0;
            if ((s = e.reduction(key, a, g.sk.k, V, g.ld, nullptr, 0, sm, sk_scale))) return s;
            PassArgs fa{};
            fa.Y = V;
            fa.ldy = g.ld;
            fa.R1 = g.rho;
            fa.X = V;
            fa.ldx = g.ld;
            PassKey fkey{W, g.f32, RED_NONE, false, 1, true};
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
            if ((s = gm_op(g, ga))) return s;
            inf.iters += S;
        }
        // big-panel close
        {
            SmallArgs sm{};
            sm.op = OP_CHOL;
            sm.w = Wb;
            sm.col0 = k0;
            sm.out = g.Gb;
            sm.R = g.Rh;
            if ((s = e.gemm_reduction(Qb, g.ld, Wb, Qb, g.ld, Wb, sm, Wb))) return s;
            if ((s = e.rowop(Wb, Qb, g.ld, nullptr, 0, 0, nullptr, g.Rh, Qb, g.ld))) return s;
        }
        const bool proj2 = g.reorth && k0 > 0;
        if (g.reorth) {
            if (proj2) {
                for (int a0 = 0; a0 < k0; a0 += 64) {
                    const int ma = std::min(64, k0 - a0);
                    SmallArgs sm{};
                    sm.op = OP_STORE;
                    sm.w = Wb;
                    sm.out = g.C2b + a0;
                    if ((s = e.gemm_reduction(col_ptr(g, a0), g.ld, ma, Qb, g.ld, Wb, sm, k0))) return s;
                }
                if ((s = e.rowop(Wb, Qb, g.ld, g.Q, g.ld, k0, g.C2b, nullptr, Qb, g.ld))) return s;
            }
            SmallArgs sm{};
            sm.op = OP_CHOL;
            sm.w = Wb;
            sm.col0 = k0;
            sm.out = g.Gb;
            sm.R = g.Rt;
            if ((s = e.gemm_reduction(Qb, g.ld, Wb, Qb, g.ld, Wb, sm, Wb))) return s;
            if ((s = e.rowop(Wb, Qb, g.ld, nullptr, 0, 0, nullptr, g.Rt, Qb, g.ld))) return s;
        }
        const int kend = k0 + g.shat;
        GmSmallArgs ga{};
        ga.op = GM_BIGCLOSE;
        ga.k0 = k0;
        ga.Wb = Wb;
        ga.kend = kend;
        ga.two_stage = 1;
        ga.Rh = g.Rh;
        ga.Rt = g.reorth ? g.Rt : nullptr;
        ga.C2 = proj2 ? g.C2b : nullptr;
        if ((s = gm_op(g, ga))) return s;
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

sko_status gmres_impl(sko_ctx c, const sko_csr* A, const double* b, double* x, const sko_gmres_opts* o,
                      sko_gmres_info* info) {
    sko_gmres_info inf{};
    if (info) *info = inf;
    if (!A || !b || !x || !o || !A->rowptr || !A->colind || !A->val || A->n < 1 || A->nnz < 1) return SKO_EINVAL;
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
    const int64_t maxiter = o->maxiter > 0 ? o->maxiter : 50000;

    GmCtx g{};
    g.c = c;
    g.st = c->stream;
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
    const int eb = g.f32 ? 4 : 8;
    const int k = need_sketch ? o->sketch.k : g.W;

    // ---- workspace
    Arena ar(c);
    const size_t o_Q = ar.reserve((size_t)eb * g.ld * (m + 1));
    const bool own_vals = g.jacobi || g.f32;
    const size_t o_val = own_vals ? ar.reserve((size_t)eb * A->nnz) : 0;
    const size_t o_dinv = g.jacobi ? ar.reserve(sizeof(double) * A->n) : 0;
    const int64_t nstrips = (A->n + kPassThreads - 1) / kPassThreads;
    const int gmax = (int)std::min<int64_t>(nstrips, (int64_t)std::max(1, c->cus) * 8);
    const int64_t rows = std::max({(int64_t)m, (int64_t)k, (int64_t)g.W});
    const int64_t part_stride = ((rows * g.W + 31) / 32) * 32;
    g.grid_cap = std::max(1, c->cus) * 8;
    const size_t part_doubles = std::max({(size_t)part_stride * gmax, (size_t)64 * 64 * std::max(1, skinny_gemm_grid_cap()),
                                          (size_t)g.grid_cap});
    const size_t o_part = ar.reserve(sizeof(double) * part_doubles);
    const int mW = m * g.W;
    const size_t o_bb = ar.reserve(sizeof(double) * (2 * (size_t)mW + (size_t)std::max(k, g.W) * g.W + 5 * g.W * g.W));
    const size_t o_gm = ar.reserve(sizeof(double) * (3 * (size_t)(m + 1) * m + 3 * (size_t)(m + 1) + 8 +
                                                     (size_t)(m + 1) * g.W));
    const size_t o_ts = two ? ar.reserve(sizeof(double) * ((size_t)mW + (size_t)k * g.Wb + (size_t)g.Wb * g.W +
                                                          g.W * g.W + 3 * (size_t)g.Wb * g.Wb + (size_t)m * g.Wb))
                            : 0;
    const size_t o_st = ar.reserve(256);
    sko_status s = ensure_workspace(c, ar.used());
    if (s) return s;
    if ((s = ensure_pinned(c, 64))) return s;
    g.host = static_cast<double*>(c->pinned);
    g.Q = ar.at<void>(o_Q);
    g.dinv = g.jacobi ? ar.at<double>(o_dinv) : nullptr;
    g.status = ar.at<int>(o_st);
    {
        double* p = ar.at<double>(o_bb);
        g.bb.C1 = p;
        g.bb.C2 = p + mW;
        g.bb.Ysk = g.bb.C2 + mW;
        g.bb.G2 = g.bb.Ysk + (int64_t)std::max(k, g.W) * g.W;
        g.bb.G3 = g.bb.G2 + g.W * g.W;
        g.bb.R1 = g.bb.G3 + g.W * g.W;
        g.bb.R2 = g.bb.R1 + g.W * g.W;
        g.bb.R3 = g.bb.R2 + g.W * g.W;
        double* q = ar.at<double>(o_gm);
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
        if (two) {
            double* t = ar.at<double>(o_ts);
            g.Cpan = t;
            g.Yacc = g.Cpan + mW;
            g.rt = g.Yacc + (int64_t)k * g.Wb;
            g.rho = g.rt + (int64_t)g.Wb * g.W;
            g.Gb = g.rho + g.W * g.W;
            g.Rh = g.Gb + g.Wb * g.Wb;
            g.Rt = g.Rh + g.Wb * g.Wb;
            g.C2b = g.Rt + g.Wb * g.Wb;
        }
    }

    hipEvent_t t0 = nullptr, t1 = nullptr;
    SKO_HIP(hipEventCreate(&t0));
    SKO_HIP(hipEventCreate(&t1));
    SKO_HIP(hipEventRecord(t0, g.st));
    SKO_HIP(hipMemsetAsync(g.status, 0, 256, g.st));
    c->tickets = 0;

    // ---- CSR structure check before any kernel indexes through it
    {
        int bad = 0;
        SKO_HIP(launch_csr_check(A->n, A->nnz, A->rowptr, A->colind, g.status + 32, g.st));
        SKO_HIP(hipMemcpyAsync(reinterpret_cast<int*>(g.host + 4), g.status + 32, sizeof(int), hipMemcpyDeviceToHost,
                               g.st));
        SKO_HIP(hipStreamSynchronize(g.st));
        bad = *reinterpret_cast<int*>(g.host + 4);
        if (bad) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return SKO_EINVAL;
        }
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
                ra.ticket0 = c->tickets;
                c->tickets += (unsigned)reduce_grid(1);
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
                if ((s = e1f.plain({1, g.f32, RED_NONE, false, 1, true}, a))) return s;
            }
            GmSmallArgs ia{};
            ia.op = GM_INIT;
            if ((s = gm_op(g, ia))) return s;
            int kreached = 0;
            s = two ? cycle_two_stage(g, e, bnorm, o->tol, inf, maxiter, &kreached)
                    : cycle_one_stage(g, e, bnorm, o->tol, inf, maxiter, &kreached);
            if (s == SKO_EBREAKDOWN) {
                result = s;
                break;
            }
            if (s) return s;
            {
                const int ev2 = c->prof.begin("update x", (double)A->n * (kreached * eb + 16.0), g.st);
                SKO_HIP(launch_update(A->n, g.f32, g.Q, g.ld, kreached, g.y, g.dinv, x, g.st));
                c->prof.end(ev2, g.st);
            }
            inf.restarts += 1;
        }
    }
    SKO_HIP(hipEventRecord(t1, g.st));
    SKO_HIP(hipEventSynchronize(t1));
    c->prof.flush();
    float ms = 0.f;
    SKO_HIP(hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    inf.t_total = ms * 1e-3;
    if (info) *info = inf;
    return result;
}

sko_status gmres_batched_impl(sko_ctx c, int32_t nsys, const sko_csr* A, const double* const* b, double* const* x,
                              const sko_gmres_opts* o, sko_gmres_info* infos) {
    if (nsys < 0 || (nsys > 0 && (!A || !b || !x || !o))) return SKO_EINVAL;
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

}  // namespace sko
