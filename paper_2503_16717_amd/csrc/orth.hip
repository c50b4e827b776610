// Block orthogonalisation on the device: one-stage BCGS2 (Fig. 2c) with a CholQR2
// (Section 5.1) or RandCholQR (Fig. 4b) first intra-block step, and the two-stage
// scheme with RandBCGS2 pre-processing (Figs. 6 and 8).
//
// Every step stays on the GPU: tall passes stream the n rows once each, the small
// dense factorisations run in the last workgroup of each reduction, and the R factor
// is assembled in device memory.  The host issues launches only and synchronises once
// at the end of a call to fetch R and the breakdown status.
//
// One-stage block j with p previous columns (passes are fused reads of the tall data):
//   P1  C1 = Q^T V                                    reduce -> C1
//   P2  Vh = V - Q C1 (written), sketch Y = Theta^T Vh (or Gram Vh^T Vh for CholQR2)
//                                                     reduce -> R1 = HH(Y) (or chol)
//   P3  Qb = Vh R1^{-1} (not stored), G2 = Qb^T Qb    reduce -> R2 = chol(G2)
//   P4  Qh = Vh R1^{-1} R2^{-1} (written), C2 = Q^T Qh reduce -> C2
//   P5  Vb = Qh - Q C2 (written), G3 = Vb^T Vb        reduce -> R3 = chol(G3), assemble R
//   P6  Qj = Vb R3^{-1} (written)
// With p = 0 the projections vanish: P2 reads V directly, P4 accumulates G3 = Qh^T Qh.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"

namespace sko {



// One-stage BCGS2 block: V (n x W) against Q (n x p) -> Qo; R columns assembled at
// Rcol (device, rows 0..p+W-1, leading dimension ldr).
sko_status one_stage_block_recursive(Engine& e, const BlockBufs& b, int p, const void* Q, int64_t ldq,
                                     const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rcol,
                                     int64_t ldr, int col0);

sko_status one_stage_block(Engine& e, const BlockBufs& b, int intra, int p, const void* Q, int64_t ldq,
                           const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rcol, int64_t ldr,
                           int col0) {
    if (intra == SKO_INTRA_CHOLQR2_RECURSIVE)
        return one_stage_block_recursive(e, b, p, Q, ldq, V, ldv, Qo, ldqo, Rcol, ldr, col0);
    const int W = e.W;
    const bool f32 = e.f32;
    const bool rand = intra == SKO_INTRA_RANDCHOLQR;
    const SketchPlan sp = sketch_plan(e.sk);
    const int red_first = rand ? sp.red : RED_GRAM;
    const int rows_first = rand ? sp.rows : W;
    const double sk_scale = rand ? sp.scale : 1.0;
    sko_status s;

    // P1: C1 = Q^T V
    if (p > 0) {
        PassArgs a{};
        a.Y = V;
        a.ldy = ldv;
        SmallArgs sm{};
        sm.op = OP_STORE;
        sm.w = W;
        sm.out = b.C1;
        if ((s = e.reduction({W, f32, RED_PROJ, false, 0, false}, a, p, V, ldv, Q, ldq, sm, 1.0))) return s;
    }
    // P2: Vh = V - Q C1 (written to Qo), reduction for the first intra-block step
    const void* Vh = V;
    int64_t ldvh = ldv;
    {
        PassArgs a{};
        a.Y = V;
        a.ldy = ldv;
        PassKey key{W, f32, red_first, false, 0, false};
        if (p > 0) {
            key.upd = true;
            key.write = true;
            a.Qu = Q;
            a.ldqu = ldq;
            a.pu = p;
            a.Cu = b.C1;
            a.X = Qo;
            a.ldx = ldqo;
            Vh = Qo;
            ldvh = ldqo;
        }
        SmallArgs sm{};
        sm.op = rand ? OP_HH : OP_CHOL;
        sm.w = W;
        sm.k = rand ? sp.k : W;
        sm.col0 = col0;
        sm.out = b.Ysk;
        sm.R = b.R1;
        if (rand) sketch_small(sm, sp);
        if ((s = e.reduction(key, a, rows_first, Vh, ldvh, nullptr, 0, sm, sk_scale))) return s;
    }
    // P3: G2 = (Vh R1^{-1})^T (Vh R1^{-1})
    {
        PassArgs a{};
        a.Y = Vh;
        a.ldy = ldvh;
        a.R1 = b.R1;
        SmallArgs sm{};
        sm.op = OP_CHOL;
        sm.w = W;
        sm.col0 = col0;
        sm.out = b.G2;
        sm.R = b.R2;
        // later Gram chunks (W > rows per launch) recompute the solve from Vh: re-run the
        // same keyed pass rather than an identity pass, since Qb is not stored.
        const int rpl = pass_rows_per_launch(W, RED_GRAM);
        if (W <= rpl) {
            if ((s = e.reduction({W, f32, RED_GRAM, false, 1, false}, a, W, nullptr, 0, nullptr, 0, sm, 1.0)))
                return s;
        } else {
            return SKO_EUNSUPPORTED;
        }
    }
    // P4: Qh = Vh R1^{-1} R2^{-1} written to Qo; C2 = Q^T Qh (or G3 = Qh^T Qh when p = 0)
    {
        PassArgs a{};
        a.Y = Vh;
        a.ldy = ldvh;
        a.R1 = b.R1;
        a.R2 = b.R2;
        a.X = Qo;
        a.ldx = ldqo;
        SmallArgs sm{};
        sm.w = W;
        sm.col0 = col0;
        if (p > 0) {
            sm.op = OP_STORE;
            sm.out = b.C2;
            if ((s = e.reduction({W, f32, RED_PROJ, false, 2, true}, a, p, Qo, ldqo, Q, ldq, sm, 1.0))) return s;
        } else {
            sm.op = OP_CHOL;
            sm.out = b.G3;
            sm.R = b.R3;
            sm.assemble = 1;
            sm.Ra = b.R2;
            sm.Rb = b.R1;
            sm.p = 0;
            sm.Rout = Rcol;
            sm.ldr = ldr;
            if ((s = e.reduction({W, f32, RED_GRAM, false, 2, true}, a, W, Qo, ldqo, nullptr, 0, sm, 1.0)))
                return s;
        }
    }
    // P5: Vb = Qh - Q C2 written in place; G3 = Vb^T Vb; R3 = chol(G3); assemble R
    if (p > 0) {
        PassArgs a{};
        a.Y = Qo;
        a.ldy = ldqo;
        a.Qu = Q;
        a.ldqu = ldq;
        a.pu = p;
        a.Cu = b.C2;
        a.X = Qo;
        a.ldx = ldqo;
        SmallArgs sm{};
        sm.op = OP_CHOL;
        sm.w = W;
        sm.col0 = col0;
        sm.out = b.G3;
        sm.R = b.R3;
        sm.assemble = 1;
        sm.Ra = b.R2;
        sm.Rb = b.R1;
        sm.C1 = b.C1;
        sm.C2 = b.C2;
        sm.p = p;
        sm.Rout = Rcol;
        sm.ldr = ldr;
        if ((s = e.reduction({W, f32, RED_GRAM, true, 0, true}, a, W, Qo, ldqo, nullptr, 0, sm, 1.0))) return s;
    }
    // P6: Qj = Vb R3^{-1}
    {
        PassArgs a{};
        a.Y = Qo;
        a.ldy = ldqo;
        a.R1 = b.R3;
        a.X = Qo;
        a.ldx = ldqo;
        if ((s = e.plain({W, f32, RED_NONE, false, 1, true}, a))) return s;
    }
    return SKO_OK;
}

namespace {

// The host reads a device status word (one synchronisation of the stream).
sko_status read_status(Engine& e, const int* word, int* out) {
    SKO_HIP(hipMemcpyAsync(e.c->status_host, word, sizeof(int), hipMemcpyDeviceToHost, e.st));
    SKO_HIP(hipStreamSynchronize(e.st));
    *out = *e.c->status_host;
    return SKO_OK;
}

// Copy a rows x cols block of doubles between device matrices (column-major).
hipError_t copy_block(double* dst, int64_t ldd, const double* src, int64_t lds, int rows, int cols, hipStream_t st) {
    if (rows < 1 || cols < 1) return hipSuccess;
    return hipMemcpy2DAsync(dst, sizeof(double) * ldd, src, sizeof(double) * lds, sizeof(double) * rows, cols,
                            hipMemcpyDeviceToDevice, st);
}

// Recursive CholQR (Fig. 3) of the w columns at X, in place, R (w x w, ld w) on the device.
// G, Rseg: w x w scratch; Rc, Cc: the compact partial factors; probe: a status word the
// host reads after every Cholesky (the global status word gets a breakdown only for a
// column that fails as the first of a recursion, i.e. is dependent on the ones before it).
sko_status cholqr_recursive_dev(Engine& e, void* X, int64_t ldx, int w, double* R, int col0, double* G,
                                double* Rseg, double* Rc, double* Cc, int* probe) {
    const bool f32 = e.f32;
    SKO_HIP(launch_zero(R, sizeof(double) * (size_t)w * w, e.st));
    int c0 = 0;
    while (c0 < w) {
        const int ws = w - c0;
        void* Xc = offset_elems(X, (int64_t)c0 * ldx, f32);
        Engine es = e;
        es.W = ws;
        es.status = probe;
        SKO_HIP(launch_zero(probe, sizeof(int), e.st));
        PassArgs a{};
        a.Y = Xc;
        a.ldy = ldx;
        SmallArgs sm{};
        sm.op = OP_CHOL;
        sm.w = ws;
        sm.col0 = col0 + c0;
        sm.out = G;
        sm.R = Rseg;
        sko_status s;
        if ((s = es.reduction({ws, f32, RED_GRAM, false, 0, false}, a, ws, nullptr, 0, nullptr, 0, sm, 1.0))) return s;
        int fail = 0;
        if ((s = read_status(e, probe, &fail))) return s;
        const int k = fail ? fail - (col0 + c0) : 0;  // 1-based within this segment
        if (k == 0) {
            PassArgs t{};
            t.Y = Xc;
            t.ldy = ldx;
            t.R1 = Rseg;
            t.X = Xc;
            t.ldx = ldx;
            if ((s = es.plain({ws, f32, RED_NONE, false, 1, true}, t))) return s;
            SKO_HIP(copy_block(R + c0 + (int64_t)c0 * w, w, Rseg, ws, ws, ws, e.st));
            return SKO_OK;
        }
        if (k == 1) {  // the segment's first column depends on the columns before it
            const int col = col0 + c0 + 1;
            SKO_HIP(hipMemcpyAsync(e.status, &col, sizeof(int), hipMemcpyHostToDevice, e.st));
            SKO_HIP(hipStreamSynchronize(e.st));
            return SKO_EBREAKDOWN;
        }
        const int m1 = k - 1;
        // the first m1 rows of the partial factor: [R11 R12]
        SKO_HIP(copy_block(Rc, m1, Rseg, ws, m1, m1, e.st));
        SKO_HIP(copy_block(Cc, m1, Rseg + (int64_t)m1 * ws, ws, m1, ws - m1, e.st));
        SKO_HIP(copy_block(R + c0 + (int64_t)c0 * w, w, Rseg, ws, m1, ws, e.st));
        {   // Q1 = X1 R11^{-1}
            Engine e1 = e;
            e1.W = m1;
            PassArgs t{};
            t.Y = Xc;
            t.ldy = ldx;
            t.R1 = Rc;
            t.X = Xc;
            t.ldx = ldx;
            if ((s = e1.plain({m1, f32, RED_NONE, false, 1, true}, t))) return s;
        }
        {   // X2 <- X2 - Q1 R12
            Engine e2 = e;
            e2.W = ws - m1;
            void* X2 = offset_elems(Xc, (int64_t)m1 * ldx, f32);
            PassArgs t{};
            t.Y = X2;
            t.ldy = ldx;
            t.Qu = Xc;
            t.ldqu = ldx;
            t.pu = m1;
            t.Cu = Cc;
            t.X = X2;
            t.ldx = ldx;
            if ((s = e2.plain({ws - m1, f32, RED_NONE, true, 0, true}, t))) return s;
        }
        c0 += m1;
    }
    return SKO_OK;
}

}  // namespace

// One-stage BCGS2 block with the recursive CholQR2 first intra step and a recursive final
// CholQR (unfused passes; the host reads every Cholesky's status).
sko_status one_stage_block_recursive(Engine& e, const BlockBufs& b, int p, const void* Q, int64_t ldq,
                                     const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rcol,
                                     int64_t ldr, int col0) {
    const int W = e.W;
    const bool f32 = e.f32;
    int* probe = e.status + 8;
    sko_status s;
    if (p > 0) {
        PassArgs a{};
        a.Y = V;
        a.ldy = ldv;
        SmallArgs sm{};
        sm.op = OP_STORE;
        sm.w = W;
        sm.out = b.C1;
        if ((s = e.reduction({W, f32, RED_PROJ, false, 0, false}, a, p, V, ldv, Q, ldq, sm, 1.0))) return s;
        PassArgs u{};
        u.Y = V;
        u.ldy = ldv;
        u.Qu = Q;
        u.ldqu = ldq;
        u.pu = p;
        u.Cu = b.C1;
        u.X = Qo;
        u.ldx = ldqo;
        if ((s = e.plain({W, f32, RED_NONE, true, 0, true}, u))) return s;
    } else if (Qo != V || ldqo != ldv) {
        const size_t eb = f32 ? 4 : 8;
        SKO_HIP(hipMemcpy2DAsync(Qo, eb * ldqo, V, eb * ldv, eb * e.n, W, hipMemcpyDeviceToDevice, e.st));
    }
    if ((s = cholqr_recursive_dev(e, Qo, ldqo, W, b.R1, col0, b.G2, b.G3, b.S1, b.S2, probe))) return s;
    if ((s = cholqr_recursive_dev(e, Qo, ldqo, W, b.R2, col0, b.G2, b.G3, b.S1, b.S2, probe))) return s;
    if (p > 0) {
        PassArgs a{};
        a.Y = Qo;
        a.ldy = ldqo;
        SmallArgs sm{};
        sm.op = OP_STORE;
        sm.w = W;
        sm.out = b.C2;
        if ((s = e.reduction({W, f32, RED_PROJ, false, 0, false}, a, p, Qo, ldqo, Q, ldq, sm, 1.0))) return s;
        PassArgs u{};
        u.Y = Qo;
        u.ldy = ldqo;
        u.Qu = Q;
        u.ldqu = ldq;
        u.pu = p;
        u.Cu = b.C2;
        u.X = Qo;
        u.ldx = ldqo;
        if ((s = e.plain({W, f32, RED_NONE, true, 0, true}, u))) return s;
    }
    if ((s = cholqr_recursive_dev(e, Qo, ldqo, W, b.R3, col0, b.G2, b.G3, b.S1, b.S2, probe))) return s;
    SmallArgs as{};
    as.w = W;
    as.R = b.R3;
    as.Ra = b.R2;
    as.Rb = b.R1;
    as.C1 = p > 0 ? b.C1 : nullptr;
    as.C2 = p > 0 ? b.C2 : nullptr;
    as.p = p;
    as.Rout = Rcol;
    as.ldr = ldr;
    SKO_HIP(launch_assemble(as, b.G2, e.st));
    return SKO_OK;
}

bool sketch_ok(const sko_sketch& sk, int64_t n) {
    if (sk.k < 1 || sk.k > 256) return false;
    auto hashed_ok = [&](int rows) {
        return sk.zeta >= 1 && sk.zeta <= 8 && rows % sk.zeta == 0 && rows / sk.zeta <= 128;
    };
    if (sk.kind == SKO_SKETCH_SPARSE_SIGN) return hashed_ok(sk.k);
    if (sk.kind == SKO_SKETCH_GAUSSIAN) return sk.theta != nullptr && sk.ld_theta >= n;
    if (sk.kind == SKO_SKETCH_COUNT_GAUSS)
        return sk.k_count >= sk.k && sk.k_count <= 256 && hashed_ok(sk.k_count) && sk.theta != nullptr &&
               sk.ld_theta >= sk.k_count;
    return false;
}

SketchPlan sketch_plan(const sko_sketch& sk) {
    SketchPlan p{};
    p.k = sk.k;
    p.rows = sk.k;
    if (sk.kind == SKO_SKETCH_GAUSSIAN) {
        p.red = RED_SKETCH_DENSE;
        p.scale = 1.0;
        return p;
    }
    p.red = RED_SKETCH_SPARSE;
    p.scale = sk.zeta > 0 ? 1.0 / std::sqrt((double)sk.zeta) : 1.0;
    if (sk.kind == SKO_SKETCH_COUNT_GAUSS) {
        p.rows = sk.k_count;
        p.theta_g = sk.theta;
        p.ld_g = sk.ld_theta;
    }
    return p;
}

namespace {

// Workspace sizing shared by the one-stage entry points.
struct OneStageLayout {
    size_t partials, small, rfull, status, total;
    int64_t part_stride;
    int gmax;
};

OneStageLayout layout_one_stage(sko_ctx c, int64_t n, int W, int pmax, int k, int N) {
    OneStageLayout L{};
    Arena ar(c);
    const int64_t nstrips = (n + kPassThreads - 1) / kPassThreads;
    L.gmax = (int)std::min<int64_t>(nstrips, (int64_t)std::max(1, c->cus) * 8);
    int64_t rows = std::max({(int64_t)pmax, (int64_t)k, (int64_t)W});
    L.part_stride = ((rows * W + 31) / 32) * 32;
    L.partials = ar.reserve(sizeof(double) * L.part_stride * L.gmax);
    const int64_t cw = std::max<int64_t>(1, (int64_t)pmax * W);
    L.small = ar.reserve(sizeof(double) * (2 * cw + (int64_t)std::max(k, W) * W + 7 * W * W));
    L.rfull = ar.reserve(sizeof(double) * (int64_t)std::max(1, N) * std::max(1, N));
    L.status = ar.reserve(256);
    L.total = ar.used();
    return L;
}

BlockBufs carve(const Arena& ar, const OneStageLayout& L, int pmax, int k, int W) {
    double* base = ar.at<double>(L.small);
    const int64_t cw = std::max<int64_t>(1, (int64_t)pmax * W);
    BlockBufs b{};
    b.C1 = base;
    b.C2 = b.C1 + cw;
    b.Ysk = b.C2 + cw;
    b.G2 = b.Ysk + (int64_t)std::max(k, W) * W;
    b.G3 = b.G2 + W * W;
    b.R1 = b.G3 + W * W;
    b.R2 = b.R1 + W * W;
    b.R3 = b.R2 + W * W;
    b.S1 = b.R3 + W * W;
    b.S2 = b.S1 + W * W;
    return b;
}

sko_status finish(sko_ctx c, int* status_dev, int32_t* breakdown_col) {
    SKO_HIP(hipMemcpyAsync(c->status_host, status_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SKO_HIP(hipStreamSynchronize(c->stream));
    c->prof.flush();
    const int col = *c->status_host;
    if (breakdown_col) *breakdown_col = col;
    return col ? SKO_EBREAKDOWN : SKO_OK;
}

}  // namespace

sko_status two_stage_blocks(sko_ctx c, int64_t n, int32_t nb, int32_t w, const void* V, int64_t ldv,
                            void* Q, int64_t ldq, double* R, int64_t ldr, const sko_orth_opts* o,
                            int32_t* breakdown_col);

sko_status orth_blocks_impl(sko_ctx c, int64_t n, int32_t nb, int32_t w, const void* V, int64_t ldv, void* Q,
                            int64_t ldq, double* R, int64_t ldr, const sko_orth_opts* o,
                            int32_t* breakdown_col) {
    if (breakdown_col) *breakdown_col = 0;
    if (!o || !V || !Q || n < 1 || nb < 1 || w < 1 || w > kMaxPassW || ldv < n || ldq < n) return SKO_EINVAL;
    if (o->precision != SKO_F64 && o->precision != SKO_MIXED_F32) return SKO_EINVAL;
    const int N = nb * w;
    if (R && ldr < N) return SKO_EINVAL;
    if (o->two_stage && o->preproc != SKO_PREPROC_RANDBCGS2 && o->preproc != SKO_PREPROC_PIP) return SKO_EINVAL;
    const bool rand = o->two_stage ? o->preproc == SKO_PREPROC_RANDBCGS2 : o->intra == SKO_INTRA_RANDCHOLQR;
    if (!o->two_stage && o->intra != SKO_INTRA_RANDCHOLQR && o->intra != SKO_INTRA_CHOLQR2 &&
        o->intra != SKO_INTRA_CHOLQR2_RECURSIVE)
        return SKO_EINVAL;
    if (rand && !sketch_ok(o->sketch, n)) return SKO_EINVAL;
    if (rand && o->sketch.k < w) return SKO_EINVAL;
    if (w > pass_rows_per_launch(w, RED_GRAM)) return SKO_EUNSUPPORTED;
    if (o->two_stage) return two_stage_blocks(c, n, nb, w, V, ldv, Q, ldq, R, ldr, o, breakdown_col);
    if ((int64_t)(N - w) * w > kMaxUpdCoef) return SKO_EUNSUPPORTED;

    const bool f32 = o->precision == SKO_MIXED_F32;
    const int k = rand ? sketch_plan(o->sketch).rows : w;
    OneStageLayout L = layout_one_stage(c, n, w, N - w, k, N);
    sko_status s = ensure_workspace(c, L.total);
    if (s) return s;
    Arena ar(c);
    Engine e(c, n, w, f32, o->sketch);
    e.partials = ar.at<double>(L.partials);
    e.part_stride = L.part_stride;
    e.gmax = L.gmax;
    e.status = ar.at<int>(L.status);
    e.counter = reinterpret_cast<unsigned*>(e.status + 16);
    double* Rfull = ar.at<double>(L.rfull);
    SKO_HIP(launch_zero(e.status, 256, c->stream));
    SKO_HIP(launch_zero(Rfull, sizeof(double) * (size_t)N * N, c->stream));
    BlockBufs bb = carve(ar, L, N - w, k, w);
    for (int j = 0; j < nb; ++j) {
        const int p = j * w;
        const void* Vj = offset_elems(V, (int64_t)p * ldv, f32);
        void* Qj = offset_elems(Q, (int64_t)p * ldq, f32);
        s = one_stage_block(e, bb, o->intra, p, Q, ldq, Vj, ldv, Qj, ldq, Rfull + (int64_t)p * N, N, p);
        // the recursive CholQR stops at a dependent column; its column is in the status word
        if (s == SKO_EBREAKDOWN) return finish(c, e.status, breakdown_col);
        if (s) return s;
    }
    double* Rh = nullptr;
    if (R) {
        if ((s = ensure_pinned(c, sizeof(double) * (size_t)N * N))) return s;
        Rh = static_cast<double*>(c->pinned);
        SKO_HIP(hipMemcpyAsync(Rh, Rfull, sizeof(double) * (size_t)N * N, hipMemcpyDeviceToHost, c->stream));
    }
    if ((s = finish(c, e.status, breakdown_col)) && s != SKO_EBREAKDOWN) return s;
    if (R)
        for (int jc = 0; jc < N; ++jc) std::memcpy(R + (int64_t)jc * ldr, Rh + (int64_t)jc * N, sizeof(double) * N);
    return s;
}

namespace {

sko_status orth_block_check(int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq, const void* V, int64_t ldv,
                            const void* Qo, int64_t ldqo, const sko_orth_opts* o) {
    if (!o || !V || !Qo || n < 1 || p < 0 || w < 1 || w > kMaxPassW || ldv < n || ldqo < n) return SKO_EINVAL;
    if (p > 0 && (!Q || ldq < n)) return SKO_EINVAL;
    if (o->two_stage) return SKO_EINVAL;
    if (o->precision != SKO_F64 && o->precision != SKO_MIXED_F32) return SKO_EINVAL;
    if (o->intra != SKO_INTRA_RANDCHOLQR && o->intra != SKO_INTRA_CHOLQR2 && o->intra != SKO_INTRA_CHOLQR2_RECURSIVE)
        return SKO_EINVAL;
    const bool rand = o->intra == SKO_INTRA_RANDCHOLQR;
    if (rand && (!sketch_ok(o->sketch, n) || o->sketch.k < w)) return SKO_EINVAL;
    if ((int64_t)p * w > kMaxUpdCoef) return SKO_EUNSUPPORTED;
    if (w > pass_rows_per_launch(w, RED_GRAM)) return SKO_EUNSUPPORTED;
    return SKO_OK;
}

// The block step on the workspace of arena `ar` laid out as L; leaves the assembled
// [R_proj; R_diag] ((p + w) x w, leading dimension p + w) at *Rcol_out on the device.
sko_status orth_block_run(sko_ctx c, const Arena& ar, const OneStageLayout& L, Engine& e, int64_t n, int32_t p,
                          int32_t w, const void* Q, int64_t ldq, const void* V, int64_t ldv, void* Qo, int64_t ldqo,
                          const sko_orth_opts* o, double** Rcol_out) {
    const bool rand = o->intra == SKO_INTRA_RANDCHOLQR;
    const int k = rand ? sketch_plan(o->sketch).rows : w;
    e.partials = ar.at<double>(L.partials);
    e.part_stride = L.part_stride;
    e.gmax = L.gmax;
    e.status = ar.at<int>(L.status);
    e.counter = reinterpret_cast<unsigned*>(e.status + 16);
    double* Rcol = ar.at<double>(L.rfull);  // (p + w) x w, ld p + w
    SKO_HIP(launch_zero(e.status, 256, c->stream));
    BlockBufs bb = carve(ar, L, p, k, w);
    *Rcol_out = Rcol;
    return one_stage_block(e, bb, o->intra, p, Q, ldq, V, ldv, Qo, ldqo, Rcol, p + w, 0);
}

}  // namespace

sko_status orth_block_impl(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq, const void* V,
                           int64_t ldv, void* Qo, int64_t ldqo, double* Rp, double* Rd, const sko_orth_opts* o,
                           int32_t* breakdown_col) {
    if (breakdown_col) *breakdown_col = 0;
    sko_status s = orth_block_check(n, p, w, Q, ldq, V, ldv, Qo, ldqo, o);
    if (s) return s;
    const bool f32 = o->precision == SKO_MIXED_F32;
    const int k = o->intra == SKO_INTRA_RANDCHOLQR ? sketch_plan(o->sketch).rows : w;
    const int N = p + w;
    OneStageLayout L = layout_one_stage(c, n, w, p, k, N);
    if ((s = ensure_workspace(c, L.total))) return s;
    Arena ar(c);
    Engine e(c, n, w, f32, o->sketch);
    double* Rcol = nullptr;
    s = orth_block_run(c, ar, L, e, n, p, w, Q, ldq, V, ldv, Qo, ldqo, o, &Rcol);
    if (s == SKO_EBREAKDOWN) return finish(c, e.status, breakdown_col);
    if (s) return s;
    if ((s = ensure_pinned(c, sizeof(double) * (size_t)N * w))) return s;
    double* Rh = static_cast<double*>(c->pinned);
    SKO_HIP(hipMemcpyAsync(Rh, Rcol, sizeof(double) * (size_t)N * w, hipMemcpyDeviceToHost, c->stream));
    if ((s = finish(c, e.status, breakdown_col)) && s != SKO_EBREAKDOWN) return s;
    for (int jc = 0; jc < w; ++jc) {
        if (Rp && p > 0) std::memcpy(Rp + (int64_t)jc * p, Rh + (int64_t)jc * N, sizeof(double) * p);
        if (Rd) std::memcpy(Rd + (int64_t)jc * w, Rh + (int64_t)jc * N + p, sizeof(double) * w);
    }
    return s;
}

// The same block step on the device's fixed scratch (noalloc.hip) instead of the context's
// workspace: no device or pinned allocation, no profiler bookkeeping; R goes straight into
// the caller's host arrays.
sko_status orth_block_noalloc_impl(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq,
                                   const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rp, double* Rd,
                                   const sko_orth_opts* o, int32_t* breakdown_col) {
    if (breakdown_col) *breakdown_col = 0;
    sko_status s = orth_block_check(n, p, w, Q, ldq, V, ldv, Qo, ldqo, o);
    if (s) return s;
    void* scratch = noalloc_scratch(c->device);
    if (!scratch) return SKO_EDEVICE;
    const bool f32 = o->precision == SKO_MIXED_F32;
    const int k = o->intra == SKO_INTRA_RANDCHOLQR ? sketch_plan(o->sketch).rows : w;
    const int N = p + w;
    OneStageLayout L = layout_one_stage(c, n, w, p, k, N);
    if (L.total > kNoallocScratchBytes) return SKO_ESCRATCH;
    Arena ar(c, scratch);
    Engine e(c, n, w, f32, o->sketch);
    e.profile = false;
    double* Rcol = nullptr;
    s = orth_block_run(c, ar, L, e, n, p, w, Q, ldq, V, ldv, Qo, ldqo, o, &Rcol);
    if (s == SKO_EBREAKDOWN) {
        SKO_HIP(hipMemcpyAsync(c->status_host, e.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        SKO_HIP(hipStreamSynchronize(c->stream));
        if (breakdown_col) *breakdown_col = *c->status_host;
        return s;
    }
    if (s) return s;
    if (Rp && p > 0)
        SKO_HIP(hipMemcpy2DAsync(Rp, sizeof(double) * p, Rcol, sizeof(double) * N, sizeof(double) * p, w,
                                 hipMemcpyDeviceToHost, c->stream));
    if (Rd)
        SKO_HIP(hipMemcpy2DAsync(Rd, sizeof(double) * w, Rcol + p, sizeof(double) * N, sizeof(double) * w, w,
                                 hipMemcpyDeviceToHost, c->stream));
    SKO_HIP(hipMemcpyAsync(c->status_host, e.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SKO_HIP(hipStreamSynchronize(c->stream));
    const int col = *c->status_host;
    if (breakdown_col) *breakdown_col = col;
    return col ? SKO_EBREAKDOWN : SKO_OK;
}

// Y = Theta^T X (Section 3), the reduction of the update + sketch pass on its own: the same
// kernels, slot decode and partial-sum order as the sketch of a RandCholQR or two-stage step.
sko_status sketch_apply_impl(sko_ctx c, int64_t n, int32_t w, const void* X, int64_t ldx, int32_t precision,
                             const sko_sketch* sk, double* Y, int64_t ldy) {
    if (!X || !sk || !Y || n < 1 || w < 1 || w > kMaxPassW || ldx < n) return SKO_EINVAL;
    if (precision != SKO_F64 && precision != SKO_MIXED_F32) return SKO_EINVAL;
    if (!sketch_ok(*sk, n) || ldy < sk->k) return SKO_EINVAL;
    const bool f32 = precision == SKO_MIXED_F32;
    const SketchPlan sp = sketch_plan(*sk);
    const int k = sk->k;
    // the C1 region (sized for pmax = k rows) receives a Count-Gauss product
    OneStageLayout L = layout_one_stage(c, n, w, k, sp.rows, w);
    sko_status s = ensure_workspace(c, L.total);
    if (s) return s;
    Arena ar(c);
    Engine e(c, n, w, f32, *sk);
    e.partials = ar.at<double>(L.partials);
    e.part_stride = L.part_stride;
    e.gmax = L.gmax;
    e.status = ar.at<int>(L.status);
    e.counter = reinterpret_cast<unsigned*>(e.status + 16);
    SKO_HIP(launch_zero(e.status, 256, c->stream));
    BlockBufs bb = carve(ar, L, k, sp.rows, w);
    PassArgs a{};
    a.Y = X;
    a.ldy = ldx;
    SmallArgs sm{};
    sm.op = OP_STORE;
    sm.w = w;
    sm.k = k;
    sm.out = bb.Ysk;
    sm.R = bb.C1;
    sketch_small(sm, sp);
    if ((s = e.reduction({w, f32, sp.red, false, 0, false}, a, sp.rows, X, ldx, nullptr, 0, sm, sp.scale))) return s;
    const double* Ydev = sp.theta_g ? bb.C1 : bb.Ysk;
    if ((s = ensure_pinned(c, sizeof(double) * (size_t)k * w))) return s;
    double* Yh = static_cast<double*>(c->pinned);
    SKO_HIP(hipMemcpyAsync(Yh, Ydev, sizeof(double) * (size_t)k * w, hipMemcpyDeviceToHost, c->stream));
    if ((s = finish(c, e.status, nullptr))) return s;
    for (int jc = 0; jc < w; ++jc) std::memcpy(Y + (int64_t)jc * ldy, Yh + (int64_t)jc * k, sizeof(double) * k);
    return SKO_OK;
}

sko_status two_stage_blocks(sko_ctx c, int64_t n, int32_t nb, int32_t w, const void* V, int64_t ldv, void* Q,
                            int64_t ldq, double* R, int64_t ldr, const sko_orth_opts* o, int32_t* breakdown_col) {
    const int ppb = o->panels_per_big;
    if (ppb < 1 || nb % ppb) return SKO_EINVAL;
    const int Wb = ppb * w;
    if (Wb > 64) return SKO_EUNSUPPORTED;
    const bool pip = o->preproc == SKO_PREPROC_PIP;
    if (!pip && o->sketch.k < Wb) return SKO_EINVAL;  // the big panel must embed into the sketch space
    const bool f32 = o->precision == SKO_MIXED_F32;
    const int N = nb * w;
    const SketchPlan sp = pip ? SketchPlan{RED_NONE, 0, 0, 1.0, nullptr, 0} : sketch_plan(o->sketch);
    const int k = sp.k;        // rows of the accumulated sketches
    // rows the passes reduce (BCGS-PIP: the projection on the previous panels of the big panel)
    const int kr = pip ? Wb - w : sp.rows;
    const int pmax = N - Wb;  // largest previous-basis width
    if ((int64_t)(Wb - w) * w > kMaxUpdCoef || (int64_t)pmax * w > kMaxUpdCoef) return SKO_EUNSUPPORTED;

    // workspace
    Arena ar(c);
    const int64_t nstrips = (n + kPassThreads - 1) / kPassThreads;
    const int gmax = (int)std::min<int64_t>(nstrips, (int64_t)std::max(1, c->cus) * 8);
    const int64_t rows = std::max({(int64_t)pmax, (int64_t)kr, (int64_t)w});
    const int64_t part_stride = ((rows * w + 31) / 32) * 32;
    const size_t part_doubles =
        std::max<size_t>((size_t)part_stride * gmax, (size_t)64 * 64 * std::max(1, skinny_gemm_grid_cap()));
    const size_t o_part = ar.reserve(sizeof(double) * part_doubles);
    const int64_t pw = std::max<int64_t>(1, (int64_t)pmax * Wb);
    const size_t o_C = ar.reserve(sizeof(double) * pw);
    const size_t o_C2 = ar.reserve(sizeof(double) * pw);
    const size_t o_Y = ar.reserve(sizeof(double) * (size_t)std::max(kr, w) * w);
    const size_t o_Gp = ar.reserve(sizeof(double) * (size_t)w * w);
    const size_t o_Yacc = ar.reserve(sizeof(double) * (size_t)k * Wb);
    const size_t o_r = ar.reserve(sizeof(double) * (size_t)Wb * w);
    const size_t o_rho = ar.reserve(sizeof(double) * (size_t)w * w);
    const size_t o_Rbar = ar.reserve(sizeof(double) * (size_t)Wb * Wb);
    const size_t o_G = ar.reserve(sizeof(double) * (size_t)Wb * Wb);
    const size_t o_Rh = ar.reserve(sizeof(double) * (size_t)Wb * Wb);
    const size_t o_Rt = ar.reserve(sizeof(double) * (size_t)Wb * Wb);
    const size_t o_Rpk = ar.reserve(sizeof(double) * (size_t)Wb * (Wb + 1) / 2);
    const size_t o_Rf = ar.reserve(sizeof(double) * (size_t)N * N);
    const size_t o_st = ar.reserve(256);
    sko_status s = ensure_workspace(c, ar.used());
    if (s) return s;
    Engine e(c, n, w, f32, o->sketch);
    e.partials = ar.at<double>(o_part);
    e.part_stride = part_stride;
    e.gmax = gmax;
    e.status = ar.at<int>(o_st);
    e.counter = reinterpret_cast<unsigned*>(e.status + 16);
    double* C = ar.at<double>(o_C);
    double* C2 = ar.at<double>(o_C2);
    double* Ysk = ar.at<double>(o_Y);
    double* Gpip = ar.at<double>(o_Gp);
    double* Yacc = ar.at<double>(o_Yacc);
    double* rt = ar.at<double>(o_r);
    double* rho = ar.at<double>(o_rho);
    double* Rbar = ar.at<double>(o_Rbar);
    double* Gb = ar.at<double>(o_G);
    double* Rh = ar.at<double>(o_Rh);
    double* Rt = ar.at<double>(o_Rt);
    double* Rpk = ar.at<double>(o_Rpk);  // packed copy of Rh, then of Rt, for the row solves
    double* Rfull = ar.at<double>(o_Rf);
    SKO_HIP(launch_zero(e.status, 256, c->stream));
    SKO_HIP(launch_zero(Rfull, sizeof(double) * (size_t)N * N, c->stream));

    const int red_sk = sp.red;
    const double sk_scale = sp.scale;
    const bool reorth = o->reorth != 0;

    for (int big = 0; big < nb / ppb; ++big) {
        const int p_old = big * Wb;
        void* Qb = offset_elems(Q, (int64_t)p_old * ldq, f32);
        SKO_HIP(launch_zero(Rbar, sizeof(double) * (size_t)Wb * Wb, c->stream));
        // ---- first stage: pre-process panel by panel (Fig. 5 Lines 10, 12; Fig. 8)
        for (int i = 0; i < ppb; ++i) {
            const int col = p_old + i * w;
            const void* Vi = offset_elems(V, (int64_t)col * ldv, f32);
            void* Qi = offset_elems(Q, (int64_t)col * ldq, f32);
            const void* Vh = Vi;
            int64_t ldvh = ldv;
            double* Ci = C + (int64_t)i * w * p_old;
            if (p_old > 0) {
                PassArgs a{};
                a.Y = Vi;
                a.ldy = ldv;
                SmallArgs sm{};
                sm.op = OP_STORE;
                sm.w = w;
                sm.out = Ci;
                if ((s = e.reduction({w, f32, RED_PROJ, false, 0, false}, a, p_old, Vi, ldv, Q, ldq, sm, 1.0)))
                    return s;
            }
            if (pip) {
                // BCGS-PIP (Fig. 7): G = V_hat^T V_hat (fused with the update against Q_old), then
                // P = Q_bar_prev^T V_hat, R = chol(G - P^T P); the first panel is CholQR.
                SmallArgs sp_{};
                sp_.op = OP_PIP;
                sp_.w = w;
                sp_.col0 = col;
                sp_.R = rho;
                sp_.r = rt;
                sp_.gram = Gpip;
                sp_.nacc = i * w;
                sp_.Rbar = Rbar;
                sp_.ldrbar = Wb;
                sp_.rbar_col0 = i * w;
                SmallArgs sg{};
                sg.op = OP_STORE;
                sg.w = w;
                sg.out = Gpip;
                PassArgs a{};
                a.Y = Vi;
                a.ldy = ldv;
                PassKey key{w, f32, RED_GRAM, false, 0, false};
                if (p_old > 0) {
                    key.upd = true;
                    key.write = true;
                    a.Qu = Q;
                    a.ldqu = ldq;
                    a.pu = p_old;
                    a.Cu = Ci;
                    a.X = Qi;
                    a.ldx = ldq;
                    Vh = Qi;
                    ldvh = ldq;
                }
                if (i == 0) {
                    sp_.out = Ysk;
                    if ((s = e.reduction(key, a, w, nullptr, 0, nullptr, 0, sp_, 1.0))) return s;
                } else {
                    if ((s = e.reduction(key, a, w, nullptr, 0, nullptr, 0, sg, 1.0))) return s;
                    PassArgs pa{};
                    pa.Y = Vh;
                    pa.ldy = ldvh;
                    sp_.out = Ysk;
                    if ((s = e.reduction({w, f32, RED_PROJ, false, 0, false}, pa, i * w, Vh, ldvh, Qb, ldq, sp_,
                                         1.0)))
                        return s;
                }
            } else {
                PassArgs a{};
                a.Y = Vi;
                a.ldy = ldv;
                PassKey key{w, f32, red_sk, false, 0, false};
                if (p_old > 0) {
                    key.upd = true;
                    key.write = true;
                    a.Qu = Q;
                    a.ldqu = ldq;
                    a.pu = p_old;
                    a.Cu = Ci;
                    a.X = Qi;
                    a.ldx = ldq;
                    Vh = Qi;
                    ldvh = ldq;
                }
                SmallArgs sm{};
                sm.op = OP_SKETCH_BCGS2;
                sm.w = w;
                sm.k = k;
                sm.col0 = col;
                sm.out = Ysk;
                sm.R = rho;
                sm.Yacc = Yacc;
                sm.nacc = i * w;
                sm.r = rt;
                sm.Rbar = Rbar;
                sm.ldrbar = Wb;
                sm.rbar_col0 = i * w;
                sketch_small(sm, sp);
                if ((s = e.reduction(key, a, kr, Vh, ldvh, nullptr, 0, sm, sk_scale))) return s;
            }
            {   // Q_bar_i = (V_hat_i - Q_bar_prev r) rho^{-1}
                PassArgs a{};
                a.Y = Vh;
                a.ldy = ldvh;
                a.R1 = rho;
                a.X = Qi;
                a.ldx = ldq;
                PassKey key{w, f32, RED_NONE, false, 1, true};
                if (i > 0) {
                    key.upd = true;
                    a.Qu = Qb;
                    a.ldqu = ldq;
                    a.pu = i * w;
                    a.Cu = rt;
                }
                if ((s = e.plain(key, a))) return s;
            }
        }
        // ---- second stage: CholQR of the big panel (Line 15), BCGS + CholQR (Line 19).
        // With the second pass, each row operation also accumulates the reduction that
        // follows it (the projection on the previous big panels, or the second Gram matrix),
        // so the panel it writes is not read again for that reduction.
        SmallArgs chol2{};   // second CholQR (R_t), which also assembles the final R
        chol2.op = OP_CHOL;
        chol2.w = Wb;
        chol2.col0 = p_old;
        chol2.out = Gb;
        chol2.R = Rt;
        chol2.Rpk = Rpk;
        chol2.assemble = 1;
        chol2.Ra = Rh;
        chol2.Rb = Rbar;
        chol2.C1 = p_old > 0 ? C : nullptr;
        chol2.C2 = p_old > 0 ? C2 : nullptr;
        chol2.p = p_old;
        chol2.Rout = Rfull + (int64_t)p_old * N;
        chol2.ldr = N;
        const bool fuse_proj = reorth && p_old > 0 && p_old <= 64;
        {
            SmallArgs sm{};
            sm.op = OP_CHOL;
            sm.w = Wb;
            sm.col0 = p_old;
            sm.out = Gb;
            sm.R = Rh;
            sm.Rpk = Rpk;
            if (!reorth) {
                sm.assemble = 1;
                sm.r_identity = 1;
                sm.Ra = Rh;
                sm.Rb = Rbar;
                sm.C1 = p_old > 0 ? C : nullptr;
                sm.p = p_old;
                sm.Rout = Rfull + (int64_t)p_old * N;
                sm.ldr = N;
            }
            if ((s = e.gemm_reduction(Qb, ldq, Wb, Qb, ldq, Wb, sm, Wb))) return s;
            if (reorth && p_old == 0) {
                // Q_b = Q_bar R_h^{-1} and its Gram matrix -> R_t
                if ((s = e.rowop_reduction(Wb, Qb, ldq, nullptr, 0, 0, nullptr, Rpk, Qb, ldq, nullptr, 0, 0, chol2,
                                           Wb)))
                    return s;
            } else if (fuse_proj) {
                // Q_b = Q_bar R_h^{-1} and C_2 = Q_old^T Q_b
                SmallArgs sp2{};
                sp2.op = OP_STORE;
                sp2.w = Wb;
                sp2.out = C2;
                if ((s = e.rowop_reduction(Wb, Qb, ldq, nullptr, 0, 0, nullptr, Rpk, Qb, ldq, Q, ldq, p_old, sp2,
                                           p_old)))
                    return s;
            } else {
                if ((s = e.rowop(Wb, Qb, ldq, nullptr, 0, 0, nullptr, Rpk, Qb, ldq))) return s;
            }
        }
        if (reorth) {
            if (p_old > 0) {
                if (!fuse_proj) {
                    for (int a0 = 0; a0 < p_old; a0 += 64) {
                        const int ma = std::min(64, p_old - a0);
                        SmallArgs sm{};
                        sm.op = OP_STORE;
                        sm.w = Wb;
                        sm.out = C2 + a0;
                        if ((s = e.gemm_reduction(offset_elems(Q, (int64_t)a0 * ldq, f32), ldq, ma, Qb, ldq, Wb, sm,
                                                  p_old)))
                            return s;
                    }
                }
                // Q_b -= Q_old C_2 and its Gram matrix -> R_t
                if ((s = e.rowop_reduction(Wb, Qb, ldq, Q, ldq, p_old, C2, nullptr, Qb, ldq, nullptr, 0, 0, chol2,
                                           Wb)))
                    return s;
            }
            if ((s = e.rowop(Wb, Qb, ldq, nullptr, 0, 0, nullptr, Rpk, Qb, ldq))) return s;
        }
    }
    double* Rhost = nullptr;
    if (R) {
        if ((s = ensure_pinned(c, sizeof(double) * (size_t)N * N))) return s;
        Rhost = static_cast<double*>(c->pinned);
        SKO_HIP(hipMemcpyAsync(Rhost, Rfull, sizeof(double) * (size_t)N * N, hipMemcpyDeviceToHost, c->stream));
    }
    if ((s = finish(c, e.status, breakdown_col)) && s != SKO_EBREAKDOWN) return s;
    if (R)
        for (int jc = 0; jc < N; ++jc)
            std::memcpy(R + (int64_t)jc * ldr, Rhost + (int64_t)jc * N, sizeof(double) * N);
    return s;
}

}  // namespace sko
