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
#include <vector>

#include "context.h"

namespace sko {
namespace {

inline const void* offset_elems(const void* p, int64_t elems, bool f32) {
    return static_cast<const char*>(p) + elems * (f32 ? 4 : 8);
}
inline void* offset_elems(void* p, int64_t elems, bool f32) {
    return static_cast<char*>(p) + elems * (f32 ? 4 : 8);
}

struct Engine {
    sko_ctx c;
    hipStream_t st;
    int64_t n;
    int W;
    bool f32;
    sko_sketch sk;
    int64_t nstrips;
    // workspace
    double* partials = nullptr;
    int64_t part_stride = 0;
    int gmax = 0;
    int* status = nullptr;
    unsigned* counter = nullptr;

    Engine(sko_ctx c_, int64_t n_, int W_, bool f32_, const sko_sketch& sk_)
        : c(c_), st(c_->stream), n(n_), W(W_), f32(f32_), sk(sk_) {
        nstrips = (n + kPassThreads - 1) / kPassThreads;
    }

    int grid_for(std::initializer_list<PassKey> keys) const {
        int cap = gmax;
        for (const PassKey& k : keys) cap = std::min(cap, std::max(1, pass_grid_cap(k)));
        return (int)std::max<int64_t>(1, std::min<int64_t>(nstrips, cap));
    }

    // One reduction: `first` pass (may update/solve/write), then identity passes over
    // Xsrc for the remaining reduction rows, then the reduce kernel with `small`.
    sko_status reduction(PassKey first, PassArgs a, int rows_total, const void* Xsrc, int64_t ldxs,
                         const void* Qp, int64_t ldqp, SmallArgs small, double scale) {
        const int rpl = pass_rows_per_launch(W);
        PassKey rest{W, f32, first.red, false, 0, false};
        const int G = (rows_total > rpl) ? grid_for({first, rest}) : grid_for({first});
        a.partials = partials;
        a.part_stride = part_stride;
        a.part_rows_total = rows_total;
        a.n = n;
        a.sk_k = sk.k;
        a.sk_zeta = sk.zeta;
        a.sk_seed = sk.seed;
        for (int r0 = 0; r0 < rows_total; r0 += rpl) {
            PassArgs b = a;
            PassKey key = first;
            if (r0 > 0) {
                key = rest;
                b.Y = Xsrc;
                b.ldy = ldxs;
            }
            b.red_row0 = r0;
            b.red_rows = std::min(rpl, rows_total - r0);
            if (first.red == RED_PROJ) {
                b.Qp = offset_elems(Qp, (int64_t)r0 * ldqp, f32);
                b.ldqp = ldqp;
            } else if (first.red == RED_SKETCH_DENSE) {
                b.theta = sk.theta + (int64_t)r0 * sk.ld_theta;
                b.ldtheta = sk.ld_theta;
            }
            SKO_HIP(launch_pass(key, b, G, st));
        }
        ReduceArgs ra{};
        ra.partials = partials;
        ra.stride = part_stride;
        ra.G = G;
        ra.count = rows_total * W;
        ra.scale = scale;
        ra.counter = counter;
        ra.small = small;
        ra.small.status = status;
        SKO_HIP(launch_reduce(ra, st));
        return SKO_OK;
    }

    sko_status plain(PassKey key, PassArgs a) {
        a.n = n;
        SKO_HIP(launch_pass(key, a, grid_for({key}), st));
        return SKO_OK;
    }
};

struct BlockBufs {
    double *C1, *C2, *Ysk, *G2, *G3, *R1, *R2, *R3;
};

// One-stage BCGS2 block: V (n x W) against Q (n x p) -> Qo; R columns assembled at
// Rcol (device, rows 0..p+W-1, leading dimension ldr).
sko_status one_stage_block(Engine& e, const BlockBufs& b, int intra, int p, const void* Q, int64_t ldq,
                           const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rcol, int64_t ldr,
                           int col0) {
    const int W = e.W;
    const bool f32 = e.f32;
    const bool rand = intra == SKO_INTRA_RANDCHOLQR;
    const int red_first = rand ? (e.sk.kind == SKO_SKETCH_SPARSE_SIGN ? RED_SKETCH_SPARSE : RED_SKETCH_DENSE)
                               : RED_GRAM;
    const int rows_first = rand ? e.sk.k : W;
    const double sk_scale =
        (rand && e.sk.kind == SKO_SKETCH_SPARSE_SIGN) ? 1.0 / std::sqrt((double)e.sk.zeta) : 1.0;
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
        sm.k = rows_first;
        sm.col0 = col0;
        sm.out = b.Ysk;
        sm.R = b.R1;
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
        const int rpl = pass_rows_per_launch(W);
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

bool sketch_ok(const sko_sketch& sk, int64_t n) {
    if (sk.k < 1 || sk.k > 256) return false;
    if (sk.kind == SKO_SKETCH_SPARSE_SIGN) {
        if (sk.zeta < 1 || sk.zeta > 8 || sk.k % sk.zeta != 0 || sk.k / sk.zeta > 128) return false;
        return true;
    }
    if (sk.kind == SKO_SKETCH_GAUSSIAN) return sk.theta != nullptr && sk.ld_theta >= n;
    return false;
}

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
    L.small = ar.reserve(sizeof(double) * (2 * cw + (int64_t)std::max(k, W) * W + 5 * W * W));
    L.rfull = ar.reserve(sizeof(double) * (int64_t)std::max(1, N) * std::max(1, N));
    L.status = ar.reserve(256);
    L.total = ar.used();
    return L;
}

BlockBufs carve(sko_ctx c, const OneStageLayout& L, int pmax, int k, int W) {
    Arena ar(c);
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
    return b;
}

sko_status finish(sko_ctx c, int* status_dev, int32_t* breakdown_col) {
    SKO_HIP(hipMemcpyAsync(c->status_host, status_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    SKO_HIP(hipStreamSynchronize(c->stream));
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
    const bool rand = o->two_stage || o->intra == SKO_INTRA_RANDCHOLQR;
    if (!o->two_stage && o->intra != SKO_INTRA_RANDCHOLQR && o->intra != SKO_INTRA_CHOLQR2) return SKO_EINVAL;
    if (rand && !sketch_ok(o->sketch, n)) return SKO_EINVAL;
    if (rand && o->sketch.k < w) return SKO_EINVAL;
    if ((int64_t)(N - w) * w > kMaxUpdCoef) return SKO_EUNSUPPORTED;
    if (w > pass_rows_per_launch(w)) return SKO_EUNSUPPORTED;
    if (o->two_stage) return two_stage_blocks(c, n, nb, w, V, ldv, Q, ldq, R, ldr, o, breakdown_col);

    const bool f32 = o->precision == SKO_MIXED_F32;
    const int k = rand ? o->sketch.k : w;
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
    SKO_HIP(hipMemsetAsync(e.status, 0, 256, c->stream));
    SKO_HIP(hipMemsetAsync(Rfull, 0, sizeof(double) * (size_t)N * N, c->stream));
    BlockBufs bb = carve(c, L, N - w, k, w);
    for (int j = 0; j < nb; ++j) {
        const int p = j * w;
        const void* Vj = offset_elems(V, (int64_t)p * ldv, f32);
        void* Qj = offset_elems(Q, (int64_t)p * ldq, f32);
        s = one_stage_block(e, bb, o->intra, p, Q, ldq, Vj, ldv, Qj, ldq, Rfull + (int64_t)p * N, N, p);
        if (s) return s;
    }
    if (R) {
        SKO_HIP(hipMemcpy2DAsync(R, sizeof(double) * ldr, Rfull, sizeof(double) * N, sizeof(double) * N, N,
                                 hipMemcpyDeviceToHost, c->stream));
    }
    return finish(c, e.status, breakdown_col);
}

sko_status orth_block_impl(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq, const void* V,
                           int64_t ldv, void* Qo, int64_t ldqo, double* Rp, double* Rd, const sko_orth_opts* o,
                           int32_t* breakdown_col) {
    if (breakdown_col) *breakdown_col = 0;
    if (!o || !V || !Qo || n < 1 || p < 0 || w < 1 || w > kMaxPassW || ldv < n || ldqo < n) return SKO_EINVAL;
    if (p > 0 && (!Q || ldq < n)) return SKO_EINVAL;
    if (o->two_stage) return SKO_EINVAL;
    if (o->precision != SKO_F64 && o->precision != SKO_MIXED_F32) return SKO_EINVAL;
    if (o->intra != SKO_INTRA_RANDCHOLQR && o->intra != SKO_INTRA_CHOLQR2) return SKO_EINVAL;
    const bool rand = o->intra == SKO_INTRA_RANDCHOLQR;
    if (rand && (!sketch_ok(o->sketch, n) || o->sketch.k < w)) return SKO_EINVAL;
    if ((int64_t)p * w > kMaxUpdCoef) return SKO_EUNSUPPORTED;
    if (w > pass_rows_per_launch(w)) return SKO_EUNSUPPORTED;
    const bool f32 = o->precision == SKO_MIXED_F32;
    const int k = rand ? o->sketch.k : w;
    const int N = p + w;
    OneStageLayout L = layout_one_stage(c, n, w, p, k, N);
    sko_status s = ensure_workspace(c, L.total);
    if (s) return s;
    Arena ar(c);
    Engine e(c, n, w, f32, o->sketch);
    e.partials = ar.at<double>(L.partials);
    e.part_stride = L.part_stride;
    e.gmax = L.gmax;
    e.status = ar.at<int>(L.status);
    e.counter = reinterpret_cast<unsigned*>(e.status + 16);
    double* Rcol = ar.at<double>(L.rfull);  // (p + w) x w, ld p + w
    SKO_HIP(hipMemsetAsync(e.status, 0, 256, c->stream));
    BlockBufs bb = carve(c, L, p, k, w);
    s = one_stage_block(e, bb, o->intra, p, Q, ldq, V, ldv, Qo, ldqo, Rcol, N, 0);
    if (s) return s;
    if (Rp && p > 0)
        SKO_HIP(hipMemcpy2DAsync(Rp, sizeof(double) * p, Rcol, sizeof(double) * N, sizeof(double) * p, w,
                                 hipMemcpyDeviceToHost, c->stream));
    if (Rd)
        SKO_HIP(hipMemcpy2DAsync(Rd, sizeof(double) * w, Rcol + p, sizeof(double) * N, sizeof(double) * w, w,
                                 hipMemcpyDeviceToHost, c->stream));
    return finish(c, e.status, breakdown_col);
}

sko_status two_stage_blocks(sko_ctx, int64_t, int32_t, int32_t, const void*, int64_t, void*, int64_t, double*,
                            int64_t, const sko_orth_opts*, int32_t*) {
    return SKO_EUNSUPPORTED;
}

}  // namespace sko
