// Launch orchestration shared by the block-orthogonalisation and GMRES drivers.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <string>

#include "batch.h"
#include "context.h"

namespace sko {

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
    // Batched mode: every launch serves the active systems of `br` (template addresses are
    // system 0's); n is the largest system's row count and rows_bytes the active systems'
    // total, for the byte accounting.
    const BatchReloc* br = nullptr;
    double rows_bytes = 0.0;
    // false: no profiler events (no host-side bookkeeping at all) for this engine's launches
    bool profile = true;
    int sk_rows;  // sketch rows the passes produce (k_count for a Count-Gauss sketch)

    Engine(sko_ctx c_, int64_t n_, int W_, bool f32_, const sko_sketch& sk_)
        : c(c_), st(c_->stream), n(n_), W(W_), f32(f32_), sk(sk_) {
        nstrips = (n + kPassThreads - 1) / kPassThreads;
        rows_bytes = (double)n;
        sk_rows = sketch_plan(sk).rows;
    }

    // Profiler bracket of one launch; the kernel-kind name is built only while profiling.
    template <typename NameFn>
    int pbegin(NameFn&& name, double bytes) {
        if (!profile || !c->prof.on) return -1;
        return c->prof.begin(name(), bytes, st);
    }
    void pend(int ev) {
        if (ev >= 0) c->prof.end(ev, st);
    }

    // Workgroups of a pass launch: the autotuned count for the variant and this row-count
    // class if sko_autotune_orth chose one, else as many as are resident at once.
    int grid_for(std::initializer_list<PassKey> keys) const {
        int cap = gmax;
        const int bucket = nstrips > 0 ? (int)std::floor(std::log2((double)nstrips)) : 0;
        for (const PassKey& k : keys) {
            int kc = pass_grid_cap(k);
            if (!c->grid_wpc.empty()) {
                const auto it = c->grid_wpc.find({pass_kernel_id(k), bucket});
                if (it != c->grid_wpc.end()) kc = it->second * std::max(1, c->cus);
            }
            cap = std::min(cap, std::max(1, kc));
        }
        return (int)std::max<int64_t>(1, std::min<int64_t>(nstrips, cap));
    }

    // One reduction: `first` pass (may update/solve/write), then identity passes over
    // Xsrc for the remaining reduction rows, then the reduce kernel with `small`.
    sko_status reduction(PassKey first, PassArgs a, int rows_total, const void* Xsrc, int64_t ldxs,
                         const void* Qp, int64_t ldqp, SmallArgs small, double scale) {
        const int rpl = pass_rows_per_launch(W, first.red);
        if (first.red == RED_PROJ || first.red == RED_SKETCH_SPARSE) first.tiles = (std::min(rpl, rows_total) + 15) / 16;
        PassKey rest{W, first.f32, first.red, false, 0, false, first.tiles};
        if (first.panel) {
            // the remaining rows read the (updated) FP64 panel: a projection still against
            // the FP32 basis, a sketch of the panel alone in FP64
            if (first.red == RED_PROJ)
                rest.panel = 1;
            else
                rest.f32 = false;
        }
        const int G = (rows_total > rpl) ? grid_for({first, rest}) : grid_for({first});
        a.partials = partials;
        a.part_stride = part_stride;
        a.part_rows_total = rows_total;
        a.n = n;
        a.sk_k = sk_rows;
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
            const int ev = pbegin([&] { return pass_name(key); }, pass_bytes(key, b));
            SKO_HIP(launch_pass(key, b, G, st, br));
            pend(ev);
        }
        ReduceArgs ra{};
        ra.partials = partials;
        ra.stride = part_stride;
        ra.G = G;
        ra.count = rows_total * W;
        ra.scale = scale;
        ra.counter = counter;
        ra.rows = ra.count;
        ra.ldo = ra.count;
        ra.small = small;
        ra.small.status = status;
        ra.unit_rows = kPassThreads;  // a strip is at least this many rows
        const int ev = pbegin([&] { return std::string(reduce_name(small.op)); }, 8.0 * G * ra.count);
        SKO_HIP(launch_reduce(ra, st, br));
        pend(ev);
        return SKO_OK;
    }

    // C = A^T B (ma, nb <= 64) reduced into out (placed with leading dimension ldo) and
    // handed to `small`.
    sko_status gemm_reduction(const void* A, int64_t lda, int ma, const void* B, int64_t ldb, int nbc,
                              SmallArgs small, int64_t ldo) {
        const int G = gemm_grid(A == B && lda == ldb && ma == nbc, ma, nbc);
        const int ev = pbegin(
            [&] { return std::string("wide_gemm_tn ") + (A == B ? "gram" : "proj") + " f" + (f32 ? "32" : "64"); },
            rows_bytes * (A == B ? ma : ma + nbc) * (f32 ? 4.0 : 8.0));
        SKO_HIP(launch_skinny_gemm_tn(n, A, lda, ma, B, ldb, nbc, f32, partials, G, st, br));
        pend(ev);
        ReduceArgs ra{};
        ra.partials = partials;
        ra.stride = (int64_t)ma * nbc;
        ra.G = G;
        ra.count = ma * nbc;
        ra.scale = 1.0;
        ra.counter = counter;
        ra.rows = ma;
        ra.ldo = ldo;
        ra.small = small;
        ra.small.status = status;
        ra.unit_rows = kGemmUnitRows;
        const int ev2 = pbegin([&] { return std::string(reduce_name(small.op)); }, 8.0 * G * ra.count);
        SKO_HIP(launch_reduce(ra, st, br));
        pend(ev2);
        return SKO_OK;
    }

    // X = (Y - Qu Cu) R^{-1} (rowop) and, in the same sweep over X, C = E^T X (E: me <= 64
    // tall columns, solve only) or the Gram X^T X (E null), reduced into `small` as
    // gemm_reduction does.  Panels wider than kFusedMaxW keep the two sweeps apart (the row
    // and the accumulators no longer fit two waves' registers), and so do projections on more
    // than 48 columns and the update form: its Q_u loads and the MFMA accumulators together
    // run slower than two sweeps (measured 5.4-5.6 ms against 4.3 ms, 36 columns on 36,
    // n = 2^24, with four or eight update columns in flight).
    sko_status rowop_reduction(int Wd, const void* Y, int64_t ldy, const void* Qu, int64_t ldqu, int pu,
                               const double* Cu, const double* Rpk, void* X, int64_t ldx, const void* E, int64_t lde,
                               int me, SmallArgs small, int64_t ldo) {
        if (pu > 0 || Wd > kFusedMaxW || (E && me > 48)) {
            sko_status s = rowop(Wd, Y, ldy, Qu, ldqu, pu, Cu, Rpk, X, ldx);
            if (s) return s;
            return E ? gemm_reduction(E, lde, me, X, ldx, Wd, small, ldo) : gemm_reduction(X, ldx, Wd, X, ldx, Wd, small, ldo);
        }
        const int ma = E ? me : Wd;
        // batched: as many workgroups per system as the wide Gram / projection would take (its
        // partial-sum regions), at most one per strip of the largest system
        int G = br ? (int)std::max<int64_t>(1, std::min<int64_t>(gemm_grid(!E, ma, Wd),
                                                                  (n + kFusedUnitRows - 1) / kFusedUnitRows))
                   : 0;
        const int ev = pbegin(
            [&] {
                return std::string("wide_rowop+") + (E ? "proj" : "gram") + " f" + (f32 ? "32" : "64") +
                       (pu > 0 ? " upd" : "") + (Rpk ? " trsm" : "");
            },
            rows_bytes * (2 * Wd + pu + (E ? me : 0)) * (f32 ? 4.0 : 8.0));
        SKO_HIP(launch_wide_rowop_reduce(n, Wd, f32, Y, ldy, Qu, ldqu, pu, Cu, Rpk, X, ldx, E, lde, me, partials, &G,
                                         st, br));
        pend(ev);
        ReduceArgs ra{};
        ra.partials = partials;
        ra.stride = (int64_t)ma * Wd;
        ra.G = G;
        ra.count = ma * Wd;
        ra.scale = 1.0;
        ra.counter = counter;
        ra.rows = ma;
        ra.ldo = ldo;
        ra.small = small;
        ra.small.status = status;
        ra.unit_rows = kFusedUnitRows;
        const int ev2 = pbegin([&] { return std::string(reduce_name(small.op)); }, 8.0 * G * ra.count);
        SKO_HIP(launch_reduce(ra, st, br));
        pend(ev2);
        return SKO_OK;
    }

    // Rpk: the triangular factor packed by the Cholesky step that produced it (SmallArgs::Rpk)
    sko_status rowop(int Wd, const void* Y, int64_t ldy, const void* Qu, int64_t ldqu, int pu, const double* Cu,
                     const double* Rpk, void* X, int64_t ldx) {
        const int ev = pbegin(
            [&] {
                return std::string("wide_rowop f") + (f32 ? "32" : "64") + (pu > 0 ? " upd" : "") + (Rpk ? " trsm" : "");
            },
            rows_bytes * (2 * Wd + pu) * (f32 ? 4.0 : 8.0));
        SKO_HIP(launch_wide_rowop(n, Wd, f32, Y, ldy, Qu, ldqu, pu, Cu, Rpk, X, ldx, st, br));
        pend(ev);
        return SKO_OK;
    }

    sko_status plain(PassKey key, PassArgs a) {
        a.n = n;
        const int ev = pbegin([&] { return pass_name(key); }, pass_bytes(key, a));
        SKO_HIP(launch_pass(key, a, grid_for({key}), st, br));
        pend(ev);
        return SKO_OK;
    }

    // Workgroups of a wide Gram / projection launch (per system in batched mode, where a
    // launch already holds many systems).
    // One system: at most the resident workgroups, so no second, partly idle round of
    // workgroups follows the first (each walks its 16-row groups).
    int gemm_grid(bool sym, int ma, int nbc) const {
        const int64_t ns32 = (n + 31) / 32;
        const int64_t want = br ? (ns32 + 63) / 64 : ns32;
        int64_t cap = skinny_gemm_grid_cap();
        if (!br) {
            const int res = skinny_gemm_resident(sym, f32, ma, nbc);
            if (res > 0) cap = std::min<int64_t>(cap, res);
        }
        return (int)std::max<int64_t>(1, std::min<int64_t>(want, cap));
    }

    // Profiler name of a reduction launch: the partial sums and the small step that ends it.
    static const char* reduce_name(int op) {
        switch (op) {
            case OP_STORE: return "reduce+store";
            case OP_HH: return "reduce+householder";
            case OP_CHOL: return "reduce+cholesky";
            case OP_SKETCH_BCGS2: return "reduce+sketch-space bcgs2";
            default: return "reduce+small";
        }
    }

    static std::string pass_name(const PassKey& k) {
        static const char* reds[] = {"none", "proj", "gram", "sketch_sparse", "sketch_dense"};
        char buf[96];
        const int mt = k.red == RED_PROJ ? (k.tiles >= 1 && k.tiles <= 4 ? 4 : k.tiles >= 5 && k.tiles <= 6 ? 6 : 8) : 0;
        char tl[16] = "";
        if (mt) snprintf(tl, sizeof tl, "/mt%d", mt);
        const char* ty = k.panel == 1 ? "f64|f32" : k.panel == 2 ? "f64>f32" : k.f32 ? "f32" : "f64";
        snprintf(buf, sizeof buf, "pass W=%d %s red=%s%s upd=%d trsm=%d write=%d", k.W, ty, reds[k.red], tl,
                 (int)k.upd, k.ntrsm, (int)k.write);
        return buf;
    }
    // Algorithmic HBM bytes of one launch: every tall operand once (read or written).
    double pass_bytes(const PassKey& k, const PassArgs& a) const {
        const double eq = k.f32 ? 4.0 : 8.0;               // basis operand
        const double ey = k.panel ? 8.0 : eq;              // input block
        const double ex = k.panel == 1 ? 8.0 : eq;         // written block
        double per_row = W * ey + (k.write ? W * ex : 0.0) +
                         ((k.upd ? a.pu : 0) + (k.red == RED_PROJ ? a.red_rows : 0)) * eq +
                         (k.red == RED_SKETCH_DENSE ? 8.0 * a.red_rows : 0.0);
        return per_row * rows_bytes;
    }
};

struct BlockBufs {
    double *C1, *C2, *Ysk, *G2, *G3, *R1, *R2, *R3;
    double *S1, *S2;  // w x w scratch of the recursive CholQR (compact partial factors)
};

// One-stage BCGS2 block (Fig. 2c): V (n x W) against Q (n x p) -> Qo (may alias V);
// [R_proj; R_diag] assembled at Rcol (device, rows 0..p+W-1, leading dimension ldr).
sko_status one_stage_block(Engine& e, const BlockBufs& b, int intra, int p, const void* Q, int64_t ldq,
                           const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rcol, int64_t ldr,
                           int col0);

bool sketch_ok(const sko_sketch& sk, int64_t n);

}  // namespace sko
