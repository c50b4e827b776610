// Launch-shape autotuning of the row-strip passes (sko_autotune_orth).
//
// The block orthogonalisation launches a handful of pass variants (one per reduction /
// update / solve / write combination and tile count).  How many workgroups per compute
// unit stream a pass fastest depends on the variant (its registers, LDS and the number of
// column streams it reads) in ways occupancy alone does not predict, so each variant the
// schedule of sko_orth_blocks(n, nb, w, opts) uses is timed on library-owned scratch blocks
// at 2..8 workgroups per CU, and the fastest count is kept in the context for that variant
// and row-count class (log2 of the strip count).  Later launches of the variant on a matrix
// of the same class use it; everything else keeps the occupancy-derived default.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "engine.h"

namespace sko {
namespace {

struct Use {
    PassKey key;
    int p;     // columns of the update / projection operand
    int rows;  // reduction rows of the whole reduction
};

// The passes of the one-stage block step (Fig. 2c with the first intra step) for p
// previous columns, in launch order.
void one_stage_uses(int W, bool f32, int red_first, int rows_first, int p, std::vector<Use>& out) {
    if (p > 0) out.push_back({{W, f32, RED_PROJ, false, 0, false}, p, p});
    out.push_back({{W, f32, red_first, p > 0, 0, p > 0}, p, rows_first});
    out.push_back({{W, f32, RED_GRAM, false, 1, false}, 0, W});
    if (p > 0)
        out.push_back({{W, f32, RED_PROJ, false, 2, true}, 0, p});
    else
        out.push_back({{W, f32, RED_GRAM, false, 2, true}, 0, W});
    if (p > 0) out.push_back({{W, f32, RED_GRAM, true, 0, true}, p, W});
    out.push_back({{W, f32, RED_NONE, false, 1, true}, 0, 0});
}

// The row-strip passes of one two-stage panel (Fig. 5): projection on the previous big
// panels, update + sketch, forward substitution against the panel's earlier blocks.
void two_stage_uses(int w, bool f32, int red_sk, int k, int p_old, int loc, std::vector<Use>& out) {
    if (p_old > 0) {
        out.push_back({{w, f32, RED_PROJ, false, 0, false}, 0, p_old});
        out.push_back({{w, f32, red_sk, true, 0, true}, p_old, k});
    } else {
        out.push_back({{w, f32, red_sk, false, 0, false}, 0, k});
    }
    out.push_back({{w, f32, RED_NONE, loc > 0, 1, true}, loc, 0});
}

}  // namespace

sko_status autotune_orth_impl(sko_ctx c, int64_t n, int32_t nb, int32_t w, const sko_orth_opts* o) {
    if (!o || n < 1 || nb < 1 || w < 1 || w > kMaxPassW) return SKO_EINVAL;
    if (o->precision != SKO_F64 && o->precision != SKO_MIXED_F32) return SKO_EINVAL;
    const bool f32 = o->precision == SKO_MIXED_F32;
    // the deterministic comparators (BCGS-PIP pre-processing, recursive CholQR2) keep the
    // default launch shapes
    if ((o->two_stage && o->preproc == SKO_PREPROC_PIP) || (!o->two_stage && o->intra == SKO_INTRA_CHOLQR2_RECURSIVE))
        return SKO_OK;
    const bool rand = o->two_stage || o->intra == SKO_INTRA_RANDCHOLQR;
    if (rand && !sketch_ok(o->sketch, n)) return SKO_EINVAL;
    const SketchPlan sp = sketch_plan(o->sketch);
    const int red_sk = sp.red;
    const int cus = std::max(1, c->cus);
    const int64_t nstrips = (n + kPassThreads - 1) / kPassThreads;
    if (nstrips < 4 * (int64_t)cus) return SKO_OK;  // too few strips for the grid to matter

    // ---- the launches of the schedule, grouped by kernel variant
    std::vector<Use> uses;
    if (!o->two_stage) {
        const int red_first = rand ? red_sk : RED_GRAM;
        const int rows_first = rand ? sp.rows : w;
        for (int j = 0; j < nb; ++j) one_stage_uses(w, f32, red_first, rows_first, j * w, uses);
    } else {
        const int ppb = std::max(1, o->panels_per_big);
        for (int j = 0; j < nb; ++j) {
            const int big = j / ppb, i = j % ppb;
            two_stage_uses(w, f32, red_sk, sp.rows, big * ppb * w, i * w, uses);
        }
    }
    std::map<const void*, std::vector<Use>> groups;
    int pmax = 1, rows_max = w;
    for (Use& u : uses) {
        const int rpl = u.key.red != RED_NONE ? pass_rows_per_launch(w, u.key.red) : 0;
        if (u.key.red == RED_PROJ || u.key.red == RED_SKETCH_SPARSE) u.key.tiles = (std::min(rpl, u.rows) + 15) / 16;
        const void* id = pass_kernel_id(u.key);
        if (!id) return SKO_EUNSUPPORTED;
        groups[id].push_back(u);
        pmax = std::max({pmax, u.p, u.key.red == RED_PROJ ? u.rows : 0});
        rows_max = std::max(rows_max, u.rows);
    }
    if ((int64_t)pmax * w > kMaxUpdCoef) return SKO_EUNSUPPORTED;

    // ---- scratch: Y, X (n x w), Q (n x pmax), coefficients, identity factors, partials
    const size_t eb = f32 ? 4 : 8;
    const int64_t rpl_max = std::max(pass_rows_per_launch(w, RED_PROJ), pass_rows_per_launch(w, red_sk));
    const int64_t part_stride = ((std::min<int64_t>(rows_max, rpl_max) * w + 31) / 32) * 32;
    const size_t tall = eb * (size_t)n;
    const size_t bytes = tall * (2 * (size_t)w + pmax) + sizeof(double) * ((size_t)pmax * w + 2 * (size_t)w * w) +
                         sizeof(double) * (size_t)part_stride * 8 * cus + 1024;
    char* buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) return SKO_ENOMEM;
    struct Free {
        char* p;
        ~Free() { (void)hipFree(p); }
    } guard{buf};
    char* Y = buf;
    char* X = Y + tall * w;
    char* Q = X + tall * w;
    double* Cu = reinterpret_cast<double*>(Q + tall * pmax);
    double* R1 = Cu + (size_t)pmax * w;
    double* partials = R1 + 2 * (size_t)w * w;
    SKO_HIP(hipMemsetAsync(buf, 0, bytes, c->stream));
    std::vector<double> eye(2 * (size_t)w * w, 0.0);
    for (int t = 0; t < 2; ++t)
        for (int i = 0; i < w; ++i) eye[(size_t)t * w * w + i + (size_t)i * w] = 1.0;
    SKO_HIP(hipMemcpyAsync(R1, eye.data(), sizeof(double) * eye.size(), hipMemcpyHostToDevice, c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SKO_HIP(hipEventCreate(&e0));
    SKO_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evg{e0, e1};

    const int bucket = (int)std::floor(std::log2((double)nstrips));
    for (auto& [id, list] : groups) {
        std::sort(list.begin(), list.end(), [](const Use& a, const Use& b) { return a.p + a.rows < b.p + b.rows; });
        const Use& u = list[list.size() / 2];
        PassArgs a{};
        a.n = n;
        a.Y = Y;
        a.ldy = n;
        a.Qu = Q;
        a.ldqu = n;
        a.pu = u.p;
        a.Cu = Cu;
        a.R1 = R1;
        a.R2 = R1 + (size_t)w * w;
        a.X = X;
        a.ldx = n;
        a.Qp = Q;
        a.ldqp = n;
        a.theta = sp.red == RED_SKETCH_DENSE ? o->sketch.theta : nullptr;
        a.ldtheta = o->sketch.ld_theta;
        a.partials = partials;
        a.part_stride = part_stride;
        a.sk_seed = o->sketch.seed;
        a.sk_k = sp.rows;
        a.sk_zeta = o->sketch.zeta;
        if (u.key.red != RED_NONE) {
            a.red_rows = std::min(u.rows, pass_rows_per_launch(w, u.key.red));
            a.red_row0 = 0;
            a.part_rows_total = a.red_rows;
        }
        int best = 0;
        float best_ms = 0.f;
        for (int wpc = 2; wpc <= 8; ++wpc) {
            const int G = (int)std::min<int64_t>(nstrips, (int64_t)wpc * cus);
            SKO_HIP(launch_pass(u.key, a, G, c->stream));  // warm-up
            SKO_HIP(hipEventRecord(e0, c->stream));
            for (int r = 0; r < 3; ++r) SKO_HIP(launch_pass(u.key, a, G, c->stream));
            SKO_HIP(hipEventRecord(e1, c->stream));
            SKO_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            SKO_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (best == 0 || ms < best_ms) {
                best = wpc;
                best_ms = ms;
            }
        }
        c->grid_wpc[{id, bucket}] = best;
    }
    SKO_HIP(hipStreamSynchronize(c->stream));
    return SKO_OK;
}

}  // namespace sko
