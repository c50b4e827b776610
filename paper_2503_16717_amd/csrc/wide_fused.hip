// The big-panel row operation with the next reduction fused into it (Fig. 6: the BCGS
// projection of the panel just written on the previous big panels, or the Gram matrix of
// the second CholQR).  One sweep computes X = (Y - Qu Cu) R^{-1} row by row, as the plain
// row operation does, writes X, and accumulates per-workgroup partial sums of
//     X^T X   (Gram, output tiles on or above the diagonal), or
//     E^T X   (projection on a tall E of at most 48 columns, read here once)
// on FP64 MFMA 16 x 16 x 4 tiles.  X is never read back from HBM for the reduction.
//
// Layout change through LDS: a thread holds one row of X, the MFMA operands want 4 rows x
// 16 columns spread over the lanes.  Each wave stages its 64 rows 16 at a time, column-major
// with a column stride of 18 doubles (lanes reading different columns fall into different
// LDS banks), and reads back the 4-row pieces of every 16-column tile.  Columns past the
// panel width hold stale values; they only reach output entries that are never written.
#include <algorithm>

#include "batch.h"
#include "sko_internal.h"
#include "uniform.h"
#include "wide_common.h"

namespace sko {
namespace {

using namespace wide;

struct FusedArgs {
    RowopArgs ra;
    const void* E;  // null: Gram of X
    int64_t lde;
    int me;
    double* partials;
    int64_t stride;
};

constexpr int SLD = 18;  // staged column stride in doubles (16 rows + 2)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// TE = 0: Gram; 1..3: tiles of E's columns (ceil(me / 16)).  At least two waves per SIMD:
// the row's values and the tile accumulators are live together, and up to 40 columns with up
// to three tiles of E fit 256 VGPRs without spilling (wider panels keep the two sweeps apart).
template <int WB, typename T, bool UPD, bool TRSM, int TE>
__device__ __forceinline__ void rowop_red_body(const FusedArgs& fa, const int wg, const int nwg) {
    constexpr int TX = (WB + 15) / 16;  // 16-column tiles of X
    constexpr bool GRAM = TE == 0;
    constexpr int TA = GRAM ? TX : TE;
    constexpr int NW = ROW_NT / 64;
    constexpr int SW = 16 * TX * SLD;  // doubles staged per wave
    static_assert(NW * SW >= 4 * 64 * NW, "the staging area also holds the cross-wave sums");
    __shared__ double stage[NW * SW];
    __shared__ double sD[TRSM ? WB : 1];
    const RowopArgs& ra = fa.ra;
    const int64_t n = ra.n;
    const int w0 = ra.w, pu = ra.pu;
    const T* __restrict__ Y = static_cast<const T*>(ra.Y);
    const T* __restrict__ Qu = static_cast<const T*>(ra.Qu);
    T* X = static_cast<T*>(ra.X);
    const T* E = static_cast<const T*>(fa.E);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, ci = lane & 15, g = lane >> 4;
    const uint32_t lane_bytes = (uint32_t)tid * (uint32_t)sizeof(T);
    if constexpr (TRSM) {
        for (int i = tid; i < w0; i += ROW_NT) sD[i] = ra.Rpk[i];
        __syncthreads();
    }
    const CD R0 = as_uniform(ra.Rpk), C0 = as_uniform(ra.Cu);
    const bool vece = !GRAM && (fa.lde % 4) == 0 && ((uintptr_t)E % (4 * sizeof(T))) == 0;
    double* st = stage + wave * SW;
    double4_t acc[TA][TX];
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int j = 0; j < TX; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

    for (int64_t r0 = (int64_t)wg * ROW_NT; r0 < n; r0 += (int64_t)nwg * ROW_NT) {
        const int64_t row = r0 + tid;
        double xa[1][WB];
        double(&x)[WB] = xa[0];
        if (row < n) {
            const CD Rs = per_strip(R0), Cs = per_strip(C0);
            const int64_t ldy = per_strip(ra.ldy), ldx = per_strip(ra.ldx), ldqu = per_strip(ra.ldqu);
            const int w = per_strip(w0);
#pragma unroll
            for (int c = 0; c < WB; ++c)
                x[c] = ldv_nt(lane_elem(Y + r0 + (int64_t)(c < w ? c : w - 1) * ldy, lane_bytes));
            if constexpr (UPD) update_rows<WB, 1, T>(xa, Qu + row, ldqu, pu, Cs, w);
            if constexpr (TRSM) solve_cols<WB, 0>(x, Rs, w, sD);
#pragma unroll
            for (int c = 0; c < WB; ++c) {
                if (c < w) {
                    const T v = static_cast<T>(x[c]);
                    stv_nt(lane_elem(X + r0 + (int64_t)c * ldx, lane_bytes), v);
                    x[c] = static_cast<double>(v);  // reduce what was stored (FP32 storage: rounded)
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < WB; ++c) x[c] = 0.0;
        }
        // the wave's 64 rows in four chunks of 16 (lanes 16q..16q+15 hold chunk q)
        const int64_t wrow0 = r0 + 64 * wave;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double ea[GRAM ? 1 : TA][4];
            if constexpr (!GRAM) {
                const int64_t crow = wrow0 + 16 * q;
                load_pieces<T, TA>(E, fa.lde, fa.me, ci, vece, crow + 16 <= n, crow + 4 * g, n, ea);
            }
            if (g == q) {
#pragma unroll
                for (int c = 0; c < WB; ++c) st[c * SLD + ci] = x[c];
            }
            wave_sync();
            // piece of tile t: rows 4g..4g+3 of the chunk, column 16t + ci
            double xb[TX][4];
#pragma unroll
            for (int t = 0; t < TX; ++t) {
                const double2* p = reinterpret_cast<const double2*>(st + (16 * t + ci) * SLD + 4 * g);
                const double2 v0 = p[0], v1 = p[1];
                xb[t][0] = v0.x;
                xb[t][1] = v0.y;
                xb[t][2] = v1.x;
                xb[t][3] = v1.y;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int i = 0; i < TA; ++i)
#pragma unroll
                    for (int j = 0; j < TX; ++j) {
                        if (!GRAM || i <= j) {
                            const double av = GRAM ? xb[i][u] : ea[GRAM ? 0 : i][u];
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, xb[j][u], acc[i][j], 0, 0, 0);
                        }
                    }
            wave_sync();
        }
    }

    // D[r][c] of a tile sits in lane c + 16 (r % 4), element r / 4; the waves' tiles are
    // summed through LDS in wave order and written once per workgroup
    __syncthreads();
    double* red = stage;
    const int ma = GRAM ? w0 : fa.me;
    double* out = fa.partials + (int64_t)wg * fa.stride;
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int j = 0; j < TX; ++j) {
            if (!GRAM || i <= j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) red[(wave * 4 + r) * 64 + lane] = acc[i][j][r];
                __syncthreads();
                if (wave == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double v = 0.0;
                        for (int w2 = 0; w2 < NW; ++w2) v += red[(w2 * 4 + r) * 64 + lane];
                        const int ca = 16 * i + g + 4 * r, cb = 16 * j + ci;
                        if (ca < ma && cb < w0) out[ca + (int64_t)cb * ma] = v;
                    }
                }
                __syncthreads();
            }
        }
}

template <int WB, typename T, bool UPD, bool TRSM, int TE>
__global__ void __launch_bounds__(ROW_NT, 2) wide_rowop_red_kernel(const FusedArgs fa) {
    rowop_red_body<WB, T, UPD, TRSM, TE>(fa, blockIdx.x, gridDim.x);
}

// Many systems at once (blockIdx.y): workgroup x walks strips x, x + gridDim.x, ... of its
// system; workgroups past the system's strips write no partial sums (the batched reduction
// reads the first ceil(n / ROW_NT) of them).
template <int WB, typename T, bool UPD, bool TRSM, int TE>
__global__ void __launch_bounds__(ROW_NT, 2) wide_rowop_red_kernel_batched(const FusedArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    if ((int64_t)blockIdx.x * ROW_NT >= d.n) return;
    FusedArgs fa = t;
    fa.ra.n = d.n;
    fa.ra.Y = batch_ptr(br, sys, d, t.ra.Y);
    fa.ra.ldy = batch_ld(br, d, t.ra.ldy);
    fa.ra.Qu = batch_ptr(br, sys, d, t.ra.Qu);
    fa.ra.ldqu = batch_ld(br, d, t.ra.ldqu);
    fa.ra.Cu = batch_ptr(br, sys, d, t.ra.Cu);
    fa.ra.Rpk = batch_ptr(br, sys, d, t.ra.Rpk);
    fa.ra.X = batch_ptr(br, sys, d, t.ra.X);
    fa.ra.ldx = batch_ld(br, d, t.ra.ldx);
    fa.E = batch_ptr(br, sys, d, t.E);
    fa.lde = batch_ld(br, d, t.lde);
    fa.partials = batch_ptr(br, sys, d, t.partials);
    rowop_red_body<WB, T, UPD, TRSM, TE>(fa, blockIdx.x, gridDim.x);
}

template <int WB, typename T, bool UPD, bool TRSM, int TE>
int fused_resident() {
    return resident_grid(reinterpret_cast<const void*>(&wide_rowop_red_kernel<WB, T, UPD, TRSM, TE>), ROW_NT);
}

// One system: as many workgroups as are resident (at most the partial-sum capacity), the
// grid returned in *grid.  Batched (br): *grid workgroups per system, given by the caller.
template <int WB, typename T, bool UPD, bool TRSM, int TE>
hipError_t fused_launch(const FusedArgs& fa, int* grid, hipStream_t st, const BatchReloc* br) {
    if (br) {
        hipLaunchKernelGGL((wide_rowop_red_kernel_batched<WB, T, UPD, TRSM, TE>), dim3(*grid, br->nact), dim3(ROW_NT),
                           0, st, fa, *br);
        return hipGetLastError();
    }
    const int64_t strips = (fa.ra.n + ROW_NT - 1) / ROW_NT;
    int64_t cap = skinny_gemm_grid_cap();  // the partial-sum buffers hold this many workgroups
    const int res = fused_resident<WB, T, UPD, TRSM, TE>();
    if (res > 0) cap = std::min<int64_t>(cap, res);
    *grid = (int)std::max<int64_t>(1, std::min<int64_t>(strips, cap));
    hipLaunchKernelGGL((wide_rowop_red_kernel<WB, T, UPD, TRSM, TE>), dim3(*grid), dim3(ROW_NT), 0, st, fa);
    return hipGetLastError();
}

template <int WB, typename T>
hipError_t fused_dispatch(const FusedArgs& fa, int* grid_out, hipStream_t st, const BatchReloc* br) {
    const bool upd = fa.ra.pu > 0, trsm = fa.ra.Rpk != nullptr;
    if (fa.E) {
        if (upd || !trsm) return hipErrorInvalidValue;
        switch ((fa.me + 15) / 16) {
            case 1: return fused_launch<WB, T, false, true, 1>(fa, grid_out, st, br);
            case 2: return fused_launch<WB, T, false, true, 2>(fa, grid_out, st, br);
            default: return fused_launch<WB, T, false, true, 3>(fa, grid_out, st, br);
        }
    }
    // the update form (upd && !trsm) is not fused: measured slower than two sweeps
    if (!upd && trsm) return fused_launch<WB, T, false, true, 0>(fa, grid_out, st, br);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_wide_rowop_reduce(int64_t n, int W, bool f32, const void* Y, int64_t ldy, const void* Qu,
                                    int64_t ldqu, int pu, const double* Cu, const double* Rpk, void* X, int64_t ldx,
                                    const void* E, int64_t lde, int me, double* partials, int* grid_out,
                                    hipStream_t st, const BatchReloc* br) {
    if (W < 1 || W > kFusedMaxW || n < 1 || !grid_out || !partials) return hipErrorInvalidValue;
    if (br && (br->nact < 1 || *grid_out < 1)) return hipErrorInvalidValue;
    if (E && (me < 1 || me > 48)) return hipErrorInvalidValue;
    const FusedArgs fa{RowopArgs{n, W, Y, ldy, Qu, ldqu, pu, Cu, Rpk, X, ldx}, E, lde, E ? me : 0, partials,
                       (int64_t)(E ? me : W) * W};
    if (W <= 16) return f32 ? fused_dispatch<16, float>(fa, grid_out, st, br) : fused_dispatch<16, double>(fa, grid_out, st, br);
    if (W <= 24) return f32 ? fused_dispatch<24, float>(fa, grid_out, st, br) : fused_dispatch<24, double>(fa, grid_out, st, br);
    if (W <= 32) return f32 ? fused_dispatch<32, float>(fa, grid_out, st, br) : fused_dispatch<32, double>(fa, grid_out, st, br);
    return f32 ? fused_dispatch<40, float>(fa, grid_out, st, br) : fused_dispatch<40, double>(fa, grid_out, st, br);
}

}  // namespace sko
