// Kernels for wide blocks (up to 64 columns): the big panels of the two-stage scheme
// (Figs. 5 and 6: CholQR of the big panel, BCGS against the previous big panels).
//
//  wide_rowop   X = (Y - Qu Cu) R^{-1} row by row, one row per thread, the row kept in
//               registers (compile-time maximum width, runtime width); R and Cu are read
//               through the scalar cache.  R comes packed (reciprocal diagonal, then the
//               strictly upper columns back to back): for 61 columns that is 14.6 KB, which
//               the scalar cache holds, where the column-major square spans 18.6 KB of lines
//               and a strip's sweep over it would miss on every chunk.
//  wide_gemm_tn per-workgroup partials of C = A^T B for tall A (n x ma), B (n x nb),
//               ma, nb <= 64, on v_mfma_f64_16x16x4 tiles.  A wave walks 16-row groups;
//               lane l loads rows 4(l/16)..+3 of column 16t + l%16 of every 16-column tile
//               t (one 32-byte piece; the 64 lanes cover 16 columns x 16 rows, whole 128-byte
//               lines).  Because the MFMA A operand (A[l%16][l/16]) and B operand
//               (B[l/16][l%16]) use the same lane mapping, the piece loaded for column tile
//               t is the A operand of output tile row t and the B operand of output tile
//               column t: no LDS staging.  For the Gram matrix (A == B) only output tiles on
//               or above the diagonal are accumulated.
#include <algorithm>
#include <type_traits>

#include "batch.h"
#include "sko_internal.h"
#include "uniform.h"
#include "wide_common.h"

namespace sko {
namespace {

using namespace wide;

// One row per thread, grid-stride over strips of ROW_NT rows.  The factor R and the update
// coefficients are read through the scalar cache (every lane uses the same entry), loaded
// again per strip; only the diagonal reciprocals sit in LDS.
template <int WB, typename T, bool UPD, bool TRSM>
__device__ __forceinline__ void rowop_body(const RowopArgs& ra, const int wg, const int nwg) {
    const int64_t n = ra.n;
    const int w0 = ra.w, pu = ra.pu;
    const T* __restrict__ Y = static_cast<const T*>(ra.Y);
    const T* __restrict__ Qu = static_cast<const T*>(ra.Qu);
    T* X = static_cast<T*>(ra.X);
    __shared__ double sD[TRSM ? WB : 1];
    const int tid = threadIdx.x;
    const uint32_t lane_bytes = (uint32_t)tid * (uint32_t)sizeof(T);
    if constexpr (TRSM) {
        for (int i = tid; i < w0; i += ROW_NT) sD[i] = ra.Rpk[i];
        __syncthreads();
    }
    const CD R0 = as_uniform(ra.Rpk), C0 = as_uniform(ra.Cu);
    for (int64_t r0 = (int64_t)wg * ROW_NT; r0 < n; r0 += (int64_t)nwg * ROW_NT) {
        const int64_t row = r0 + tid;
        if (row >= n) continue;
        const CD Rs = per_strip(R0), Cs = per_strip(C0);
        // column offsets from leading dimensions re-derived per strip (held for the sweep,
        // 64 of them would not fit the SGPRs)
        const int64_t ldy = per_strip(ra.ldy), ldx = per_strip(ra.ldx), ldqu = per_strip(ra.ldqu);
        const int w = per_strip(w0);
        double xa[1][WB];
        double(&x)[WB] = xa[0];
        // Every slot loads, without a branch: slots past the width read the last live column
        // again (same lines, no extra HBM traffic) and are never used.  A per-column branch
        // around the load would hold the FP32-to-FP64 conversion, and with it a wait for
        // that load, inside the branch, one column at a time.
#pragma unroll
        for (int c = 0; c < WB; ++c) x[c] = ldv_nt(lane_elem(Y + r0 + (int64_t)(c < w ? c : w - 1) * ldy, lane_bytes));
        if constexpr (UPD) update_rows<WB, 1, T>(xa, Qu + row, ldqu, pu, Cs, w);
        if constexpr (TRSM) solve_cols<WB, 0>(x, Rs, w, sD);
#pragma unroll
        for (int c = 0; c < WB; ++c)
            if (c < w) stv_nt(lane_elem(X + r0 + (int64_t)c * ldx, lane_bytes), static_cast<T>(x[c]));
    }
}

template <int WB, typename T, bool UPD, bool TRSM>
__global__ void __launch_bounds__(ROW_NT) wide_rowop_kernel(const RowopArgs ra) {
    rowop_body<WB, T, UPD, TRSM>(ra, blockIdx.x, gridDim.x);
}

template <int WB, typename T, bool UPD, bool TRSM>
__global__ void __launch_bounds__(ROW_NT) wide_rowop_kernel_batched(const RowopArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    RowopArgs ra = t;
    ra.n = d.n;
    ra.Y = batch_ptr(br, sys, d, t.Y);
    ra.ldy = batch_ld(br, d, t.ldy);
    ra.Qu = batch_ptr(br, sys, d, t.Qu);
    ra.ldqu = batch_ld(br, d, t.ldqu);
    ra.Cu = batch_ptr(br, sys, d, t.Cu);
    ra.Rpk = batch_ptr(br, sys, d, t.Rpk);
    ra.X = batch_ptr(br, sys, d, t.X);
    ra.ldx = batch_ld(br, d, t.ldx);
    rowop_body<WB, T, UPD, TRSM>(ra, blockIdx.x, gridDim.x);
}

// TA = ceil(ma / 16) and TB = ceil(nb / 16) tiles at compile time: only the accumulators
// and pieces a launch uses occupy registers (more resident waves to cover the load latency).
template <typename T, bool SYM, int TA, int TB>
__device__ __forceinline__ void gemm_body(const GemmArgs& ga) {
    __shared__ double red[4 * 64 * (GT / 64)];
    const int64_t n = ga.n;
    const T* A = static_cast<const T*>(ga.A);
    const T* B = static_cast<const T*>(ga.B);
    const int ma = ga.ma, nb = ga.nb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ci = lane & 15, g = lane >> 4;
    constexpr int NW = GT / 64;
    // 4-row pieces can be read as vectors when every column start is aligned
    const bool veca = (ga.lda % 4) == 0 && ((uintptr_t)A % (4 * sizeof(T))) == 0;
    const bool vecb = (ga.ldb % 4) == 0 && ((uintptr_t)B % (4 * sizeof(T))) == 0;
    double4_t acc[TA][TB];
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

    const int64_t ngroups = (n + 15) / 16;
    for (int64_t grp = (int64_t)blockIdx.x * NW + wave; grp < ngroups; grp += (int64_t)gridDim.x * NW) {
        const int64_t row0 = grp * 16 + 4 * g;
        const bool full = grp * 16 + 16 <= n;
        double a[TA][4], b[SYM ? 1 : TB][4];
        load_pieces<T, TA>(A, ga.lda, ma, ci, veca, full, row0, n, a);
        if constexpr (!SYM) load_pieces<T, TB>(B, ga.ldb, nb, ci, vecb, full, row0, n, b);
        // row step outermost: consecutive MFMAs go to different accumulator tiles
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < TA; ++i)
#pragma unroll
                for (int j = 0; j < TB; ++j) {
                    if (!SYM || i <= j) {
                        const double bj = SYM ? a[j][u] : b[SYM ? 0 : j][u];
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][u], bj, acc[i][j], 0, 0, 0);
                    }
                }
    }

    // D[r][c] of a tile sits in lane c + 16 (r % 4), element r / 4; the waves' tiles are
    // summed through LDS in wave order and written once per workgroup
    double* out = ga.partials + (int64_t)blockIdx.x * ga.stride;
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) {
            if (!SYM || i <= j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) red[(wave * 4 + r) * 64 + lane] = acc[i][j][r];
                __syncthreads();
                if (wave == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double v = 0.0;
                        for (int w2 = 0; w2 < NW; ++w2) v += red[(w2 * 4 + r) * 64 + lane];
                        const int ca = 16 * i + g + 4 * r, cb = 16 * j + ci;
                        if (ca < ma && cb < nb) out[ca + (int64_t)cb * ma] = v;
                    }
                }
                __syncthreads();
            }
        }
}

template <typename T, bool SYM, int TA, int TB>
__global__ void __launch_bounds__(GT) wide_gemm_tn_kernel(const GemmArgs ga) {
    gemm_body<T, SYM, TA, TB>(ga);
}

template <typename T, bool SYM, int TA, int TB>
__global__ void __launch_bounds__(GT) wide_gemm_tn_kernel_batched(const GemmArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    GemmArgs ga = t;
    ga.n = d.n;
    ga.A = batch_ptr(br, sys, d, t.A);
    ga.lda = batch_ld(br, d, t.lda);
    ga.B = batch_ptr(br, sys, d, t.B);
    ga.ldb = batch_ld(br, d, t.ldb);
    ga.partials = batch_ptr(br, sys, d, t.partials);
    gemm_body<T, SYM, TA, TB>(ga);
}

template <int WB, typename T, bool UPD, bool TRSM>
void rowop_launch(const RowopArgs& ra, hipStream_t st, const BatchReloc* br) {
    const int64_t strips = (ra.n + ROW_NT - 1) / ROW_NT;
    if (br) {
        // many systems at once: each workgroup takes up to 8 strips of its system
        const int grid = (int)((strips + 7) / 8);
        hipLaunchKernelGGL((wide_rowop_kernel_batched<WB, T, UPD, TRSM>), dim3(grid, br->nact), dim3(ROW_NT), 0, st,
                           ra, *br);
        return;
    }
    // resident workgroups only: each walks its strips
    int cap = resident_grid(reinterpret_cast<const void*>(&wide_rowop_kernel<WB, T, UPD, TRSM>), ROW_NT);
    if (cap < 1) cap = 1024;
    const int grid = (int)std::min<int64_t>(strips, cap);
    hipLaunchKernelGGL((wide_rowop_kernel<WB, T, UPD, TRSM>), dim3(grid), dim3(ROW_NT), 0, st, ra);
}

template <int WB, typename T>
hipError_t rowop_dispatch(const RowopArgs& ra, hipStream_t st, const BatchReloc* br) {
    if (ra.pu > 0 && ra.Rpk)
        rowop_launch<WB, T, true, true>(ra, st, br);
    else if (ra.pu > 0)
        rowop_launch<WB, T, true, false>(ra, st, br);
    else if (ra.Rpk)
        rowop_launch<WB, T, false, true>(ra, st, br);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T, bool SYM, int TA, int TB>
void gemm_launch_t(const GemmArgs& ga, int grid, hipStream_t st, const BatchReloc* br) {
    if (br)
        hipLaunchKernelGGL((wide_gemm_tn_kernel_batched<T, SYM, TA, TB>), dim3(grid, br->nact), dim3(GT), 0, st, ga,
                           *br);
    else
        hipLaunchKernelGGL((wide_gemm_tn_kernel<T, SYM, TA, TB>), dim3(grid), dim3(GT), 0, st, ga);
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<TA>, IC<TB>) for the tile counts of ma x nb (each 1..4).
template <typename F>
void tile_dispatch(int ma, int nb, F&& f) {
    const int ta = (ma + 15) / 16, tb = (nb + 15) / 16;
    auto inner = [&](auto tac) {
        switch (tb) {
            case 1: f(tac, IC<1>{}); break;
            case 2: f(tac, IC<2>{}); break;
            case 3: f(tac, IC<3>{}); break;
            default: f(tac, IC<4>{}); break;
        }
    };
    switch (ta) {
        case 1: inner(IC<1>{}); break;
        case 2: inner(IC<2>{}); break;
        case 3: inner(IC<3>{}); break;
        default: inner(IC<4>{}); break;
    }
}

template <typename T, bool SYM>
void gemm_launch(const GemmArgs& ga, int grid, hipStream_t st, const BatchReloc* br) {
    if constexpr (SYM) {
        // A == B: square tile grid
        switch ((ga.ma + 15) / 16) {
            case 1: gemm_launch_t<T, true, 1, 1>(ga, grid, st, br); break;
            case 2: gemm_launch_t<T, true, 2, 2>(ga, grid, st, br); break;
            case 3: gemm_launch_t<T, true, 3, 3>(ga, grid, st, br); break;
            default: gemm_launch_t<T, true, 4, 4>(ga, grid, st, br); break;
        }
    } else {
        tile_dispatch(ga.ma, ga.nb, [&](auto ta, auto tb) {
            gemm_launch_t<T, false, decltype(ta)::value, decltype(tb)::value>(ga, grid, st, br);
        });
    }
}

}  // namespace

hipError_t launch_wide_rowop(int64_t n, int W, bool f32, const void* Y, int64_t ldy, const void* Qu, int64_t ldqu,
                             int pu, const double* Cu, const double* Rpk, void* X, int64_t ldx, hipStream_t st,
                             const BatchReloc* br) {
    if (W < 1 || W > 64 || n < 1) return hipErrorInvalidValue;
    if (br && br->nact < 1) return hipErrorInvalidValue;
    const RowopArgs ra{n, W, Y, ldy, Qu, ldqu, pu, Cu, Rpk, X, ldx};
    if (W <= 16) return f32 ? rowop_dispatch<16, float>(ra, st, br) : rowop_dispatch<16, double>(ra, st, br);
    if (W <= 24) return f32 ? rowop_dispatch<24, float>(ra, st, br) : rowop_dispatch<24, double>(ra, st, br);
    if (W <= 32) return f32 ? rowop_dispatch<32, float>(ra, st, br) : rowop_dispatch<32, double>(ra, st, br);
    if (W <= 40) return f32 ? rowop_dispatch<40, float>(ra, st, br) : rowop_dispatch<40, double>(ra, st, br);
    if (W <= 48) return f32 ? rowop_dispatch<48, float>(ra, st, br) : rowop_dispatch<48, double>(ra, st, br);
    return f32 ? rowop_dispatch<64, float>(ra, st, br) : rowop_dispatch<64, double>(ra, st, br);
}

template <typename T, bool SYM, int TA, int TB>
int gemm_resident_t() {
    return resident_grid(reinterpret_cast<const void*>(&wide_gemm_tn_kernel<T, SYM, TA, TB>), GT);
}

template <typename T>
int gemm_resident(bool sym, int ma, int nb) {
    int r = -1;
    if (sym) {
        switch ((ma + 15) / 16) {
            case 1: r = gemm_resident_t<T, true, 1, 1>(); break;
            case 2: r = gemm_resident_t<T, true, 2, 2>(); break;
            case 3: r = gemm_resident_t<T, true, 3, 3>(); break;
            default: r = gemm_resident_t<T, true, 4, 4>(); break;
        }
    } else {
        tile_dispatch(ma, nb, [&](auto ta, auto tb) {
            r = gemm_resident_t<T, false, decltype(ta)::value, decltype(tb)::value>();
        });
    }
    return r;
}

int skinny_gemm_resident(bool sym, bool f32, int ma, int nb) {
    return f32 ? gemm_resident<float>(sym, ma, nb) : gemm_resident<double>(sym, ma, nb);
}

int skinny_gemm_grid_cap() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    return 4 * (cus > 0 ? cus : 1);
}

hipError_t launch_skinny_gemm_tn(int64_t n, const void* A, int64_t lda, int ma, const void* B, int64_t ldb, int nb,
                                 bool f32, double* partials, int grid, hipStream_t st, const BatchReloc* br) {
    if (ma < 1 || nb < 1 || ma > 64 || nb > 64 || grid < 1) return hipErrorInvalidValue;
    if (br && br->nact < 1) return hipErrorInvalidValue;
    const bool sym = (A == B) && (lda == ldb) && (ma == nb);
    const GemmArgs ga{n, A, lda, ma, B, ldb, nb, partials, (int64_t)ma * nb};
    if (f32) {
        if (sym)
            gemm_launch<float, true>(ga, grid, st, br);
        else
            gemm_launch<float, false>(ga, grid, st, br);
    } else {
        if (sym)
            gemm_launch<double, true>(ga, grid, st, br);
        else
            gemm_launch<double, false>(ga, grid, st, br);
    }
    return hipGetLastError();
}

}  // namespace sko
