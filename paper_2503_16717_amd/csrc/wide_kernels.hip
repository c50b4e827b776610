// Kernels for wide blocks (up to 64 columns): the big panels of the two-stage scheme
// (Figs. 5 and 6: CholQR of the big panel, BCGS against the previous big panels).
//
//  wide_rowop   X = (Y - Qu Cu) R^{-1} row by row, one row per thread, the row kept in
//               registers (compile-time maximum width, runtime width).
//  wide_gemm_tn per-workgroup partials of C = A^T B for tall A (n x ma), B (n x nb),
//               ma, nb <= 64, on v_mfma_f64_16x16x4 tiles.  A wave walks 16-row groups;
//               lane l loads rows 4(l/16)..+3 of column 16t + l%16 of every 16-column tile
//               t (one 32-byte piece; the 64 lanes cover 16 columns x 16 rows, whole 128-byte
//               lines).  Because the MFMA A operand (A[l%16][l/16]) and B operand
//               (B[l/16][l%16]) use the same lane mapping, the piece loaded for column tile
//               t is the A operand of output tile row t and the B operand of output tile
//               column t: no LDS staging.  For the Gram matrix (A == B) only output tiles on
//               or above the diagonal are accumulated.
#include "batch.h"
#include "sko_internal.h"

namespace sko {
namespace {

template <typename T>
__device__ __forceinline__ double ldv(const T* p) {
    return static_cast<double>(*p);
}

constexpr int ROW_NT = 256;

struct RowopArgs {
    int64_t n;
    int w;
    const void* Y;
    int64_t ldy;
    const void* Qu;
    int64_t ldqu;
    int pu;
    const double* Cu;
    const double* R;
    void* X;
    int64_t ldx;
};

template <int WB, typename T, bool UPD, bool TRSM>
__device__ __forceinline__ void rowop_body(const RowopArgs& ra) {
    const int64_t n = ra.n;
    const int w = ra.w, pu = ra.pu;
    const T* __restrict__ Y = static_cast<const T*>(ra.Y);
    const T* __restrict__ Qu = static_cast<const T*>(ra.Qu);
    const double* __restrict__ Cu = ra.Cu;
    const double* __restrict__ R = ra.R;
    T* X = static_cast<T*>(ra.X);
    const int64_t ldy = ra.ldy, ldqu = ra.ldqu, ldx = ra.ldx;
    extern __shared__ double lds[];
    double* sR = lds;                              // w * w, then the w diagonal reciprocals
    double* sD = lds + w * w;
    double* sC = lds + (TRSM ? w * w + w : 0);     // pu * w
    const int tid = threadIdx.x;
    if (TRSM) {
        for (int i = tid; i < w * w; i += ROW_NT) sR[i] = R[i];
        for (int i = tid; i < w; i += ROW_NT) sD[i] = 1.0 / R[i + i * w];
    }
    if (UPD)
        for (int i = tid; i < pu * w; i += ROW_NT) sC[i] = Cu[i];
    __syncthreads();
    for (int64_t row = (int64_t)blockIdx.x * ROW_NT + tid; row < n; row += (int64_t)gridDim.x * ROW_NT) {
    double x[WB];
#pragma unroll
    for (int c = 0; c < WB; ++c) x[c] = (c < w) ? ldv(Y + row + (int64_t)c * ldy) : 0.0;
    if (UPD) {
        for (int a = 0; a < pu; ++a) {
            const double q = ldv(Qu + row + (int64_t)a * ldqu);
#pragma unroll
            for (int c = 0; c < WB; ++c)
                if (c < w) x[c] -= q * sC[a + c * pu];
        }
    }
    if (TRSM) {
#pragma unroll
        for (int c = 0; c < WB; ++c) {
            if (c < w) {
                double v = x[c];
#pragma unroll
                for (int q = 0; q < c; ++q) v -= x[q] * sR[q + c * w];
                x[c] = v * sD[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < WB; ++c)
        if (c < w) X[row + (int64_t)c * ldx] = static_cast<T>(x[c]);
    }
}

template <int WB, typename T, bool UPD, bool TRSM>
__global__ void __launch_bounds__(ROW_NT) wide_rowop_kernel(const RowopArgs ra) {
    rowop_body<WB, T, UPD, TRSM>(ra);
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
    ra.R = batch_ptr(br, sys, d, t.R);
    ra.X = batch_ptr(br, sys, d, t.X);
    ra.ldx = batch_ld(br, d, t.ldx);
    rowop_body<WB, T, UPD, TRSM>(ra);
}

constexpr int GT = 256;   // threads (4 waves)

typedef double double4_t __attribute__((ext_vector_type(4)));

struct GemmArgs {
    int64_t n;
    const void* A;
    int64_t lda;
    int ma;
    const void* B;
    int64_t ldb;
    int nb;
    double* partials;
    int64_t stride;
};

// Rows row0..row0+3 of one column into v (zero past n or for a column past the block).
template <typename T>
__device__ __forceinline__ void load_piece(const T* col, bool live, bool vec, int64_t row0, int64_t n, double v[4]) {
    if (!live) {
        v[0] = v[1] = v[2] = v[3] = 0.0;
    } else if (vec && row0 + 3 < n) {
        if constexpr (sizeof(T) == 8) {
            const double2 p0 = *reinterpret_cast<const double2*>(col + row0);
            const double2 p1 = *reinterpret_cast<const double2*>(col + row0 + 2);
            v[0] = p0.x;
            v[1] = p0.y;
            v[2] = p1.x;
            v[3] = p1.y;
        } else {
            const float4 p = *reinterpret_cast<const float4*>(col + row0);
            v[0] = p.x;
            v[1] = p.y;
            v[2] = p.z;
            v[3] = p.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (row0 + u < n) ? ldv(col + row0 + u) : 0.0;
    }
}

template <typename T, bool SYM>
__device__ __forceinline__ void gemm_body(const GemmArgs& ga) {
    __shared__ double red[4 * 64 * (GT / 64)];
    const int64_t n = ga.n;
    const T* A = static_cast<const T*>(ga.A);
    const T* B = static_cast<const T*>(ga.B);
    const int ma = ga.ma, nb = ga.nb;
    const int ta = (ma + 15) / 16, tb = (nb + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ci = lane & 15, g = lane >> 4;
    constexpr int NW = GT / 64;
    // 4-row pieces can be read as vectors when every column start is aligned
    const bool veca = (ga.lda % 4) == 0 && ((uintptr_t)A % (4 * sizeof(T))) == 0;
    const bool vecb = (ga.ldb % 4) == 0 && ((uintptr_t)B % (4 * sizeof(T))) == 0;
    double4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

    const int64_t ngroups = (n + 15) / 16;
    for (int64_t grp = (int64_t)blockIdx.x * NW + wave; grp < ngroups; grp += (int64_t)gridDim.x * NW) {
        const int64_t row0 = grp * 16 + 4 * g;
        double a[4][4], b[SYM ? 1 : 4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = 16 * t + ci;
            if (t < ta) load_piece(A + (int64_t)(c < ma ? c : 0) * ga.lda, c < ma, veca, row0, n, a[t]);
        }
        if constexpr (!SYM) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 16 * t + ci;
                if (t < tb) load_piece(B + (int64_t)(c < nb ? c : 0) * ga.ldb, c < nb, vecb, row0, n, b[t]);
            }
        }
        // row step outermost: consecutive MFMAs go to different accumulator tiles
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (i < ta && j < tb && (!SYM || i <= j)) {
                        const double bj = SYM ? a[j][u] : b[SYM ? 0 : j][u];
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][u], bj, acc[i][j], 0, 0, 0);
                    }
                }
    }

    // D[r][c] of a tile sits in lane c + 16 (r % 4), element r / 4; the waves' tiles are
    // summed through LDS in wave order and written once per workgroup
    double* out = ga.partials + (int64_t)blockIdx.x * ga.stride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i < ta && j < tb && (!SYM || i <= j)) {
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

template <typename T, bool SYM>
__global__ void __launch_bounds__(GT) wide_gemm_tn_kernel(const GemmArgs ga) {
    gemm_body<T, SYM>(ga);
}

template <typename T, bool SYM>
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
    gemm_body<T, SYM>(ga);
}

template <int WB, typename T, bool UPD, bool TRSM>
void rowop_launch(const RowopArgs& ra, int grid, size_t lds, hipStream_t st, const BatchReloc* br) {
    if (br)
        hipLaunchKernelGGL((wide_rowop_kernel_batched<WB, T, UPD, TRSM>), dim3(grid, br->nact), dim3(ROW_NT), lds, st,
                           ra, *br);
    else
        hipLaunchKernelGGL((wide_rowop_kernel<WB, T, UPD, TRSM>), dim3(grid), dim3(ROW_NT), lds, st, ra);
}

template <int WB, typename T>
hipError_t rowop_dispatch(const RowopArgs& ra, hipStream_t st, const BatchReloc* br) {
    // one row per thread; in a batched launch (many systems at once) each workgroup takes
    // up to 8 strips of its system
    const int64_t strips = (ra.n + ROW_NT - 1) / ROW_NT;
    const int grid = (int)(br ? (strips + 7) / 8 : strips);
    const size_t lds = sizeof(double) * ((ra.R ? (size_t)ra.w * ra.w + ra.w : 0) + (ra.pu > 0 ? (size_t)ra.pu * ra.w : 0));
    if (ra.pu > 0 && ra.R)
        rowop_launch<WB, T, true, true>(ra, grid, lds, st, br);
    else if (ra.pu > 0)
        rowop_launch<WB, T, true, false>(ra, grid, lds, st, br);
    else if (ra.R)
        rowop_launch<WB, T, false, true>(ra, grid, lds, st, br);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T, bool SYM>
void gemm_launch(const GemmArgs& ga, int grid, hipStream_t st, const BatchReloc* br) {
    if (br)
        hipLaunchKernelGGL((wide_gemm_tn_kernel_batched<T, SYM>), dim3(grid, br->nact), dim3(GT), 0, st, ga, *br);
    else
        hipLaunchKernelGGL((wide_gemm_tn_kernel<T, SYM>), dim3(grid), dim3(GT), 0, st, ga);
}

}  // namespace

hipError_t launch_wide_rowop(int64_t n, int W, bool f32, const void* Y, int64_t ldy, const void* Qu, int64_t ldqu,
                             int pu, const double* Cu, const double* R, void* X, int64_t ldx, hipStream_t st,
                             const BatchReloc* br) {
    if (W < 1 || W > 64 || n < 1) return hipErrorInvalidValue;
    if (br && br->nact < 1) return hipErrorInvalidValue;
    if (sizeof(double) * ((R ? (size_t)W * W + W : 0) + (size_t)(pu > 0 ? pu : 0) * W) > 60 * 1024)
        return hipErrorInvalidValue;
    const RowopArgs ra{n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx};
    if (W <= 16) return f32 ? rowop_dispatch<16, float>(ra, st, br) : rowop_dispatch<16, double>(ra, st, br);
    if (W <= 24) return f32 ? rowop_dispatch<24, float>(ra, st, br) : rowop_dispatch<24, double>(ra, st, br);
    if (W <= 32) return f32 ? rowop_dispatch<32, float>(ra, st, br) : rowop_dispatch<32, double>(ra, st, br);
    if (W <= 40) return f32 ? rowop_dispatch<40, float>(ra, st, br) : rowop_dispatch<40, double>(ra, st, br);
    if (W <= 48) return f32 ? rowop_dispatch<48, float>(ra, st, br) : rowop_dispatch<48, double>(ra, st, br);
    return f32 ? rowop_dispatch<64, float>(ra, st, br) : rowop_dispatch<64, double>(ra, st, br);
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
