// Kernels for wide blocks (up to 64 columns): the big panels of the two-stage scheme
// (Figs. 5 and 6: CholQR of the big panel, BCGS against the previous big panels).
//
//  wide_rowop   X = (Y - Qu Cu) R^{-1} row by row, one row per thread, the row kept in
//               registers (compile-time maximum width, runtime width).
//  wide_gemm_tn per-workgroup partials of C = A^T B for tall A (n x ma), B (n x nb),
//               ma, nb <= 64: 32-row strips of A and B staged in LDS, each of 256 threads
//               accumulating a 4 x 4 tile of C in registers.  For the Gram matrix (A == B)
//               only tiles on or above the diagonal are computed.
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
    double* sR = lds;                          // w * w
    double* sC = lds + (TRSM ? w * w : 0);     // pu * w
    const int tid = threadIdx.x;
    if (TRSM)
        for (int i = tid; i < w * w; i += ROW_NT) sR[i] = R[i];
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
                x[c] = v / sR[c + c * w];
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

constexpr int GT = 256;   // threads
constexpr int GS = 32;    // rows per strip
constexpr int GLD = 65;   // padded LDS row length

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

template <typename T, bool SYM>
__device__ __forceinline__ void gemm_body(const GemmArgs& ga) {
    const int64_t n = ga.n;
    const T* __restrict__ A = static_cast<const T*>(ga.A);
    const T* __restrict__ B = static_cast<const T*>(ga.B);
    const int64_t lda = ga.lda, ldb = ga.ldb;
    const int ma = ga.ma, nb = ga.nb;
    __shared__ double As[GS * GLD];
    __shared__ double Bs[SYM ? 1 : GS * GLD];
    const int tid = threadIdx.x;
    const int ti = tid / 16, tj = tid % 16;
    const bool active = !SYM || ti <= tj;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int64_t nstrips = (n + GS - 1) / GS;
    for (int64_t s = blockIdx.x; s < nstrips; s += gridDim.x) {
        const int64_t base = s * GS;
        for (int idx = tid; idx < GS * ma; idx += GT) {
            const int r = idx % GS, c = idx / GS;
            const int64_t row = base + r;
            As[r * GLD + c] = row < n ? ldv(A + row + (int64_t)c * lda) : 0.0;
        }
        if (!SYM) {
            for (int idx = tid; idx < GS * nb; idx += GT) {
                const int r = idx % GS, c = idx / GS;
                const int64_t row = base + r;
                Bs[r * GLD + c] = row < n ? ldv(B + row + (int64_t)c * ldb) : 0.0;
            }
        }
        __syncthreads();
        const double* Bsrc = SYM ? As : Bs;
        if (active) {
            for (int r = 0; r < GS; ++r) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ca = 4 * ti + i, cb = 4 * tj + i;
                    a[i] = ca < ma ? As[r * GLD + ca] : 0.0;
                    b[i] = cb < nb ? Bsrc[r * GLD + cb] : 0.0;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
            }
        }
        __syncthreads();
    }
    double* out = ga.partials + (int64_t)blockIdx.x * ga.stride;
    if (active) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ca = 4 * ti + i, cb = 4 * tj + j;
                if (ca < ma && cb < nb) out[ca + (int64_t)cb * ma] = acc[i][j];
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
    const size_t lds = sizeof(double) * ((ra.R ? (size_t)ra.w * ra.w : 0) + (ra.pu > 0 ? (size_t)ra.pu * ra.w : 0));
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
    if (sizeof(double) * ((R ? (size_t)W * W : 0) + (size_t)(pu > 0 ? pu : 0) * W) > 60 * 1024)
        return hipErrorInvalidValue;
    const RowopArgs ra{n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx};
    if (W <= 16) return f32 ? rowop_dispatch<16, float>(ra, st, br) : rowop_dispatch<16, double>(ra, st, br);
    if (W <= 32) return f32 ? rowop_dispatch<32, float>(ra, st, br) : rowop_dispatch<32, double>(ra, st, br);
    return f32 ? rowop_dispatch<64, float>(ra, st, br) : rowop_dispatch<64, double>(ra, st, br);
}

int skinny_gemm_grid_cap() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    return 2 * (cus > 0 ? cus : 1);
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
