// Kernels for wide blocks (up to 64 columns): the big panels of the two-stage scheme
// (Figs. 5 and 6: CholQR of the big panel, BCGS against the previous big panels).
//
//  wide_rowop   X = (Y - Qu Cu) R^{-1} row by row, one row per thread, the row kept in
//               registers (compile-time maximum width, runtime width).
//  wide_gemm_tn per-workgroup partials of C = A^T B for tall A (n x ma), B (n x nb),
//               ma, nb <= 64: 32-row strips of A and B staged in LDS, each of 256 threads
//               accumulating a 4 x 4 tile of C in registers.  For the Gram matrix (A == B)
//               only tiles on or above the diagonal are computed.
#include "sko_internal.h"

namespace sko {
namespace {

template <typename T>
__device__ __forceinline__ double ldv(const T* p) {
    return static_cast<double>(*p);
}

constexpr int ROW_NT = 256;

template <int WB, typename T, bool UPD, bool TRSM>
__global__ void __launch_bounds__(ROW_NT) wide_rowop_kernel(int64_t n, int w, const T* __restrict__ Y, int64_t ldy,
                                                            const T* __restrict__ Qu, int64_t ldqu, int pu,
                                                            const double* __restrict__ Cu,
                                                            const double* __restrict__ R, T* X, int64_t ldx) {
    extern __shared__ double lds[];
    double* sR = lds;                          // w * w
    double* sC = lds + (TRSM ? w * w : 0);     // pu * w
    const int tid = threadIdx.x;
    if (TRSM)
        for (int i = tid; i < w * w; i += ROW_NT) sR[i] = R[i];
    if (UPD)
        for (int i = tid; i < pu * w; i += ROW_NT) sC[i] = Cu[i];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * ROW_NT + tid;
    if (row >= n) return;
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

constexpr int GT = 256;   // threads
constexpr int GS = 32;    // rows per strip
constexpr int GLD = 65;   // padded LDS row length

template <typename T, bool SYM>
__global__ void __launch_bounds__(GT) wide_gemm_tn_kernel(int64_t n, const T* __restrict__ A, int64_t lda, int ma,
                                                          const T* __restrict__ B, int64_t ldb, int nb,
                                                          double* partials, int64_t stride) {
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
    double* out = partials + (int64_t)blockIdx.x * stride;
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

template <int WB, typename T>
hipError_t rowop_dispatch(int64_t n, int w, const void* Y, int64_t ldy, const void* Qu, int64_t ldqu, int pu,
                          const double* Cu, const double* R, void* X, int64_t ldx, hipStream_t st) {
    const int grid = (int)((n + ROW_NT - 1) / ROW_NT);
    const size_t lds = sizeof(double) * ((R ? (size_t)w * w : 0) + (pu > 0 ? (size_t)pu * w : 0));
    const T* y = static_cast<const T*>(Y);
    const T* q = static_cast<const T*>(Qu);
    T* x = static_cast<T*>(X);
    if (pu > 0 && R)
        hipLaunchKernelGGL((wide_rowop_kernel<WB, T, true, true>), dim3(grid), dim3(ROW_NT), lds, st, n, w, y, ldy, q,
                           ldqu, pu, Cu, R, x, ldx);
    else if (pu > 0)
        hipLaunchKernelGGL((wide_rowop_kernel<WB, T, true, false>), dim3(grid), dim3(ROW_NT), lds, st, n, w, y, ldy, q,
                           ldqu, pu, Cu, R, x, ldx);
    else if (R)
        hipLaunchKernelGGL((wide_rowop_kernel<WB, T, false, true>), dim3(grid), dim3(ROW_NT), lds, st, n, w, y, ldy, q,
                           ldqu, pu, Cu, R, x, ldx);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_wide_rowop(int64_t n, int W, bool f32, const void* Y, int64_t ldy, const void* Qu, int64_t ldqu,
                             int pu, const double* Cu, const double* R, void* X, int64_t ldx, hipStream_t st) {
    if (W < 1 || W > 64 || n < 1) return hipErrorInvalidValue;
    if (sizeof(double) * ((R ? (size_t)W * W : 0) + (size_t)(pu > 0 ? pu : 0) * W) > 60 * 1024)
        return hipErrorInvalidValue;
    if (W <= 16)
        return f32 ? rowop_dispatch<16, float>(n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx, st)
                   : rowop_dispatch<16, double>(n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx, st);
    if (W <= 32)
        return f32 ? rowop_dispatch<32, float>(n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx, st)
                   : rowop_dispatch<32, double>(n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx, st);
    return f32 ? rowop_dispatch<64, float>(n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx, st)
               : rowop_dispatch<64, double>(n, W, Y, ldy, Qu, ldqu, pu, Cu, R, X, ldx, st);
}

int skinny_gemm_grid_cap() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    return 2 * (cus > 0 ? cus : 1);
}

hipError_t launch_skinny_gemm_tn(int64_t n, const void* A, int64_t lda, int ma, const void* B, int64_t ldb, int nb,
                                 bool f32, double* partials, int grid, hipStream_t st) {
    if (ma < 1 || nb < 1 || ma > 64 || nb > 64 || grid < 1) return hipErrorInvalidValue;
    const bool sym = (A == B) && (lda == ldb) && (ma == nb);
    const int64_t stride = (int64_t)ma * nb;
    if (f32) {
        const float* a = static_cast<const float*>(A);
        const float* b = static_cast<const float*>(B);
        if (sym)
            hipLaunchKernelGGL((wide_gemm_tn_kernel<float, true>), dim3(grid), dim3(GT), 0, st, n, a, lda, ma, b, ldb,
                               nb, partials, stride);
        else
            hipLaunchKernelGGL((wide_gemm_tn_kernel<float, false>), dim3(grid), dim3(GT), 0, st, n, a, lda, ma, b,
                               ldb, nb, partials, stride);
    } else {
        const double* a = static_cast<const double*>(A);
        const double* b = static_cast<const double*>(B);
        if (sym)
            hipLaunchKernelGGL((wide_gemm_tn_kernel<double, true>), dim3(grid), dim3(GT), 0, st, n, a, lda, ma, b,
                               ldb, nb, partials, stride);
        else
            hipLaunchKernelGGL((wide_gemm_tn_kernel<double, false>), dim3(grid), dim3(GT), 0, st, n, a, lda, ma, b,
                               ldb, nb, partials, stride);
    }
    return hipGetLastError();
}

}  // namespace sko
