// Device kernels of restarted s-step GMRES (Fig. 1, Fig. 5):
//   * CSR SpMV for the matrix-powers kernel (MPK), L lanes per row, FP64 accumulation,
//     double or float vectors and values;
//   * explicit residual r = b - A x (FP64) written into the first basis column, with
//     per-workgroup partial sums of r^2;
//   * solution update x += D^{-1} Q y;
//   * Jacobi set-up: D^{-1} and the column-scaled values of A D^{-1};
//   * the small Hessenberg bookkeeping (T_in / T_out, Givens least squares).
#include <cmath>

#include "batch.h"
#include "gmres_internal.h"
#include "hessenberg_eig.h"
#include "uniform.h"

namespace sko {
namespace {

constexpr int NT = 256;

template <typename T>
__device__ __forceinline__ double ld_(const T* p) {
    return static_cast<double>(*p);
}
// Streamed operands read exactly once (the staged copy of a workgroup's matrix values and
// column indices) are loaded non-temporally, so they do not push the gathered vector out of
// the L2.  (The lanes-per-row kernels read each line of them in two passes and keep normal
// loads.)
__device__ __forceinline__ int32_t ldnt_i(const int32_t* p) { return __builtin_nontemporal_load(p); }

// Orders one wave's LDS accesses: writes before the barrier are seen by reads after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Newton-basis step of the matrix-powers kernel (a device pair, null for a monomial step):
// y = A x - a x + b z, with a = *na, b = *nb (z: the vector before x, read only if b != 0).
template <typename TX>
struct NewtonStep {
    const double* na = nullptr;
    const double* nb = nullptr;
    const TX* z = nullptr;
};

template <typename TX>
__device__ __forceinline__ double newton_term(const NewtonStep<TX>& ns, const TX* __restrict__ x, int64_t row) {
    if (!ns.na) return 0.0;
    double t = -(*ns.na) * ld_(x + row);
    const double b = *ns.nb;
    if (b != 0.0) t += b * ld_(ns.z + row);
    return t;
}

// y = A x with L lanes per row, workgroup wg of nwg striding over groups of NT/L rows.
template <int L, typename TV, typename TX, typename TY>
__device__ __forceinline__ void spmv_rows(int64_t n, const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ colind, const TV* __restrict__ val,
                                          const TX* __restrict__ x, TY* __restrict__ y, int wg, int nwg,
                                          const NewtonStep<TX>& ns = NewtonStep<TX>{}) {
    const int tid = threadIdx.x;
    const int sub = tid % L;
    const int64_t rows_per_block = NT / L;
    for (int64_t base = (int64_t)wg * rows_per_block; base < n; base += (int64_t)nwg * rows_per_block) {
        const int64_t row = base + tid / L;
        double sum = 0.0;
        if (row < n) {
            const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
            for (int32_t e = e0 + sub; e < e1; e += L) sum += ld_(val + e) * ld_(x + colind[e]);
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (sub == 0 && row < n) y[row] = static_cast<TY>(sum + newton_term(ns, x, row));
    }
}

template <int L, typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(NT) spmv_kernel(int64_t n, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind, const TV* __restrict__ val,
                                                  const TX* __restrict__ x, TY* __restrict__ y,
                                                  const NewtonStep<TX> ns) {
    spmv_rows<L, TV, TX, TY>(n, rowptr, colind, val, x, y, blockIdx.x, gridDim.x, ns);
}

// One row per thread; each workgroup first copies the contiguous nonzero range of its NT
// rows into LDS with coalesced loads (when it holds at most 8 entries per row on average,
// else the rows read the arrays directly), so the per-row loops touch only LDS and x.
constexpr int STAGE = 8 * NT;

typedef float f4v_t __attribute__((ext_vector_type(4)));
typedef int i4v_t __attribute__((ext_vector_type(4)));

// nnz: length of the value and index arrays (bounds the 16-byte staging loads).  FP32
// values are staged with 16-byte loads of four values and four indices from the aligned
// element at or below the range start (the up to three elements before it land in LDS slots
// no row reads): 121 -> 112 us on the 192^3 7-point matrix.  FP64 values gained nothing
// from it and keep single-element loads.
template <typename TV, typename TX, typename TY>
__device__ __forceinline__ void spmv_staged_body(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ colind, const TV* __restrict__ val,
                                                 const TX* __restrict__ x, TY* __restrict__ y, int wg, int nwg,
                                                 const NewtonStep<TX>& ns = NewtonStep<TX>{}) {
    __shared__ TV sv[STAGE + 4];
    __shared__ int32_t sc[STAGE + 4];
    const int tid = threadIdx.x;
    const bool vec = sizeof(TV) == 4 && ((uintptr_t)val % 16) == 0 && ((uintptr_t)colind % 16) == 0;
    for (int64_t base = (int64_t)wg * NT; base < n; base += (int64_t)nwg * NT) {
        const int64_t rend = base + NT < n ? base + NT : n;
        const int32_t e0 = rowptr[base], e1 = rowptr[rend], cnt = e1 - e0;
        const bool staged = cnt <= STAGE;
        // LDS slot of element e: e - o
        const int32_t o = vec ? (e0 & ~3) : e0;
        if (staged) {
            if (vec) {
                const int32_t nv = (e1 - o + 3) / 4;
                for (int i = tid; i < nv; i += NT) {
                    const int64_t e = (int64_t)o + 4 * i;
                    if (e + 4 <= nnz) {
                        const f4v_t tv = __builtin_nontemporal_load(reinterpret_cast<const f4v_t*>(val + e));
                        const i4v_t tc = __builtin_nontemporal_load(reinterpret_cast<const i4v_t*>(colind + e));
                        sv[4 * i] = static_cast<TV>(tv.x);
                        sv[4 * i + 1] = static_cast<TV>(tv.y);
                        sv[4 * i + 2] = static_cast<TV>(tv.z);
                        sv[4 * i + 3] = static_cast<TV>(tv.w);
                        sc[4 * i] = tc.x;
                        sc[4 * i + 1] = tc.y;
                        sc[4 * i + 2] = tc.z;
                        sc[4 * i + 3] = tc.w;
                    } else {
                        for (int u = 0; u < 4; ++u)
                            if (e + u < nnz) {
                                sv[4 * i + u] = val[e + u];
                                sc[4 * i + u] = colind[e + u];
                            }
                    }
                }
            } else {
                for (int i = tid; i < cnt; i += NT) {
                    sv[i] = __builtin_nontemporal_load(val + e0 + i);
                    sc[i] = ldnt_i(colind + e0 + i);
                }
            }
        }
        __syncthreads();
        const int64_t row = base + tid;
        if (row < n) {
            const int32_t a = rowptr[row], b = rowptr[row + 1];
            double sum = 0.0;
            if (staged)
                for (int32_t e = a - o; e < b - o; ++e) sum += ld_(sv + e) * ld_(x + sc[e]);
            else
                for (int32_t e = a; e < b; ++e) sum += ld_(val + e) * ld_(x + colind[e]);
            y[row] = static_cast<TY>(sum + newton_term(ns, x, row));
        }
        __syncthreads();
    }
}

template <typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(NT) spmv_staged_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const TV* __restrict__ val, const TX* __restrict__ x,
                                                         TY* __restrict__ y, const NewtonStep<TX> ns) {
    spmv_staged_body<TV, TX, TY>(n, nnz, rowptr, colind, val, x, y, blockIdx.x, gridDim.x, ns);
}

template <typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(NT) spmv_staged_kernel_batched(const TX* x0, TY* y0, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    spmv_staged_body<TV, TX, TY>(d.n, d.nnz, d.rowptr, d.colind, static_cast<const TV*>(d.val_op),
                                 batch_ptr(br, sys, d, x0), batch_ptr(br, sys, d, y0), blockIdx.x, gridDim.x);
}

// Flat batched MPK step: workgroup b serves rows [r0, r0 + chunk) of the system of its
// active slot; the row range is handed to the one-system bodies as a sub-matrix (row
// pointers and y offset by r0; column indices and x stay absolute).
template <typename TV, typename TX, typename TY>
__device__ __forceinline__ void flat_range(const BatchReloc& br, const TX* x0, TY* y0, const BatchSys*& dp,
                                           int64_t& r0, int64_t& nr, const TX*& x, TY*& y) {
    const int slot = flat_slot(br);
    const int sys = br.active[slot];
    const BatchSys& d = br.sys[sys];
    dp = &d;
    r0 = (int64_t)(blockIdx.x - br.blk0[slot]) * br.chunk;
    nr = d.n - r0 < br.chunk ? d.n - r0 : br.chunk;
    x = batch_ptr(br, sys, d, x0);
    y = batch_ptr(br, sys, d, y0) + r0;
}

template <int L, typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(NT) spmv_kernel_flat(const TX* x0, TY* y0, const BatchReloc br) {
    const BatchSys* d;
    int64_t r0, nr;
    const TX* x;
    TY* y;
    flat_range<TV, TX, TY>(br, x0, y0, d, r0, nr, x, y);
    spmv_rows<L, TV, TX, TY>(nr, d->rowptr + r0, d->colind, static_cast<const TV*>(d->val_op), x, y, 0, 1);
}

template <typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(NT) spmv_staged_kernel_flat(const TX* x0, TY* y0, const BatchReloc br) {
    const BatchSys* d;
    int64_t r0, nr;
    const TX* x;
    TY* y;
    flat_range<TV, TX, TY>(br, x0, y0, d, r0, nr, x, y);
    spmv_staged_body<TV, TX, TY>(nr, d->nnz, d->rowptr + r0, d->colind, static_cast<const TV*>(d->val_op), x, y, 0,
                                 1);
}

// Batched MPK step: x and y are template basis columns.
template <int L, typename TV, typename TX, typename TY>
__global__ void __launch_bounds__(NT) spmv_kernel_batched(const TX* x0, TY* y0, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    const TX* __restrict__ x = batch_ptr(br, sys, d, x0);
    TY* __restrict__ y = batch_ptr(br, sys, d, y0);
    const TV* __restrict__ val = static_cast<const TV*>(d.val_op);
    const int32_t* __restrict__ rowptr = d.rowptr;
    const int32_t* __restrict__ colind = d.colind;
    const int64_t n = d.n;
    const int tid = threadIdx.x;
    const int sub = tid % L;
    const int64_t rows_per_block = NT / L;
    for (int64_t base = (int64_t)blockIdx.x * rows_per_block; base < n; base += (int64_t)gridDim.x * rows_per_block) {
        const int64_t row = base + tid / L;
        double sum = 0.0;
        if (row < n) {
            const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
            for (int32_t e = e0 + sub; e < e1; e += L) sum += ld_(val + e) * ld_(x + colind[e]);
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (sub == 0 && row < n) y[row] = static_cast<TY>(sum);
    }
}

// r = b - A x (double), stored into R (type T); partials[blockIdx.x] = sum of r^2.
template <int L, typename T>
__device__ __forceinline__ void residual_body(int64_t n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colind, const double* __restrict__ val,
                                              const double* __restrict__ x, const double* __restrict__ b,
                                              T* __restrict__ r, double* __restrict__ partials) {
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    const int sub = tid % L;
    const int64_t rows_per_block = NT / L;
    double acc = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * rows_per_block; base < n; base += (int64_t)gridDim.x * rows_per_block) {
        const int64_t row = base + tid / L;
        double sum = 0.0;
        if (row < n) {
            const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
            for (int32_t e = e0 + sub; e < e1; e += L) sum += val[e] * x[colind[e]];
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (sub == 0 && row < n) {
            const double rv = b[row] - sum;
            r[row] = static_cast<T>(rv);
            acc += rv * rv;
        }
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        partials[blockIdx.x] = s;
    }
}

template <int L, typename T>
__global__ void __launch_bounds__(NT) residual_kernel(int64_t n, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const double* __restrict__ val, const double* __restrict__ x,
                                                      const double* __restrict__ b, T* __restrict__ r,
                                                      double* __restrict__ partials) {
    residual_body<L, T>(n, rowptr, colind, val, x, b, r, partials);
}

template <int L, typename T>
__global__ void __launch_bounds__(NT) residual_kernel_batched(T* r0, double* partials0, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    residual_body<L, T>(d.n, d.rowptr, d.colind, d.val, d.x, d.b, batch_ptr(br, sys, d, r0),
                        batch_ptr(br, sys, d, partials0));
}

// x[row] += dinv[row] * sum_a Q[row, a] y[a]
template <typename T>
__device__ __forceinline__ void update_body(int64_t n, const T* __restrict__ Q, int64_t ldq, int k,
                                            const double* __restrict__ y, const double* __restrict__ dinv,
                                            double* __restrict__ x) {
    extern __shared__ double sy[];
    for (int i = threadIdx.x; i < k; i += NT) sy[i] = y[i];
    __syncthreads();
    for (int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x; row < n; row += (int64_t)gridDim.x * NT) {
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += static_cast<double>(__builtin_nontemporal_load(Q + row + (int64_t)a * ldq)) * sy[a];
        x[row] += dinv ? dinv[row] * s : s;
    }
}

template <typename T>
__global__ void __launch_bounds__(NT) update_kernel(int64_t n, const T* __restrict__ Q, int64_t ldq, int k,
                                                    const double* __restrict__ y, const double* __restrict__ dinv,
                                                    double* __restrict__ x) {
    update_body<T>(n, Q, ldq, k, y, dinv, x);
}

// Batched update: each system adds its own d.kupd basis vectors (none when 0).
template <typename T>
__global__ void __launch_bounds__(NT) update_kernel_batched(const T* Q0, const double* y0, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    if (d.kupd < 1) return;
    update_body<T>(d.n, batch_ptr(br, sys, d, Q0), d.ld, d.kupd, batch_ptr(br, sys, d, y0), d.dinv, d.x);
}

// CSR structure check; touches rowptr[0..n] and colind[0..nnz) only by their own indices.
__global__ void csr_check_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                                 const int32_t* __restrict__ colind, int* bad) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i <= n) {
        const int32_t r = rowptr[i];
        if (r < 0 || r > nnz || (i == 0 && r != 0) || (i == n && r != nnz)) atomicOr(bad, 1);
        if (i < n && rowptr[i + 1] < r) atomicOr(bad, 1);
    }
    for (int64_t e = i; e < nnz; e += (int64_t)gridDim.x * NT) {
        const int32_t c = colind[e];
        if (c < 0 || c >= n) atomicOr(bad, 1);
    }
}

__global__ void diag_inv_kernel(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                const double* __restrict__ val, double* __restrict__ dinv, int* status) {
    const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (row >= n) return;
    double d = 0.0;
    for (int32_t e = rowptr[row]; e < rowptr[row + 1]; ++e)
        if (colind[e] == row) d = val[e];
    if (d == 0.0) atomicCAS(status, 0, -1);  // zero diagonal: Jacobi undefined
    dinv[row] = 1.0 / d;
}

template <typename TV>
__global__ void scale_values_kernel(int64_t nnz, const int32_t* __restrict__ colind, const double* __restrict__ val,
                                    const double* __restrict__ dinv, TV* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= nnz) return;
    const double v = dinv ? val[e] * dinv[colind[e]] : val[e];
    out[e] = static_cast<TV>(v);
}

// y = (double) x, grid-stride.
__global__ void __launch_bounds__(NT) widen_kernel(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        y[i] = static_cast<double>(x[i]);
}

// ---------------------------------------------------------------------------
// Hessenberg bookkeeping (one workgroup).  Column-major (m+1) x m arrays Tin, Tout;
// g (m+1); scratch H ((m+1) x m).
// ---------------------------------------------------------------------------
// Stored coefficient vector c of the replacement below: columns < row of T_in, then of
// T_out, then g.
__device__ __forceinline__ double* coef_vec(const GmSmallArgs& a, int row, int c) {
    const int ld = a.m + 1;
    if (c < row) return a.Tin + (int64_t)c * ld;
    if (c < 2 * row) return a.Tout + (int64_t)(c - row) * ld;
    return a.g;
}

__device__ void replace_row(const GmSmallArgs& a, int row, const double* sub) {
    // Old basis vector `row` = sum_{i <= row} sub[i] * new vector i: rewrite every stored
    // coefficient vector (columns < row of T_in and T_out, and g).  Entry i of vector c
    // becomes col[i] + t sub[i] (i < row) or t sub[row] (i == row), t = col[row]; the
    // entries are spread over the threads, eight loads in flight per thread.
    __shared__ double tv[2 * 256 + 1];
    const int ncol = 2 * row + 1, len = row + 1, total = ncol * len;
    for (int c = threadIdx.x; c < ncol; c += NT) tv[c] = coef_vec(a, row, c)[row];
    __syncthreads();
    for (int b = threadIdx.x; b < total; b += 8 * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = b + u * NT;
            if (idx < total) {
                const int c = idx / len, i = idx - c * len;
                v[u] = coef_vec(a, row, c)[i];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = b + u * NT;
            if (idx < total) {
                const int c = idx / len, i = idx - c * len;
                const double t = tv[c];
                if (t != 0.0) coef_vec(a, row, c)[i] = (i < row) ? v[u] + t * sub[i] : t * sub[row];
            }
        }
    }
    __syncthreads();
}

__device__ void store_block(const GmSmallArgs& a, int kk, const double* coef) {
    // inputs coef[:, 0..s-1] -> T_in[:, kk..kk+s-1]; outputs coef[:, 1..s] -> T_out, or with
    // the Newton recurrence (a_i, b_i) the output A v_i = v_{i+1} + a_i v_i - b_i v_{i-1}
    const int ld = a.m + 1;
    const int rows = kk + a.s + 1;
    for (int idx = threadIdx.x; idx < ld * a.s; idx += NT) {
        const int r = idx % ld, i = idx / ld;
        double out = 0.0;
        if (r < rows) {
            out = coef[r + (int64_t)(i + 1) * ld];
            if (a.newton) {
                out += a.newton[i] * coef[r + (int64_t)i * ld];
                const double bi = a.newton[a.s + i];
                if (bi != 0.0) out -= bi * coef[r + (int64_t)(i - 1) * ld];
            }
        }
        a.Tin[r + (int64_t)(kk + i) * ld] = r < rows ? coef[r + (int64_t)i * ld] : 0.0;
        a.Tout[r + (int64_t)(kk + i) * ld] = out;
    }
    __syncthreads();
}

// H = T_out T_in^{-1} on the leading k columns, Givens least squares, y and residual.
__device__ void lsq(const GmSmallArgs& a, int k) {
    const int ld = a.m + 1;
    double* H = a.H;
    __shared__ double cs[2];
    // H[r, c] = (T_out[r, c] - sum_{q<c} H[r, q] T_in[q, c]) / T_in[c, c]
    for (int r = threadIdx.x; r <= k; r += NT) {
        for (int c = 0; c < k; ++c) {
            double v = a.Tout[r + (int64_t)c * ld];
            for (int q = 0; q < c; ++q) v -= H[r + (int64_t)q * ld] * a.Tin[q + (int64_t)c * ld];
            H[r + (int64_t)c * ld] = v / a.Tin[c + (int64_t)c * ld];
        }
    }
    __syncthreads();
    double* g = a.gw;
    for (int i = threadIdx.x; i <= k; i += NT) g[i] = a.g[i];
    __syncthreads();
    for (int i = 0; i < k; ++i) {
        if (threadIdx.x == 0) {
            const double x = H[i + (int64_t)i * ld], z = H[i + 1 + (int64_t)i * ld];
            const double rad = hypot(x, z);
            cs[0] = rad == 0.0 ? 1.0 : x / rad;
            cs[1] = rad == 0.0 ? 0.0 : z / rad;
        }
        __syncthreads();
        const double c = cs[0], sn = cs[1];
        for (int j = i + threadIdx.x; j < k; j += NT) {
            const double top = H[i + (int64_t)j * ld], bot = H[i + 1 + (int64_t)j * ld];
            H[i + (int64_t)j * ld] = c * top + sn * bot;
            H[i + 1 + (int64_t)j * ld] = -sn * top + c * bot;
        }
        if (threadIdx.x == 0) {
            const double gi = g[i], gj = g[i + 1];
            g[i] = c * gi + sn * gj;
            g[i + 1] = -sn * gi + c * gj;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double v = g[i];
            for (int j = i + 1; j < k; ++j) v -= H[i + (int64_t)j * ld] * a.y[j];
            a.y[i] = v / H[i + (int64_t)i * ld];
        }
        a.res[0] = fabs(g[k]);
    }
    __syncthreads();
}

// lsq with T_in, H and g staged in LDS (rows 0..k, leading dimension k + 1), k <= 62: the
// workgroup loads them, then one wave forms H, applies the rotations and back-substitutes
// without global memory or workgroup barriers.  Lds holds 2 k (k + 1) + (k + 1) + k doubles.
__device__ void lsq_lds(const GmSmallArgs& a, int k, double* lds) {
    const int ld = a.m + 1, lh = k + 1;
    double* Hs = lds;
    double* Ts = lds + (int64_t)lh * k;
    double* gs = Ts + (int64_t)lh * k;
    // T_in into Ts and T_out into Hs (each row of H then overwrites its own T_out row),
    // eight loads of each in flight per thread
    for (int b = threadIdx.x; b < lh * k; b += 8 * NT) {
        double ti[8], to[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = b + u * NT;
            if (idx < lh * k) {
                const int r = idx % lh, c = idx / lh;
                ti[u] = a.Tin[r + (int64_t)c * ld];
                to[u] = a.Tout[r + (int64_t)c * ld];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = b + u * NT;
            if (idx < lh * k) {
                Ts[idx] = ti[u];
                Hs[idx] = to[u];
            }
        }
    }
    for (int i = threadIdx.x; i <= k; i += NT) gs[i] = a.g[i];
    __syncthreads();
    // The rest runs on wave 0 alone (k + 1 <= 63 rows, k <= 62 columns: one lane each), in
    // wave order, with no workgroup barrier per column.
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        // reciprocals of T_in's diagonal, one per lane, off the sequential path below
        double* rinv = gs + lh;  // k doubles past g (the LDS holds 2 k (k + 1) + (k + 1) + k)
        if (lane < k) rinv[lane] = 1.0 / Ts[lane + lane * lh];
        wave_lds_sync();
        // H = T_out T_in^{-1}, right-looking: lane r finishes H[r, c], then removes its term
        // from the later columns of its row.  Each entry H[r, c2] is formed as
        // (T_out[r, c2] - H[r, 0] T_in[0, c2] - ... - H[r, c2 - 1] T_in[c2 - 1, c2]) / T_in[c2, c2],
        // the row-wise recurrence with the division taken as a product by the reciprocal.
        if (lane <= k) {
            for (int c = 0; c < k; ++c) {
                const double h = Hs[lane + c * lh] * rinv[c];
                Hs[lane + c * lh] = h;
#pragma unroll 4
                for (int c2 = c + 1; c2 < k; ++c2) Hs[lane + c2 * lh] -= h * Ts[c + c2 * lh];
            }
        }
        wave_lds_sync();
        // Givens rotations, lane j owning column j; every lane forms the rotation itself from
        // 1 / sqrt(x^2 + z^2) (hardware estimate plus one Newton step: no division or hypot on
        // the sequential path; the Hessenberg entries are far from the FP64 range limits)
        for (int i = 0; i < k; ++i) {
            const double x = Hs[i + i * lh], z = Hs[i + 1 + i * lh];
            const double ss = x * x + z * z;
            double c = 1.0, sn = 0.0;
            if (ss > 0.0) {
                double r = __builtin_amdgcn_rsq(ss);
                r = r * (1.5 - 0.5 * ss * r * r);
                c = x * r;
                sn = z * r;
            }
            if (lane >= i && lane < k) {
                const double top = Hs[i + lane * lh], bot = Hs[i + 1 + lane * lh];
                Hs[i + lane * lh] = c * top + sn * bot;
                Hs[i + 1 + lane * lh] = -sn * top + c * bot;
            }
            if (lane == 0) {
                const double gi = gs[i], gj = gs[i + 1];
                gs[i] = c * gi + sn * gj;
                gs[i + 1] = -sn * gi + c * gj;
            }
            wave_lds_sync();
        }
        // back substitution by columns: lane i holds y[i]; y[i] is final once the columns to
        // its right have been removed from it (the diagonal's reciprocals formed in parallel)
        double yv = lane < k ? gs[lane] : 0.0;
        const double dinv = lane < k ? 1.0 / Hs[lane + lane * lh] : 0.0;
        for (int i = k - 1; i >= 0; --i) {
            const double yi = __shfl(yv, i, 64) * __shfl(dinv, i, 64);
            if (lane == i) yv = yi;
            if (lane < i) yv -= Hs[lane + i * lh] * yi;
        }
        if (lane < k) a.y[lane] = yv;
        if (lane == 0) a.res[0] = fabs(gs[k]);
    }
    __syncthreads();
}

// Doubles of dynamic LDS the staged least squares needs for basis size up to m.
constexpr int lsq_lds_doubles(int m) { return 2 * m * (m + 1) + (m + 1) + m; }
constexpr int kLsqLdsMax = 8000;  // 62.5 KiB

__device__ __forceinline__ void gm_small_body(const GmSmallArgs& a) {
    extern __shared__ double gm_dyn[];
    const int ld = a.m + 1;
    __shared__ double sub[256];
    if (a.op == GM_INIT) {
        for (int idx = threadIdx.x; idx < ld * a.m; idx += NT) {
            a.Tin[idx] = 0.0;
            a.Tout[idx] = 0.0;
        }
        for (int i = threadIdx.x; i < ld; i += NT) a.g[i] = (i == 0) ? a.beta[0] : 0.0;
        return;
    }
    if (a.op == GM_BLOCK) {
        const int kk = a.kk;
        // coefficient rows 0..k0-1 of a two-stage panel come from the projection buffer
        if (a.Cpan) {
            for (int idx = threadIdx.x; idx < a.k0 * (a.s + 1); idx += NT) {
                const int r = idx % a.k0, c = idx / a.k0;
                a.coef[r + (int64_t)c * ld] = a.Cpan[idx];
            }
        } else if (a.two_stage) {
            for (int idx = threadIdx.x; idx < a.k0 * (a.s + 1); idx += NT) {
                const int r = idx % a.k0, c = idx / a.k0;
                a.coef[r + (int64_t)c * ld] = 0.0;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i <= kk; i += NT) sub[i] = a.coef[i];
        __syncthreads();
        replace_row(a, kk, sub);
        store_block(a, kk, a.coef);
        if (a.do_lsq) {
            if (lsq_lds_doubles(a.m) <= kLsqLdsMax)
                lsq_lds(a, kk + a.s, gm_dyn);
            else
                lsq(a, kk + a.s);
            // publish the residual (thread 0 wrote it) and the block's status word to the host
            if (a.host_res && threadIdx.x == 0) {
                volatile double* hr = a.host_res;
                hr[0] = a.res[0];
                reinterpret_cast<volatile int*>(a.host_res + 1)[0] = *a.status_in;
                __threadfence_system();
            }
        }
        return;
    }
    if (a.op == GM_BIGCLOSE) {
        // rows k0..k0+W-1 of every stored vector refer to the pre-processed big panel:
        // t[:k0] += C2 Rh t[k0:], t[k0:] = Rt Rh t[k0:]  (Rt = I without the second pass)
        const int k0 = a.k0, W = a.Wb, kend = a.kend;
        const int ncol = 2 * kend + 1;
        if (lsq_lds_doubles(a.m) <= kLsqLdsMax) {
            // Each thread's segment t[k0:k0+W] in LDS (X[j * ncol + c], (2 kend + 1) W <= the
            // least squares' LDS), loaded eight at a time, then both triangular products in
            // place (row i ascending reads only entries j >= i, which are still inputs); the
            // sums run in the same order as the global-memory form below.
            double* X = gm_dyn;
            // the factors and C2 are read-only here: scalar loads, shared by the wave
            const CD Rh = as_uniform(a.Rh), Rt = as_uniform(a.Rt), C2 = as_uniform(a.C2);
            for (int c = threadIdx.x; c < ncol; c += NT) {
                const double* col = coef_vec(a, kend, c);
                for (int j0 = 0; j0 < W; j0 += 8) {
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (j0 + u < W) t[u] = col[k0 + j0 + u];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (j0 + u < W) X[(j0 + u) * ncol + c] = t[u];
                }
                // y = R x in place, column j of R at a time: entry i < j gains R[i, j] x[j],
                // entry j starts as R[j, j] x[j] (x[j] read first), so each y[i] sums its
                // terms in ascending j, as the row-wise form does
                auto upper_times = [&](CD Rm) {
                    for (int j = 0; j < W; ++j) {
                        const double xj = X[j * ncol + c];
                        const CD Rc = Rm + (int64_t)j * W;
                        for (int i = 0; i < j; ++i) X[i * ncol + c] += Rc[i] * xj;
                        X[j * ncol + c] = 0.0 + Rc[j] * xj;
                    }
                };
                upper_times(Rh);
                double* colw = coef_vec(a, kend, c);
                if (a.C2) {
                    for (int r = 0; r < k0; ++r) {
                        double v = 0.0;
                        for (int j = 0; j < W; ++j) v += C2[r + (int64_t)j * k0] * X[j * ncol + c];
                        colw[r] += v;
                    }
                }
                if (a.Rt) upper_times(Rt);
                for (int i = 0; i < W; ++i) colw[k0 + i] = X[i * ncol + c];
            }
        } else {
            for (int c = threadIdx.x; c < 2 * kend + 1; c += NT) {
                double* col;
                if (c < kend)
                    col = a.Tin + (int64_t)c * ld;
                else if (c < 2 * kend)
                    col = a.Tout + (int64_t)(c - kend) * ld;
                else
                    col = a.g;
                // u = Rh t[k0:] in place (entry i reads only entries j >= i, still inputs), the
                // projection term from u, then Rt u in place the same way
                double* u = col + k0;
                for (int i = 0; i < W; ++i) {
                    double v = 0.0;
                    for (int j = i; j < W; ++j) v += a.Rh[i + j * W] * u[j];
                    u[i] = v;
                }
                if (a.C2) {
                    for (int r = 0; r < k0; ++r) {
                        double v = 0.0;
                        for (int j = 0; j < W; ++j) v += a.C2[r + (int64_t)j * k0] * u[j];
                        col[r] += v;
                    }
                }
                if (a.Rt) {
                    for (int i = 0; i < W; ++i) {
                        double v = 0.0;
                        for (int j = i; j < W; ++j) v += a.Rt[i + j * W] * u[j];
                        u[i] = v;
                    }
                }
            }
        }
        __syncthreads();
        if (lsq_lds_doubles(a.m) <= kLsqLdsMax)
            lsq_lds(a, kend, gm_dyn);
        else
            lsq(a, kend);
        return;
    }
}

__global__ void __launch_bounds__(NT) gm_small_kernel(const GmSmallArgs a) { gm_small_body(a); }

// Newton basis shifts: the Ritz values of the cycle just finished (eigenvalues of the square
// k x k Hessenberg matrix H = T_out T_in^{-1}) in Leja order give the recurrence coefficients
// of s matrix-powers steps, newton[0..s) = a and newton[s..2s) = b.  The rows of H are formed
// in parallel as in the least squares (entries below the subdiagonal, rounding noise of an
// exactly Hessenberg matrix, are set to zero); the QR iteration and the ordering run on one
// thread.  Without convergence the coefficients stay zero (monomial steps).
__global__ void __launch_bounds__(NT) ritz_kernel(const GmSmallArgs a, int k, double* newton) {
    extern __shared__ double rz[];
    const int ld = a.m + 1;
    double* Hs = rz;
    double* wr = Hs + k * k;
    double* wi = wr + k;
    double* cre = wi + k;
    double* cim = cre + k;
    double* ore = cim + k;
    double* oim = ore + 2 * k;
    for (int r = threadIdx.x; r < k; r += NT) {
        for (int c = 0; c < k; ++c) {
            double v = a.Tout[r + (int64_t)c * ld];
            for (int q = 0; q < c; ++q) v -= Hs[r + q * k] * a.Tin[q + (int64_t)c * ld];
            Hs[r + c * k] = v / a.Tin[c + (int64_t)c * ld];
        }
        for (int c = 0; c + 1 < r; ++c) Hs[r + c * k] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* A = newton;
        double* B = newton + a.s;
        for (int j = 0; j < a.s; ++j) A[j] = B[j] = 0.0;
        if (hessenberg_eigenvalues(Hs, k, k, wr, wi)) leja_newton_coefficients(wr, wi, k, a.s, cre, cim, ore, oim, A, B);
    }
}

__global__ void __launch_bounds__(NT) gm_small_kernel_batched(const GmSmallArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    GmSmallArgs a = t;
    a.Tin = batch_ptr(br, sys, d, t.Tin);
    a.Tout = batch_ptr(br, sys, d, t.Tout);
    a.g = batch_ptr(br, sys, d, t.g);
    a.gw = batch_ptr(br, sys, d, t.gw);
    a.H = batch_ptr(br, sys, d, t.H);
    a.y = batch_ptr(br, sys, d, t.y);
    a.res = batch_ptr(br, sys, d, t.res);
    a.beta = batch_ptr(br, sys, d, t.beta);
    a.coef = batch_ptr(br, sys, d, t.coef);
    a.Cpan = batch_ptr(br, sys, d, t.Cpan);
    a.Rh = batch_ptr(br, sys, d, t.Rh);
    a.Rt = batch_ptr(br, sys, d, t.Rt);
    a.C2 = batch_ptr(br, sys, d, t.C2);
    gm_small_body(a);
}

// Kernel choice (measured on the 7-point 192^3 matrix, ~7 entries per row): one row per
// thread over an LDS-staged nonzero range, one workgroup per NT rows (no grid stride, so
// workgroups waiting at the staging barriers leave room for others), is fastest for FP64
// and FP32 values (FP64: 161 us against 183 us for 4 lanes per row under a capped grid);
// rows much longer than 8 entries go to 8 lanes per row.
enum SpmvKind { SPMV_L2, SPMV_L4, SPMV_L8, SPMV_STAGED };

template <typename TV>
SpmvKind spmv_kind(double avg) {
    if (avg > 12.0) return SPMV_L8;
    if (avg <= 8.0) return SPMV_STAGED;
    return avg > 3.0 ? SPMV_L4 : SPMV_L2;
}

int spmv_rows_per_block(SpmvKind k) { return k == SPMV_L8 ? NT / 8 : k == SPMV_L4 ? NT / 4 : k == SPMV_L2 ? NT / 2 : NT; }

template <typename TV, typename TX, typename TY>
hipError_t spmv_dispatch(int64_t n, int64_t nnz, double avg, const int32_t* rp, const int32_t* ci, const TV* v,
                         const TX* x, TY* y, int grid_cap, hipStream_t st, const NewtonStep<TX>& ns = NewtonStep<TX>{}) {
    const SpmvKind k = spmv_kind<TV>(avg);
    const int rpb = spmv_rows_per_block(k);
    const int64_t groups = (n + rpb - 1) / rpb;
    const int64_t cap = k == SPMV_STAGED ? std::max<int64_t>(grid_cap, (int64_t)1 << 30) : grid_cap;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, cap));
    switch (k) {
        case SPMV_L8:
            hipLaunchKernelGGL((spmv_kernel<8, TV, TX, TY>), dim3(grid), dim3(NT), 0, st, n, rp, ci, v, x, y, ns);
            break;
        case SPMV_L4:
            hipLaunchKernelGGL((spmv_kernel<4, TV, TX, TY>), dim3(grid), dim3(NT), 0, st, n, rp, ci, v, x, y, ns);
            break;
        case SPMV_L2:
            hipLaunchKernelGGL((spmv_kernel<2, TV, TX, TY>), dim3(grid), dim3(NT), 0, st, n, rp, ci, v, x, y, ns);
            break;
        case SPMV_STAGED:
            hipLaunchKernelGGL((spmv_staged_kernel<TV, TX, TY>), dim3(grid), dim3(NT), 0, st, n, nnz, rp, ci, v, x, y,
                               ns);
            break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_spmv(const CsrView& A, bool f32, const void* x, void* y, int grid_cap, hipStream_t st,
                       const double* na, const double* nb, const void* z) {
    const double avg = (double)A.nnz / (double)std::max<int64_t>(1, A.n);
    if (f32)
        return spmv_dispatch<float, float, float>(A.n, A.nnz, avg, A.rowptr, A.colind, static_cast<const float*>(A.val_op),
                                                  static_cast<const float*>(x), static_cast<float*>(y), grid_cap, st,
                                                  NewtonStep<float>{na, nb, static_cast<const float*>(z)});
    return spmv_dispatch<double, double, double>(A.n, A.nnz, avg, A.rowptr, A.colind, static_cast<const double*>(A.val_op),
                                                 static_cast<const double*>(x), static_cast<double*>(y), grid_cap, st,
                                                 NewtonStep<double>{na, nb, static_cast<const double*>(z)});
}

hipError_t launch_spmv_panel(const CsrView& A, const double* x, double* y, int grid_cap, hipStream_t st,
                             const double* na, const double* nb, const double* z) {
    const double avg = (double)A.nnz / (double)std::max<int64_t>(1, A.n);
    return spmv_dispatch<float, double, double>(A.n, A.nnz, avg, A.rowptr, A.colind, static_cast<const float*>(A.val_op), x,
                                                y, grid_cap, st, NewtonStep<double>{na, nb, z});
}

hipError_t launch_widen(int64_t n, const float* x, double* y, int grid_cap, hipStream_t st) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, grid_cap));
    hipLaunchKernelGGL(widen_kernel, dim3(grid), dim3(NT), 0, st, n, x, y);
    return hipGetLastError();
}

int residual_grid(int64_t n, int grid_cap) {
    const int64_t groups = (n + NT / 4 - 1) / (NT / 4);
    return (int)std::max<int64_t>(1, std::min<int64_t>(groups, grid_cap));
}

hipError_t launch_residual(const CsrView& A, const double* x, const double* b, bool f32, void* r, double* partials,
                           int grid, hipStream_t st) {
    const double avg = (double)A.nnz / (double)std::max<int64_t>(1, A.n);
    const bool l8 = avg > 12.0;
    if (f32) {
        if (l8)
            hipLaunchKernelGGL((residual_kernel<8, float>), dim3(grid), dim3(NT), 0, st, A.n, A.rowptr, A.colind, A.val,
                               x, b, static_cast<float*>(r), partials);
        else
            hipLaunchKernelGGL((residual_kernel<4, float>), dim3(grid), dim3(NT), 0, st, A.n, A.rowptr, A.colind, A.val,
                               x, b, static_cast<float*>(r), partials);
    } else {
        if (l8)
            hipLaunchKernelGGL((residual_kernel<8, double>), dim3(grid), dim3(NT), 0, st, A.n, A.rowptr, A.colind,
                               A.val, x, b, static_cast<double*>(r), partials);
        else
            hipLaunchKernelGGL((residual_kernel<4, double>), dim3(grid), dim3(NT), 0, st, A.n, A.rowptr, A.colind,
                               A.val, x, b, static_cast<double*>(r), partials);
    }
    return hipGetLastError();
}

hipError_t launch_update(int64_t n, bool f32, const void* Q, int64_t ldq, int k, const double* y, const double* dinv,
                         double* x, hipStream_t st) {
    if (k < 1) return hipSuccess;
    const int grid = (int)((n + NT - 1) / NT);
    const size_t lds = sizeof(double) * (size_t)k;
    if (f32)
        hipLaunchKernelGGL((update_kernel<float>), dim3(grid), dim3(NT), lds, st, n, static_cast<const float*>(Q), ldq,
                           k, y, dinv, x);
    else
        hipLaunchKernelGGL((update_kernel<double>), dim3(grid), dim3(NT), lds, st, n, static_cast<const double*>(Q),
                           ldq, k, y, dinv, x);
    return hipGetLastError();
}

hipError_t launch_csr_check(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind, int* bad,
                            hipStream_t st) {
    const unsigned grid = (unsigned)((n + 1 + NT - 1) / NT);
    hipLaunchKernelGGL(csr_check_kernel, dim3(grid), dim3(NT), 0, st, n, nnz, rowptr, colind, bad);
    return hipGetLastError();
}

hipError_t launch_jacobi_setup(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                               const double* val, double* dinv, int* status, hipStream_t st) {
    hipLaunchKernelGGL(diag_inv_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, rowptr, colind, val,
                       dinv, status);
    (void)nnz;
    return hipGetLastError();
}

hipError_t launch_scale_values(int64_t nnz, const int32_t* colind, const double* val, const double* dinv, bool f32,
                               void* out, hipStream_t st) {
    const unsigned grid = (unsigned)((nnz + NT - 1) / NT);
    if (f32)
        hipLaunchKernelGGL((scale_values_kernel<float>), dim3(grid), dim3(NT), 0, st, nnz, colind, val, dinv,
                           static_cast<float*>(out));
    else
        hipLaunchKernelGGL((scale_values_kernel<double>), dim3(grid), dim3(NT), 0, st, nnz, colind, val, dinv,
                           static_cast<double*>(out));
    return hipGetLastError();
}

hipError_t launch_ritz(const GmSmallArgs& a, int k, double* newton, hipStream_t st) {
    if (k < 1 || k > 64 || k > a.m || !newton) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * ((size_t)k * k + 8 * (size_t)k);
    hipLaunchKernelGGL(ritz_kernel, dim3(1), dim3(NT), lds, st, a, k, newton);
    return hipGetLastError();
}

hipError_t launch_gm_small(const GmSmallArgs& a, hipStream_t st, const BatchReloc* br) {
    if (a.m + 1 > 256 || a.Wb > 64) return hipErrorInvalidValue;
    // the big-panel close stages (2 kend + 1) x Wb values in the least squares' LDS
    if (a.op == GM_BIGCLOSE && (a.kend > a.m || a.k0 < 0 || a.k0 + a.Wb > a.m + 1)) return hipErrorInvalidValue;
    const size_t lds = lsq_lds_doubles(a.m) <= kLsqLdsMax ? sizeof(double) * lsq_lds_doubles(a.m) : 0;
    if (br) {
        if (br->nact < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(gm_small_kernel_batched, dim3(1, br->nact), dim3(NT), lds, st, a, *br);
    } else {
        hipLaunchKernelGGL(gm_small_kernel, dim3(1), dim3(NT), lds, st, a);
    }
    return hipGetLastError();
}

int spmv_flat_unit(bool f32, double avg_nnz) {
    const SpmvKind k = f32 ? spmv_kind<float>(avg_nnz) : spmv_kind<double>(avg_nnz);
    return spmv_rows_per_block(k);
}

template <typename TV, typename TX, typename TY>
void spmv_flat_launch(SpmvKind k, const TX* x, TY* y, hipStream_t st, const BatchReloc& br) {
    const dim3 g(br.nblk);
    switch (k) {
        case SPMV_L8: hipLaunchKernelGGL((spmv_kernel_flat<8, TV, TX, TY>), g, dim3(NT), 0, st, x, y, br); break;
        case SPMV_L4: hipLaunchKernelGGL((spmv_kernel_flat<4, TV, TX, TY>), g, dim3(NT), 0, st, x, y, br); break;
        case SPMV_L2: hipLaunchKernelGGL((spmv_kernel_flat<2, TV, TX, TY>), g, dim3(NT), 0, st, x, y, br); break;
        case SPMV_STAGED:
            hipLaunchKernelGGL((spmv_staged_kernel_flat<TV, TX, TY>), g, dim3(NT), 0, st, x, y, br);
            break;
    }
}

hipError_t launch_spmv_batched(bool f32, double avg_nnz, int64_t max_n, const void* x, void* y, int grid_cap,
                               hipStream_t st, const BatchReloc& br) {
    if (br.nact < 1) return hipErrorInvalidValue;
    const SpmvKind k = f32 ? spmv_kind<float>(avg_nnz) : spmv_kind<double>(avg_nnz);
    if (br.blk0) {
        if (br.nblk < br.nact || br.chunk < 1 || br.chunk % spmv_flat_unit(f32, avg_nnz) != 0)
            return hipErrorInvalidValue;
        if (f32)
            spmv_flat_launch<float, float, float>(k, static_cast<const float*>(x), static_cast<float*>(y), st, br);
        else
            spmv_flat_launch<double, double, double>(k, static_cast<const double*>(x), static_cast<double*>(y), st,
                                                     br);
        return hipGetLastError();
    }
    const int rpb = spmv_rows_per_block(k);
    const int64_t groups = (max_n + rpb - 1) / rpb;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(groups, grid_cap));
    const dim3 g(grid, br.nact);
    if (f32) {
        const float* xx = static_cast<const float*>(x);
        float* yy = static_cast<float*>(y);
        switch (k) {
            case SPMV_L8:
                hipLaunchKernelGGL((spmv_kernel_batched<8, float, float, float>), g, dim3(NT), 0, st, xx, yy, br);
                break;
            case SPMV_L4:
                hipLaunchKernelGGL((spmv_kernel_batched<4, float, float, float>), g, dim3(NT), 0, st, xx, yy, br);
                break;
            case SPMV_L2:
                hipLaunchKernelGGL((spmv_kernel_batched<2, float, float, float>), g, dim3(NT), 0, st, xx, yy, br);
                break;
            case SPMV_STAGED:
                hipLaunchKernelGGL((spmv_staged_kernel_batched<float, float, float>), g, dim3(NT), 0, st, xx, yy, br);
                break;
        }
    } else {
        const double* xx = static_cast<const double*>(x);
        double* yy = static_cast<double*>(y);
        switch (k) {
            case SPMV_L8:
                hipLaunchKernelGGL((spmv_kernel_batched<8, double, double, double>), g, dim3(NT), 0, st, xx, yy, br);
                break;
            case SPMV_L4:
                hipLaunchKernelGGL((spmv_kernel_batched<4, double, double, double>), g, dim3(NT), 0, st, xx, yy, br);
                break;
            case SPMV_L2:
                hipLaunchKernelGGL((spmv_kernel_batched<2, double, double, double>), g, dim3(NT), 0, st, xx, yy, br);
                break;
            case SPMV_STAGED:
                hipLaunchKernelGGL((spmv_staged_kernel_batched<double, double, double>), g, dim3(NT), 0, st, xx, yy,
                                   br);
                break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_residual_batched(bool f32, double avg_nnz, void* r, double* partials, int grid, hipStream_t st,
                                   const BatchReloc& br) {
    if (br.nact < 1 || grid < 1) return hipErrorInvalidValue;
    const bool l8 = avg_nnz > 12.0;
    const dim3 g(grid, br.nact);
    if (f32) {
        if (l8)
            hipLaunchKernelGGL((residual_kernel_batched<8, float>), g, dim3(NT), 0, st, static_cast<float*>(r),
                               partials, br);
        else
            hipLaunchKernelGGL((residual_kernel_batched<4, float>), g, dim3(NT), 0, st, static_cast<float*>(r),
                               partials, br);
    } else {
        if (l8)
            hipLaunchKernelGGL((residual_kernel_batched<8, double>), g, dim3(NT), 0, st, static_cast<double*>(r),
                               partials, br);
        else
            hipLaunchKernelGGL((residual_kernel_batched<4, double>), g, dim3(NT), 0, st, static_cast<double*>(r),
                               partials, br);
    }
    return hipGetLastError();
}

hipError_t launch_update_batched(bool f32, int64_t max_n, const void* Q, int max_k, const double* y, hipStream_t st,
                                 const BatchReloc& br) {
    if (br.nact < 1 || max_k < 1) return hipErrorInvalidValue;
    const dim3 g((unsigned)((max_n + 8 * NT - 1) / (8 * NT)), br.nact);
    const size_t lds = sizeof(double) * (size_t)max_k;
    if (f32)
        hipLaunchKernelGGL((update_kernel_batched<float>), g, dim3(NT), lds, st, static_cast<const float*>(Q), y, br);
    else
        hipLaunchKernelGGL((update_kernel_batched<double>), g, dim3(NT), lds, st, static_cast<const double*>(Q), y,
                           br);
    return hipGetLastError();
}

}  // namespace sko
