// Deterministic reduction of per-workgroup partials, followed by the small dense step
// that consumes the reduced matrix (Householder QR of a sketch, Cholesky of a Gram
// matrix, or the sketch-space BCGS2-HH step), run by the last workgroup to finish.
//
// Partials are summed in a fixed order (workgroup g in strides of 32, then the 32
// part sums in order), so results are bitwise reproducible for a given grid.  All
// small factorisations are in double precision regardless of the storage type.
#include "batch.h"
#include "sko_internal.h"

#include <cmath>

namespace sko {
namespace {

constexpr int RT = 256;          // threads of the reduce kernel
constexpr int EPW = 8;           // reduced elements per workgroup
constexpr int PARTS = RT / EPW;  // partial sums per element

__device__ __forceinline__ double load_coherent(const double* p) {
    unsigned long long bits =
        __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(static_cast<long long>(bits));
}

// put(i, src[i]) for i = tid, tid + RT, ... < count, with eight of each thread's loads in
// flight before the first is used (a plain loop waits for every load before the next).
// COHERENT: the source was written by other workgroups of this launch.
template <bool COHERENT, typename Put>
__device__ __forceinline__ void fill_from(const double* src, int count, Put&& put) {
    int i = threadIdx.x;
    for (; i + 7 * RT < count; i += 8 * RT) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = COHERENT ? load_coherent(src + i + u * RT) : src[i + u * RT];
#pragma unroll
        for (int u = 0; u < 8; ++u) put(i + u * RT, t[u]);
    }
    for (; i < count; i += RT) put(i, COHERENT ? load_coherent(src + i) : src[i]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum NV per-thread values over the workgroup; results land in out[0..NV) (LDS),
// visible to every thread on return.  Order: lanes by xor-butterfly, waves 0..3.
template <int NVMAX>
__device__ void block_sum(const double* vals, int nv, double* red /* LDS 4*NVMAX */, double* out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int v = 0; v < nv; ++v) {
        const double s = wave_sum(vals[v]);
        if (lane == 0) red[wave * NVMAX + v] = s;
    }
    __syncthreads();
    if (tid < nv) {
        double s = 0.0;
        for (int w = 0; w < RT / 64; ++w) s += red[w * NVMAX + tid];
        out[tid] = s;
    }
    __syncthreads();
}

// Householder QR of the k x w matrix A (LDS, column-major, ld k), k <= 256 (one row per
// thread), w <= 16.  On return A's upper triangle holds R (diag >= 0 after the sign
// fix applied to R and, if E != nullptr, to the explicit thin Q formed in E (k x w)).
// Reflector j is v = A[j:, j] (below-diagonal part kept in A) with v_0 in vhead[j].
__device__ void householder_lds(double* A, int k, int w, double* E, double* R, int ldr,
                                int* status, int col0, double* red, double* scal) {
    const int tid = threadIdx.x;
    double* vhead = scal;        // w
    double* beta = scal + 16;    // w
    double* dots = scal + 32;    // w (block_sum results)
    double* sgn = scal + 48;     // w
    double vals[16];
    for (int j = 0; j < w; ++j) {
        // ||A[j+1:k, j]||^2
        vals[0] = (tid > j && tid < k) ? A[tid + j * k] * A[tid + j * k] : 0.0;
        block_sum<16>(vals, 1, red, dots);
        const double ss = dots[0];
        const double x0 = A[j + j * k];
        const double normx = sqrt(x0 * x0 + ss);
        double alpha = 0.0, b = 0.0, v0 = 0.0;
        if (normx != 0.0) {
            alpha = -copysign(normx, x0);
            v0 = x0 - alpha;
            b = 2.0 / (v0 * v0 + ss);
        }
        // d_c = v^T A[j:, c] for the trailing columns
        const int nt = w - j - 1;
        for (int c = 0; c < nt; ++c) {
            const int cc = j + 1 + c;
            double vi = 0.0;
            if (tid == j) vi = v0;
            else if (tid > j && tid < k) vi = A[tid + j * k];
            vals[c] = (tid >= j && tid < k) ? vi * A[tid + cc * k] : 0.0;
        }
        block_sum<16>(vals, nt, red, dots);
        if (tid >= j && tid < k) {
            const double vi = (tid == j) ? v0 : A[tid + j * k];
            for (int c = 0; c < nt; ++c) {
                const int cc = j + 1 + c;
                A[tid + cc * k] -= b * dots[c] * vi;
            }
        }
        __syncthreads();
        if (tid == 0) {
            A[j + j * k] = alpha;
            vhead[j] = v0;
            beta[j] = b;
        }
        __syncthreads();
    }
    // R with non-negative diagonal; breakdown on an exactly zero diagonal.
    if (tid < w) {
        const double d = A[tid + tid * k];
        sgn[tid] = d < 0.0 ? -1.0 : 1.0;
        if (d == 0.0 && status) atomicCAS(status, 0, col0 + tid + 1);
    }
    __syncthreads();
    for (int idx = tid; idx < w * w; idx += RT) {
        const int r = idx % w, c = idx / w;
        R[r + c * ldr] = (r <= c) ? sgn[r] * A[r + c * k] : 0.0;
    }
    if (!E) {
        __syncthreads();
        return;
    }
    // Explicit thin Q: apply H_{w-1} ... H_0 in reverse to [I; 0].
    for (int idx = tid; idx < k * w; idx += RT) {
        const int r = idx % k, c = idx / k;
        E[idx] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = w - 1; j >= 0; --j) {
        const double v0 = vhead[j], b = beta[j];
        for (int c = 0; c < w; ++c) {
            double vi = 0.0;
            if (tid == j) vi = v0;
            else if (tid > j && tid < k) vi = A[tid + j * k];
            vals[c] = (tid >= j && tid < k) ? vi * E[tid + c * k] : 0.0;
        }
        block_sum<16>(vals, w, red, dots);
        if (tid >= j && tid < k) {
            const double vi = (tid == j) ? v0 : A[tid + j * k];
            for (int c = 0; c < w; ++c) E[tid + c * k] -= b * dots[c] * vi;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < k * w; idx += RT) {
        const int c = idx / k;
        E[idx] *= sgn[c];
    }
    __syncthreads();
}

// Orders this wave's LDS writes before its later LDS reads (no other wave involved).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// householder_lds for k <= 64 RPL, run by one wave (rows lane, lane + 64, ... of each
// lane): the column norms and reflector products are per-lane partial sums then shuffle
// reductions, and no step waits for the other waves.  The caller synchronises the
// workgroup afterwards.
template <int RPL>
__device__ void householder_wave(double* A, int k, int w, double* E, double* R, int ldr, int* status, int col0,
                                 double* scal) {
    const int lane = threadIdx.x & 63;
    double* vhead = scal;      // w
    double* beta = scal + 16;  // w
    double* sgn = scal + 48;   // w
    for (int j = 0; j < w; ++j) {
        double aj[RPL], vi[RPL];
        double sl = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            aj[r] = (i > j && i < k) ? A[i + j * k] : 0.0;
            sl += aj[r] * aj[r];
        }
        const double ss = wave_sum(sl);
        const double x0 = A[j + j * k];
        const double normx = sqrt(x0 * x0 + ss);
        double alpha = 0.0, b = 0.0, v0 = 0.0;
        if (normx != 0.0) {
            alpha = -copysign(normx, x0);
            v0 = x0 - alpha;
            b = 2.0 / (v0 * v0 + ss);
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) vi[r] = (lane + 64 * r == j) ? v0 : aj[r];
        for (int c = j + 1; c < w; ++c) {
            double ac[RPL];
            double dl = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                ac[r] = i < k ? A[i + c * k] : 0.0;
                dl += vi[r] * ac[r];
            }
            const double d = wave_sum(dl);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i >= j && i < k) A[i + c * k] = ac[r] - b * d * vi[r];
            }
        }
        wave_sync();
        if (lane == 0) {
            A[j + j * k] = alpha;
            vhead[j] = v0;
            beta[j] = b;
        }
        wave_sync();
    }
    if (lane < w) {
        const double d = A[lane + lane * k];
        sgn[lane] = d < 0.0 ? -1.0 : 1.0;
        if (d == 0.0 && status) atomicCAS(status, 0, col0 + lane + 1);
    }
    wave_sync();
    for (int idx = lane; idx < w * w; idx += 64) {
        const int r = idx % w, c = idx / w;
        R[r + c * ldr] = (r <= c) ? sgn[r] * A[r + c * k] : 0.0;
    }
    if (!E) return;
    // explicit thin Q: H_0 ... H_{w-1} applied in reverse to [I; 0]
    for (int idx = lane; idx < k * w; idx += 64) {
        const int r = idx % k, c = idx / k;
        E[idx] = (r == c) ? 1.0 : 0.0;
    }
    wave_sync();
    for (int j = w - 1; j >= 0; --j) {
        const double v0 = vhead[j], b = beta[j];
        double vi[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + 64 * r;
            vi[r] = (i == j) ? v0 : ((i > j && i < k) ? A[i + j * k] : 0.0);
        }
        for (int c = 0; c < w; ++c) {
            double ec[RPL];
            double dl = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                ec[r] = i < k ? E[i + c * k] : 0.0;
                dl += vi[r] * ec[r];
            }
            const double d = wave_sum(dl);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i >= j && i < k) E[i + c * k] = ec[r] - b * d * vi[r];
            }
        }
        wave_sync();
    }
    for (int idx = lane; idx < k * w; idx += 64) E[idx] *= sgn[idx / k];
    wave_sync();
}

// Householder QR of the k x w matrix A in LDS by one wave (k <= 128) or the workgroup.
__device__ __forceinline__ void householder(double* A, int k, int w, double* E, double* R, int ldr, int* status,
                                            int col0, double* red, double* scal) {
    if (k <= 64) {
        if (threadIdx.x < 64) householder_wave<1>(A, k, w, E, R, ldr, status, col0, scal);
        __syncthreads();
    } else if (k <= 128) {
        if (threadIdx.x < 64) householder_wave<2>(A, k, w, E, R, ldr, status, col0, scal);
        __syncthreads();
    } else {
        householder_lds(A, k, w, E, R, ldr, status, col0, red, scal);
    }
}

// Right-looking upper Cholesky of the w x w matrix G (LDS, column-major), w <= 64, run by
// one wave: each column's pivot, row scaling and trailing update are wave-parallel and
// ordered by wave-level fences only.  Rpk (optional) receives the packed copy described at
// SmallArgs::Rpk.  The caller synchronises the workgroup afterwards.
__device__ void cholesky_wave(double* G, int w, double* R, double* Rpk, int* status, int col0, double* scal) {
    const int lane = threadIdx.x & 63;
    for (int idx = lane; idx < w * w; idx += 64) R[idx] = 0.0;
    for (int j = 0; j < w; ++j) {
        const double d = G[j + j * w];
        if (lane == 0 && (!(d > 0.0) || !isfinite(d)) && status) atomicCAS(status, 0, col0 + j + 1);
        const double r = sqrt(d);
        for (int c = j + lane; c < w; c += 64) {
            const double v = (c == j) ? r : G[j + c * w] / r;
            R[j + c * w] = v;
            scal[8 + c] = v;  // row j of R for the trailing update
            if (Rpk) {
                if (c == j)
                    Rpk[j] = 1.0 / r;
                else
                    Rpk[w + c * (c - 1) / 2 + j] = v;
            }
        }
        wave_sync();
        const int m = w - j - 1;
        for (int idx = lane; idx < m * m; idx += 64) {
            const int a = j + 1 + idx % m, c = j + 1 + idx / m;
            if (a <= c) G[a + c * w] -= scal[8 + a] * scal[8 + c];
        }
        wave_sync();
    }
}

// Rhat = Ra * Rb (upper, w x w) -> rh (global); Rdiag = R * Rhat; Rproj = C1 + C2 * Rhat.
// R and rh were written by this workgroup just before, so they are read coherently.
__device__ void assemble(const SmallArgs& s, double* rh) {
    const int tid = threadIdx.x;
    const int w = s.w;
    for (int idx = tid; idx < w * w; idx += RT) {
        const int a = idx % w, c = idx / w;
        double v = 0.0;
        for (int t = a; t <= c; ++t) v += s.Ra[a + t * w] * s.Rb[t + c * w];
        rh[idx] = (a <= c) ? v : 0.0;
    }
    __syncthreads();
    if (s.Rout) {
        for (int idx = tid; idx < w * w; idx += RT) {
            const int a = idx % w, c = idx / w;
            double v = 0.0;
            if (s.r_identity)
                v = load_coherent(rh + a + c * w);
            else
                for (int t = a; t <= c; ++t) v += load_coherent(s.R + a + t * w) * load_coherent(rh + t + c * w);
            s.Rout[(s.p + a) + c * s.ldr] = (a <= c) ? v : 0.0;
        }
        for (int idx = tid; idx < s.p * w; idx += RT) {
            const int a = idx % s.p, c = idx / s.p;
            double v = s.C1 ? s.C1[a + c * s.p] : 0.0;
            if (s.C2) {
                double t2 = 0.0;
                for (int t = 0; t <= c; ++t) t2 += s.C2[a + t * s.p] * load_coherent(rh + t + c * w);
                v += t2;
            }
            s.Rout[a + c * s.ldr] = v;
        }
    }
    __syncthreads();
}

// Count-Gauss sketch (Section 5.2): Z = theta_g^T Yc (k x w), Yc the reduced kc x w Count
// part in s.out (written by other workgroups, read coherently into T in LDS).  Each entry
// sums over the kc rows in ascending order.
__device__ void count_gauss_product(const SmallArgs& s, double* Z, double* T) {
    const int tid = threadIdx.x;
    const int k = s.k, w = s.w, kc = s.kc;
    fill_from<true>(s.out, kc * w, [&](int i, double v) { T[i] = v; });
    __syncthreads();
    for (int idx = tid; idx < k * w; idx += RT) {
        const int i = idx % k, c = idx / k;
        const double* g = s.theta_g + (int64_t)i * s.ld_g;
        double v = 0.0;
        for (int t = 0; t < kc; ++t) v += g[t] * T[t + c * kc];
        Z[idx] = v;
    }
    __syncthreads();
}

// Sketch-space BCGS2 with Householder (Fig. 8a): y (k x w) against Yacc[:, 0:nacc].
// Ys: LDS copy of Yacc[:, 0:nacc] with leading dimension k + 1 (so lanes reading different
// columns at one row index fall in different banks); the dot products then never wait on
// global memory.
// T: LDS scratch for the Count part of a Count-Gauss sketch (kc x w).
__device__ void sketch_bcgs2(const SmallArgs& s, double* Z, double* E, double* Ys, double* T, double* red,
                             double* scal) {
    const int tid = threadIdx.x;
    const int k = s.k, w = s.w, na = s.nacc;
    const int ldy = k + 1;
    if (s.theta_g)
        count_gauss_product(s, Z, T);
    else
        fill_from<true>(s.out, k * w, [&](int i, double v) { Z[i] = v; });
    fill_from<false>(s.Yacc, k * na, [&](int i, double v) { Ys[i % k + (i / k) * ldy] = v; });
    __syncthreads();
    if (na > 0) {
        for (int pass = 0; pass < 2; ++pass) {
            // r_pass = Yacc^T z ; accumulate into s.r (pass 0 stores, pass 1 adds)
            for (int idx = tid; idx < na * w; idx += RT) {
                const int a = idx % na, c = idx / na;
                double d = 0.0;
                for (int i = 0; i < k; ++i) d += Ys[i + a * ldy] * Z[i + c * k];
                E[idx] = d;
            }
            __syncthreads();
            for (int idx = tid; idx < k * w; idx += RT) {
                const int i = idx % k, c = idx / k;
                double v = Z[idx];
                for (int a = 0; a < na; ++a) v -= Ys[i + a * ldy] * E[a + c * na];
                Z[idx] = v;
            }
            for (int idx = tid; idx < na * w; idx += RT) s.r[idx] = (pass == 0) ? E[idx] : s.r[idx] + E[idx];
            __syncthreads();
        }
    }
    householder(Z, k, w, E, s.R, w, s.status, s.col0, red, scal);
    // append q to the accumulated sketches (replacing the boundary column at nacc)
    for (int idx = tid; idx < k * w; idx += RT) s.Yacc[(int64_t)na * k + idx] = E[idx];
    if (s.Rbar) {
        __syncthreads();
        for (int idx = tid; idx < (na + w) * w; idx += RT) {
            const int a = idx % (na + w), c = idx / (na + w);
            double v;
            if (a < na)
                v = load_coherent(s.r + a + c * na);
            else
                v = load_coherent(s.R + (a - na) + c * w);
            s.Rbar[a + (int64_t)(s.rbar_col0 + c) * s.ldrbar] = v;
        }
    }
    __syncthreads();
}

// BCGS-PIP step (Fig. 7): S = G - P^T P in LDS, R = chol(S) by one wave; r = P and, if
// requested, [r; R] into Rbar.  P (nacc x w) is the reduction just finished (read
// coherently); G was stored by an earlier launch (nacc > 0) or is the reduction itself.
__device__ void pip_step(const SmallArgs& s, double* S, double* P, double* scal) {
    const int tid = threadIdx.x;
    const int w = s.w, na = s.nacc;
    if (na == 0) {
        fill_from<true>(s.out, w * w, [&](int i, double v) { S[i] = v; });
    } else {
        fill_from<true>(s.out, na * w, [&](int i, double v) { P[i] = v; });
        fill_from<false>(s.gram, w * w, [&](int i, double v) { S[i] = v; });
    }
    __syncthreads();
    if (na > 0) {
        for (int idx = tid; idx < w * w; idx += RT) {
            const int a = idx % w, c = idx / w;
            double d = 0.0;
            for (int t = 0; t < na; ++t) d += P[t + a * na] * P[t + c * na];
            S[idx] -= d;
        }
        for (int idx = tid; idx < na * w; idx += RT) s.r[idx] = P[idx];
    }
    __syncthreads();
    if (tid < 64) cholesky_wave(S, w, s.R, nullptr, s.status, s.col0, scal);
    __syncthreads();
    if (s.Rbar) {
        __threadfence();
        for (int idx = tid; idx < (na + w) * w; idx += RT) {
            const int a = idx % (na + w), c = idx / (na + w);
            const double v = a < na ? P[a + c * na] : load_coherent(s.R + (a - na) + c * w);
            s.Rbar[a + (int64_t)(s.rbar_col0 + c) * s.ldrbar] = v;
        }
    }
    __syncthreads();
}

// Sums this workgroup's EPW reduced values over the G partials and stores them (scaled)
// into small.out.  Only threads of wave 0 store.
__device__ __forceinline__ void reduce_partials(const ReduceArgs& a) {
    __shared__ double part[RT];
    const int tid = threadIdx.x;
    const int el = tid % EPW, pt = tid / EPW;
    const int e = blockIdx.x * EPW + el;
    double v = 0.0;
    if (e < a.count) {
        // partial g's of this thread in ascending order; eight loads in flight at a time
        const double* p = a.partials + e;
        int g = pt;
        for (; g + 7 * PARTS < a.G; g += 8 * PARTS) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = p[(int64_t)(g + u * PARTS) * a.stride];
#pragma unroll
            for (int u = 0; u < 8; ++u) v += t[u];
        }
        for (; g < a.G; g += PARTS) v += p[(int64_t)g * a.stride];
    }
    part[tid] = v;
    __syncthreads();
    if (tid < EPW) {
        const int ee = blockIdx.x * EPW + tid;
        if (ee < a.count) {
            double s = 0.0;
            for (int p = 0; p < PARTS; ++p) s += part[p * EPW + tid];
            a.small.out[(ee % a.rows) + (int64_t)(ee / a.rows) * a.ldo] = s * a.scale;
        }
    }
}

// The small dense step on the reduced values in s.out (one workgroup).
__device__ __forceinline__ void small_step(const SmallArgs& s) {
    extern __shared__ double lds[];
    __shared__ double red[4 * 16];
    __shared__ double scal[128];
    const int tid = threadIdx.x;
    if (s.op == OP_STORE) {
        if (!s.theta_g) return;
        double* Z = lds;
        count_gauss_product(s, Z, lds + s.k * s.w);
        for (int idx = tid; idx < s.k * s.w; idx += RT) s.R[idx] = Z[idx];
    } else if (s.op == OP_HH) {
        double* A = lds;
        if (s.theta_g) {
            count_gauss_product(s, A, lds + s.k * s.w);
        } else {
            fill_from<true>(s.out, s.k * s.w, [&](int i, double v) { A[i] = v; });
            __syncthreads();
        }
        householder(A, s.k, s.w, nullptr, s.R, s.w, s.status, s.col0, red, scal);
    } else if (s.op == OP_CHOL) {
        double* G = lds;
        fill_from<true>(s.out, s.w * s.w, [&](int i, double v) { G[i] = v; });
        __syncthreads();
        if (tid < 64) cholesky_wave(G, s.w, s.R, s.Rpk, s.status, s.col0, scal);
        __syncthreads();
        if (s.assemble) {
            __threadfence();
            assemble(s, s.out);  // Rhat overwrites the consumed Gram matrix
        }
    } else if (s.op == OP_PIP) {
        pip_step(s, lds, lds + s.w * s.w, scal);
    } else if (s.op == OP_SKETCH_BCGS2) {
        double* Z = lds;
        double* E = lds + s.k * s.w;
        double* Ys = E + (s.k * s.w > s.nacc * s.w ? s.k * s.w : s.nacc * s.w);
        sketch_bcgs2(s, Z, E, Ys, Ys + (s.k + 1) * s.nacc, red, scal);
    }
}

// Reduction and small step in one launch: the last workgroup to arrive runs the step.
// Only wave 0 stored sums, so it alone makes them visible device-wide before taking its
// ticket (a device-scope release writes back the L2 once per wave that executes it).
__device__ __forceinline__ void reduce_body(const ReduceArgs& a) {
    __shared__ int s_last;
    const int tid = threadIdx.x;
    reduce_partials(a);
    if (tid < 64) __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned prev = atomicAdd(a.counter, 1u);
        s_last = (prev == gridDim.x - 1) ? 1 : 0;
        if (s_last) atomicExch(a.counter, 0u);  // every workgroup has arrived: reset for the next launch
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    small_step(a.small);
}

__global__ void __launch_bounds__(RT) reduce_kernel(const ReduceArgs a) { reduce_body(a); }

// Batched form, in two launches: the reductions of every active system (blockIdx.y), with
// no device-scope fence or ticket per workgroup (thousands of workgroups per launch), then
// one workgroup per system for the small step, ordered after them by the launch boundary.
// The template arguments are moved to the system of blockIdx.y.
__global__ void __launch_bounds__(RT) reduce_kernel_batched(const ReduceArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    ReduceArgs a = t;
    if (t.unit_rows > 0) {
        const int64_t units = (d.n + t.unit_rows - 1) / t.unit_rows;
        if (units < a.G) a.G = (int)units;
    }
    a.partials = batch_ptr(br, sys, d, t.partials);
    a.small.out = batch_ptr(br, sys, d, t.small.out);
    reduce_partials(a);
}

__global__ void __launch_bounds__(RT) small_step_kernel_batched(const SmallArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    SmallArgs m = t;
    m.out = batch_ptr(br, sys, d, t.out);
    m.R = batch_ptr(br, sys, d, t.R);
    m.Rpk = batch_ptr(br, sys, d, t.Rpk);
    m.status = batch_ptr(br, sys, d, t.status);
    m.Yacc = batch_ptr(br, sys, d, t.Yacc);
    m.r = batch_ptr(br, sys, d, t.r);
    m.Rbar = batch_ptr(br, sys, d, t.Rbar);
    m.Ra = batch_ptr(br, sys, d, t.Ra);
    m.Rb = batch_ptr(br, sys, d, t.Rb);
    m.C1 = batch_ptr(br, sys, d, t.C1);
    m.C2 = batch_ptr(br, sys, d, t.C2);
    m.Rout = batch_ptr(br, sys, d, t.Rout);
    m.gram = batch_ptr(br, sys, d, t.gram);
    small_step(m);
}

__global__ void __launch_bounds__(RT) assemble_kernel(const SmallArgs s, double* rh) { assemble(s, rh); }

__global__ void zero_words_kernel(uint32_t* base, int64_t pitch_words, int64_t width_words, int64_t total) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
        const int64_t r = i / width_words;
        base[r * pitch_words + (i - r * width_words)] = 0u;
    }
}

__global__ void matmul_upper_kernel(int w, const double* A, const double* B, double* C) {
    for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) {
        const int a = idx % w, c = idx / w;
        double v = 0.0;
        for (int t = a; t <= c; ++t) v += A[a + t * w] * B[t + c * w];
        C[idx] = (a <= c) ? v : 0.0;
    }
}

}  // namespace

int reduce_grid(int count) { return (count + EPW - 1) / EPW; }

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t stream, const BatchReloc* br) {
    if (a.count <= 0 || a.G <= 0) return hipErrorInvalidValue;
    const SmallArgs& s = a.small;
    size_t lds = 0;
    if (s.theta_g) {
        if (s.op != OP_STORE && s.op != OP_HH && s.op != OP_SKETCH_BCGS2) return hipErrorInvalidValue;
        if (s.kc < s.k || s.kc > RT || s.k < 1 || s.w > 16 || s.ld_g < s.kc) return hipErrorInvalidValue;
        lds = sizeof(double) * (size_t)s.kc * s.w;  // the Count part, staged before the product
        if (s.op == OP_STORE) lds += sizeof(double) * (size_t)s.k * s.w;
    }
    if (s.op == OP_HH) {
        if (s.k > RT || s.w > 16 || s.k < s.w) return hipErrorInvalidValue;
        lds += sizeof(double) * (size_t)s.k * s.w;
    } else if (s.op == OP_CHOL) {
        if (s.w > 64) return hipErrorInvalidValue;
        lds = sizeof(double) * (size_t)s.w * s.w;
    } else if (s.op == OP_PIP) {
        if (s.w > 64 || s.nacc < 0 || (s.nacc > 0 && (!s.gram || !s.r))) return hipErrorInvalidValue;
        lds = sizeof(double) * ((size_t)s.w * s.w + (size_t)s.nacc * s.w);
    } else if (s.op == OP_SKETCH_BCGS2) {
        if (s.k > RT || s.w > 16 || s.k < s.w) return hipErrorInvalidValue;
        const size_t e = (size_t)s.k * s.w > (size_t)s.nacc * s.w ? (size_t)s.k * s.w : (size_t)s.nacc * s.w;
        lds += sizeof(double) * ((size_t)s.k * s.w + e + (size_t)(s.k + 1) * s.nacc);
    }
    // dynamic LDS beyond 64 KiB needs the kernels' limit raised once (gfx950: 160 KiB per CU)
    constexpr size_t kMaxLds = 150 * 1024;
    if (lds > kMaxLds) return hipErrorInvalidValue;
    static bool raised = false;
    if (lds > 60 * 1024 && !raised) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(reduce_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void*>(small_step_kernel_batched),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds) != hipSuccess)
            return hipErrorInvalidValue;
        raised = true;
    }
    const int grid = reduce_grid(a.count);
    if (br) {
        if (br->nact < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(reduce_kernel_batched, dim3(grid, br->nact), dim3(RT), 0, stream, a, *br);
        if (s.op != OP_STORE || s.theta_g) {
            if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
            hipLaunchKernelGGL(small_step_kernel_batched, dim3(1, br->nact), dim3(RT), lds, stream, s, *br);
        }
    } else {
        hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(RT), lds, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const SmallArgs& s, double* rh, hipStream_t stream) {
    if (s.w < 1 || s.w > 64 || !s.Ra || !s.Rb || !s.R || !s.Rout || !rh) return hipErrorInvalidValue;
    hipLaunchKernelGGL(assemble_kernel, dim3(1), dim3(RT), 0, stream, s, rh);
    return hipGetLastError();
}

hipError_t launch_zero_2d(void* p, size_t pitch, size_t width, size_t rows, hipStream_t stream) {
    if (rows == 0 || width == 0) return hipSuccess;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 3) || (pitch & 3) || (width & 3) || width > pitch)
        return hipErrorInvalidValue;
    const int64_t ww = (int64_t)(width / 4), total = ww * (int64_t)rows;
    const int64_t grid = std::min<int64_t>((total + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)grid), dim3(256), 0, stream, static_cast<uint32_t*>(p),
                       (int64_t)(pitch / 4), ww, total);
    return hipGetLastError();
}

hipError_t launch_small_matmul_upper(int w, const double* A, const double* B, double* C, hipStream_t stream) {
    hipLaunchKernelGGL(matmul_upper_kernel, dim3(1), dim3(256), 0, stream, w, A, B, C);
    return hipGetLastError();
}

}  // namespace sko
