// Helpers shared by the streaming kernels: read-only operands that every lane of a
// workgroup reads alike (update coefficients, triangular factors), and the column-group
// update x <- x - Q C of a thread's rows.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sko {

// Read-only uniform operands (update coefficients, triangular factors) are addressed
// through the constant address space: every lane reads the same entry, so the loads go
// through the scalar cache into SGPRs and the FMAs take them as scalar operands.  Through
// LDS each entry would be a full wave-wide read, one per FMA, and the LDS read rate, not
// HBM, would bound the wide passes.  The arrays are written by earlier launches only.
typedef const __attribute__((address_space(4))) double* CD;

// The pointer is the same for the whole workgroup; readfirstlane puts it in SGPRs even
// where it was computed with vector instructions (the batched kernels' relocation).
__device__ __forceinline__ CD as_uniform(const double* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (CD)(((unsigned long long)hi << 32) | lo);
}

// Hides from the compiler that the pointer is the same in every strip, so the entries it
// addresses are loaded again per strip instead of being held in registers for the whole
// sweep (which for wide blocks costs more registers than the kernel can spare).
__device__ __forceinline__ CD per_strip(CD p) {
    unsigned long long v = (unsigned long long)p;
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (CD)(((unsigned long long)hi << 32) | lo);
}

// A uniform integer the compiler must treat as changed per strip, so values derived from
// it (column offsets) are recomputed in the strip instead of being held for the sweep.
__device__ __forceinline__ int64_t per_strip(int64_t v) {
    unsigned lo = (unsigned)(uint64_t)v, hi = (unsigned)((uint64_t)v >> 32);
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int per_strip(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

// A wave-uniform double moved into SGPRs.
__device__ __forceinline__ double uniform_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// R consecutive rows of one column in the storage type, loaded as one access (R == 2:
// pair-aligned).  Kept unconverted until use, so a load issued ahead stays in flight.
template <int R, typename T>
struct RawRows {
    T v[R];
};
template <int R, typename T>
__device__ __forceinline__ RawRows<R, T> load_raw(const T* p) {
    RawRows<R, T> r;
    if constexpr (R == 2) {
        if constexpr (sizeof(T) == 4) {
            const float2 f = *reinterpret_cast<const float2*>(p);
            r.v[0] = f.x;
            r.v[1] = f.y;
        } else {
            const double2 f = *reinterpret_cast<const double2*>(p);
            r.v[0] = f.x;
            r.v[1] = f.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) r.v[i] = __builtin_nontemporal_load(p + i);
    }
    return r;
}

// x[r][c] -= sum_{u<G} Q(r, j + u) C(j + u, c): one group of G update columns.
template <int W, int R, typename T, int G>
__device__ __forceinline__ void update_group(double (&x)[R][W], const RawRows<R, T> (&q)[G], CD C, int j, int pu,
                                             int w) {
#pragma unroll
    for (int c = 0; c < W; ++c) {
        if (c < w) {
            double cu[G];
#pragma unroll
            for (int u = 0; u < G; ++u) cu[u] = C[j + u + c * pu];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double v = x[r][c];
#pragma unroll
                for (int u = 0; u < G; ++u) v -= static_cast<double>(q[u].v[r]) * cu[u];
                x[r][c] = v;
            }
        }
    }
}

template <int R, typename T, int G>
__device__ __forceinline__ void load_group(RawRows<R, T> (&q)[G], const T* Q, int64_t ldq, int j) {
#pragma unroll
    for (int u = 0; u < G; ++u) q[u] = load_raw<R>(Q + (int64_t)(j + u) * ldq);
    // keep the loads here: the scheduler would otherwise sink them to their first use
    __builtin_amdgcn_sched_barrier(0);
}

// x[r][c] -= Q(r, j) C(j, c) for one loaded column j.
template <int W, int R, typename T>
__device__ __forceinline__ void update_col(double (&x)[R][W], const RawRows<R, T>& q, CD C, int j, int pu, int w) {
#pragma unroll
    for (int c = 0; c < W; ++c) {
        if (c < w) {
            const double cj = C[j + c * pu];
#pragma unroll
            for (int r = 0; r < R; ++r) x[r][c] -= static_cast<double>(q.v[r]) * cj;
        }
    }
}

// x[r][c] -= sum_j Q(r, j) C(j, c) over the pu columns of Q for the w <= W live columns of
// x (Q points at this thread's first row; all R rows lie below n).  Columns go in groups of
// G, and the next group's loads are issued before the current group's FMAs (two register
// buffers in turn), so each wave keeps a group of loads in flight while it computes; the
// pu mod G remaining columns follow one by one.  Every column is loaded once: non-temporal
// lines leave the cache early, so a second load of a column would come from HBM again.
// Single rows of 4-byte storage take groups of eight: each load moves half the bytes of a
// double one, so twice as many are kept in flight.  The subtraction order (j ascending per
// output column) is the same as in the generic path and does not depend on G.
template <int W, int R, typename T>
__device__ __forceinline__ void update_rows(double (&x)[R][W], const T* Q, int64_t ldq, int pu, CD C, int w = W) {
    constexpr int G = (sizeof(T) == 4 && R == 1) ? 8 : 4;
    int j = 0;
    if (pu >= G) {
        RawRows<R, T> qa[G], qb[G];
        load_group<R, T, G>(qa, Q, ldq, 0);
        while (true) {
            const bool more = j + 2 * G <= pu;
            if (more) load_group<R, T, G>(qb, Q, ldq, j + G);
            update_group<W, R, T, G>(x, qa, C, j, pu, w);
            j += G;
            if (!more) break;
            const bool more2 = j + 2 * G <= pu;
            if (more2) load_group<R, T, G>(qa, Q, ldq, j + G);
            update_group<W, R, T, G>(x, qb, C, j, pu, w);
            j += G;
            if (!more2) break;
        }
    }
    for (; j < pu; ++j) update_col<W, R, T>(x, load_raw<R>(Q + (int64_t)j * ldq), C, j, pu, w);
}

}  // namespace sko
