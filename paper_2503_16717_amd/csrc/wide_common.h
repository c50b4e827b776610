// Device helpers shared by the wide-block kernels (wide_kernels.hip, wide_fused.hip): the
// row operation's solve and element addressing, and the 4-row operand pieces of the FP64
// MFMA 16 x 16 x 4 tiles.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "sko_internal.h"
#include "uniform.h"

namespace sko {
namespace wide {

template <typename T>
__device__ __forceinline__ double ldv(const T* p) {
    return static_cast<double>(*p);
}
// The row operation's input and output columns stream through it once: non-temporal.
template <typename T>
__device__ __forceinline__ double ldv_nt(const T* p) {
    return static_cast<double>(__builtin_nontemporal_load(p));
}
template <typename T>
__device__ __forceinline__ void stv_nt(T* p, T v) {
    __builtin_nontemporal_store(v, p);
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
    const double* Rpk;   // packed factor: w reciprocal diagonal entries, then column c's c
                         // strictly upper entries at w + c(c-1)/2
    void* X;
    int64_t ldx;
};

// v - sum_{q < c} x[q] Rc[q] for column c of a triangular solve, the factor entries loaded
// in chunks of 8 (one chunk ahead of the FMAs that use it) so that only two chunks occupy
// SGPRs at a time.
template <int WB, int C>
__device__ __forceinline__ double solve_col(const double (&x)[WB], CD Rc, double v) {
    constexpr int NCH = (C + 7) / 8;
    if constexpr (NCH > 0) {
        double r[2][8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < C) r[0][u] = Rc[u];
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            if (k + 1 < NCH) {
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (8 * (k + 1) + u < C) r[(k + 1) & 1][u] = Rc[8 * (k + 1) + u];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (8 * k + u < C) v -= x[8 * k + u] * r[k & 1][u];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return v;
}

template <int WB, int C>
__device__ __forceinline__ void solve_cols(double (&x)[WB], CD Rs, int w, const double* sD) {
    if constexpr (C < WB) {
        if (C < w) {
            x[C] = solve_col<WB, C>(x, Rs + w + C * (C - 1) / 2, x[C]) * sD[C];
            solve_cols<WB, C + 1>(x, Rs, w, sD);
        }
    }
}

// The element a lane handles in a column, given the column's address at the strip's first
// row (the same for the whole workgroup, so it is formed in SGPRs) and the lane's byte
// offset in the strip (one VGPR shared by every column).
template <typename T>
__device__ __forceinline__ T* lane_elem(T* strip_col, uint32_t lane_bytes) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(strip_col) + lane_bytes);
}

constexpr int GT = 256;   // threads (4 waves)
static_assert(16 * (GT / 64) == kGemmUnitRows, "a workgroup index covers 16 rows per wave");

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

// The four pieces (16-column tiles t) of one operand for a group of 16 rows.  In a full
// group every lane loads every piece without a branch: a column past m reads column m - 1
// (lines already requested) and is zeroed after the loads, so all loads of the group are in
// flight together.  A branch per piece would wait for each load in turn.  The group at the
// end of the rows keeps the guarded loads.
template <typename T, int NTL>
__device__ __forceinline__ void load_pieces(const T* base, int64_t ld, int m, int ci, bool vec, bool full,
                                            int64_t row0, int64_t n, double (&v)[NTL][4]) {
    if (full && vec) {
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
            const int c = 16 * t + ci;
            const T* col = base + (int64_t)(c < m ? c : m - 1) * ld;
            if constexpr (sizeof(T) == 8) {
                const double2 p0 = *reinterpret_cast<const double2*>(col + row0);
                const double2 p1 = *reinterpret_cast<const double2*>(col + row0 + 2);
                v[t][0] = p0.x;
                v[t][1] = p0.y;
                v[t][2] = p1.x;
                v[t][3] = p1.y;
            } else {
                const float4 p = *reinterpret_cast<const float4*>(col + row0);
                v[t][0] = p.x;
                v[t][1] = p.y;
                v[t][2] = p.z;
                v[t][3] = p.w;
            }
        }
    } else if (full) {
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
            const int c = 16 * t + ci;
            const T* col = base + (int64_t)(c < m ? c : m - 1) * ld;
#pragma unroll
            for (int u = 0; u < 4; ++u) v[t][u] = ldv(col + row0 + u);
        }
    } else {
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
            const int c = 16 * t + ci;
            load_piece(base + (int64_t)(c < m ? c : 0) * ld, c < m, vec, row0, n, v[t]);
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < NTL; ++t)
        if (16 * t + ci >= m) v[t][0] = v[t][1] = v[t][2] = v[t][3] = 0.0;
}

}  // namespace wide
}  // namespace sko
