// Row-strip streaming pass kernel template for tall-skinny blocks on gfx950.
//
// A workgroup (4 or 8 waves of 64) walks strips of NT consecutive rows (grid-stride over
// strips).  Phase A gives each thread one row: the block row is loaded with one coalesced
// access per column, updated, triangular-solved and written back; the result is staged in
// LDS column-major (padded leading dimension, so column reads across lanes do not collide
// in the LDS banks).  Phase B computes the pass's one reduction from the staged strip:
//
//  * projection Q^T x: FP64 MFMA (v_mfma_f64_16x16x4) tiles of 16 Q columns.  The waves
//    split the strip's 16-row groups; per group every lane loads 4 consecutive rows of one
//    Q column (one 32-byte piece; 16 lanes cover 16 columns, so each 128-byte line is used
//    whole) and the matching 4 rows of x from LDS, and issues 4 MFMAs per tile.  A 16 x 16
//    accumulator is 4 doubles per lane, so one launch covers up to 16 * MT columns of Q;
//    the waves' tiles are summed through LDS once at the end.
//  * Gram x^T x and the sketches Theta^T x: lanes own strip rows, waves own output rows,
//    FP64 FMAs into register accumulators.
//
// Every tall operand is read from HBM once per pass; partial sums stay in registers for the
// whole sweep and are written once per workgroup at the end.
#pragma once
#include "sko_internal.h"

namespace sko {
namespace passk {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Per-(width, reduction) launch configuration.
template <int W, int RED>
struct Cfg {
    // sketch passes use 8 waves (more output rows per launch) while the strip fits LDS
    static constexpr bool SK = RED == RED_SKETCH_SPARSE || RED == RED_SKETCH_DENSE;
    static constexpr int NT = (SK && W <= 12) ? 512 : 256;
    static constexpr int NWAVE = NT / 64;
    static constexpr int LDX = NT + 1;  // padded LDS leading dimension of the strip
    // vector reductions: output rows per wave (accumulators per lane = MAXA * W)
    static constexpr int MAXA_GRAM = (40 / W) > (W + NWAVE - 1) / NWAVE ? (40 / W) : (W + NWAVE - 1) / NWAVE;
    static constexpr int MAXA_SK = (64 / W) < 8 ? ((64 / W) < 1 ? 1 : (64 / W)) : 8;
    static constexpr int MAXA = SK ? MAXA_SK : MAXA_GRAM;
    // MFMA projection: 16-column tiles accumulated by every wave
    static constexpr int MT = 8;
    static constexpr int ROWS = RED == RED_PROJ ? 16 * MT : NWAVE * MAXA;
};

template <typename T>
__device__ __forceinline__ double ldv(const T* p) {
    return static_cast<double>(*p);
}
template <typename T>
__device__ __forceinline__ void stv(T* p, double v) {
    *p = static_cast<T>(v);
}

// SplitMix64 output number c+1 of the stream started at `seed` (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int W, typename T, int RED, bool UPD, int NTRSM, bool WRITE>
__global__ void __launch_bounds__((Cfg<W, RED>::NT)) pass_kernel(const PassArgs a) {
    using C = Cfg<W, RED>;
    constexpr int NT = C::NT;
    constexpr int LDX = C::LDX;
    constexpr int RPL = NT / 64;
    constexpr int MAXA = C::MAXA;
    constexpr int MT = C::MT;
    constexpr bool HAS_RED = RED != RED_NONE;
    constexpr bool VEC_RED = HAS_RED && RED != RED_PROJ;
    __shared__ double xs[HAS_RED ? W * LDX : 1];
    __shared__ uint64_t hs[RED == RED_SKETCH_SPARSE ? NT : 1];
    __shared__ double sR[NTRSM > 0 ? NTRSM * W * W : 1];
    __shared__ double pred[RED == RED_PROJ ? 4 * 64 * C::NWAVE : 1];  // cross-wave tile sums
    extern __shared__ double sC[];  // UPD coefficients, pu * W doubles (dynamic LDS)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t n = a.n;

    if constexpr (NTRSM > 0) {
        for (int i = tid; i < W * W; i += NT) {
            sR[i] = a.R1[i];
            if constexpr (NTRSM > 1) sR[W * W + i] = a.R2[i];
        }
    }
    if constexpr (UPD) {
        for (int i = tid; i < a.pu * W; i += NT) sC[i] = a.Cu[i];
    }
    if constexpr (NTRSM > 0 || UPD) __syncthreads();

    double rinv[NTRSM > 0 ? NTRSM * W : 1];
    if constexpr (NTRSM > 0) {
#pragma unroll
        for (int t = 0; t < NTRSM; ++t)
#pragma unroll
            for (int c = 0; c < W; ++c) rinv[t * W + c] = 1.0 / sR[t * W * W + c * W + c];
    }

    // vector reductions: this wave accumulates output rows [a_lo, a_lo + MAXA)
    const int a_lo = wave * MAXA;
    double acc[VEC_RED ? MAXA : 1][W];
#pragma unroll
    for (int i = 0; i < (VEC_RED ? MAXA : 1); ++i)
#pragma unroll
        for (int c = 0; c < W; ++c) acc[i][c] = 0.0;
    // MFMA projection accumulators: tile m covers Q columns 16m..16m+15 of this launch
    double4_t dacc[RED == RED_PROJ ? MT : 1];
    const int ntiles = (a.red_rows + 15) / 16;
#pragma unroll
    for (int m = 0; m < (RED == RED_PROJ ? MT : 1); ++m) dacc[m] = double4_t{0.0, 0.0, 0.0, 0.0};

    // Sparse sketch: slot block t and slot j of each owned output row (wave-uniform).
    int sk_shift[RED == RED_SKETCH_SPARSE ? MAXA : 1];
    int sk_slot[RED == RED_SKETCH_SPARSE ? MAXA : 1];
    int sk_B = 1;
    if constexpr (RED == RED_SKETCH_SPARSE) {
        sk_B = a.sk_k / a.sk_zeta;
#pragma unroll
        for (int i = 0; i < MAXA; ++i) {
            const int g = a.red_row0 + a_lo + i;
            const int t = g / sk_B;
            const bool live = (a_lo + i) < a.red_rows && t < a.sk_zeta;
            sk_shift[i] = live ? 8 * t : 0;
            sk_slot[i] = live ? g - t * sk_B : -1;  // -1 never matches a slot
        }
    }

    const int64_t nstrips = (n + NT - 1) / NT;
    for (int64_t s = blockIdx.x; s < nstrips; s += gridDim.x) {
        const int64_t base = s * NT;
        // ---------------- phase A: one row per thread ----------------
        {
            const int64_t row = base + tid;
            double x[W];
            if (row < n) {
                const T* Y = static_cast<const T*>(a.Y);
#pragma unroll
                for (int c = 0; c < W; ++c) x[c] = ldv(Y + row + c * a.ldy);
                if constexpr (UPD) {
                    const T* Q = static_cast<const T*>(a.Qu) + row;
                    const int pu = a.pu;
                    int j = 0;
                    for (; j + 4 <= pu; j += 4) {
                        const double q0 = ldv(Q + (int64_t)(j + 0) * a.ldqu);
                        const double q1 = ldv(Q + (int64_t)(j + 1) * a.ldqu);
                        const double q2 = ldv(Q + (int64_t)(j + 2) * a.ldqu);
                        const double q3 = ldv(Q + (int64_t)(j + 3) * a.ldqu);
#pragma unroll
                        for (int c = 0; c < W; ++c) {
                            double v = x[c];
                            v -= q0 * sC[j + 0 + c * pu];
                            v -= q1 * sC[j + 1 + c * pu];
                            v -= q2 * sC[j + 2 + c * pu];
                            v -= q3 * sC[j + 3 + c * pu];
                            x[c] = v;
                        }
                    }
                    for (; j < pu; ++j) {
                        const double q = ldv(Q + (int64_t)j * a.ldqu);
#pragma unroll
                        for (int c = 0; c < W; ++c) x[c] -= q * sC[j + c * pu];
                    }
                }
#pragma unroll
                for (int t = 0; t < NTRSM; ++t) {
                    const double* R = sR + t * W * W;
#pragma unroll
                    for (int c = 0; c < W; ++c) {
                        double v = x[c];
#pragma unroll
                        for (int q = 0; q < c; ++q) v -= x[q] * R[q + c * W];
                        x[c] = v * rinv[t * W + c];
                    }
                }
                if constexpr (WRITE) {
                    T* X = static_cast<T*>(a.X);
#pragma unroll
                    for (int c = 0; c < W; ++c) stv(X + row + c * a.ldx, x[c]);
                }
                if constexpr (RED == RED_SKETCH_SPARSE) hs[tid] = splitmix64(a.sk_seed, (uint64_t)row);
            } else {
#pragma unroll
                for (int c = 0; c < W; ++c) x[c] = 0.0;
                if constexpr (RED == RED_SKETCH_SPARSE) hs[tid] = 0;
            }
            if constexpr (HAS_RED) {
#pragma unroll
                for (int c = 0; c < W; ++c) xs[c * LDX + tid] = x[c];
            }
        }
        if constexpr (HAS_RED) {
            __syncthreads();
            if constexpr (RED == RED_PROJ) {
                // ---------------- phase B, MFMA projection ----------------
                const int g = lane >> 4, ci = lane & 15;
                const T* Qp = static_cast<const T*>(a.Qp);
                // 32-byte row pieces can be read as two 16-byte vectors when aligned
                const bool vec = sizeof(T) == 8 && (a.ldqp % 4) == 0 && ((uintptr_t)Qp % 32) == 0;
                for (int gam = wave; gam < NT / 16; gam += C::NWAVE) {
                    const int r0 = gam * 16 + 4 * g;  // strip-local rows r0..r0+3 for this lane
                    const bool full = base + r0 + 3 < n;
                    double bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) bv[u] = (ci < W) ? xs[ci * LDX + r0 + u] : 0.0;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (m < ntiles) {
                            const int col = 16 * m + ci;
                            double av[4] = {0.0, 0.0, 0.0, 0.0};
                            if (col < a.red_rows) {
                                const T* q = Qp + (int64_t)col * a.ldqp + base + r0;
                                if (vec && full) {
                                    const double2 v0 = *reinterpret_cast<const double2*>(q);
                                    const double2 v1 = *reinterpret_cast<const double2*>(q + 2);
                                    av[0] = v0.x;
                                    av[1] = v0.y;
                                    av[2] = v1.x;
                                    av[3] = v1.y;
                                } else {
#pragma unroll
                                    for (int u = 0; u < 4; ++u) av[u] = (base + r0 + u < n) ? ldv(q + u) : 0.0;
                                }
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                dacc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], dacc[m], 0, 0, 0);
                        }
                    }
                }
            } else {
                // ---------------- phase B, lanes over rows, waves over output rows ----------------
#pragma unroll 2
                for (int r = 0; r < RPL; ++r) {
                    const int rr = r * 64 + lane;
                    const int64_t row = base + rr;
                    double x[W];
#pragma unroll
                    for (int c = 0; c < W; ++c) x[c] = xs[c * LDX + rr];
                    if constexpr (RED == RED_GRAM) {
#pragma unroll
                        for (int i = 0; i < MAXA; ++i) {
                            const int al = a_lo + i;
                            if (al < a.red_rows) {
                                const double xa = xs[(a.red_row0 + al) * LDX + rr];
#pragma unroll
                                for (int c = 0; c < W; ++c) acc[i][c] += xa * x[c];
                            }
                        }
                    } else if constexpr (RED == RED_SKETCH_SPARSE) {
                        // decode the row's slot and sign once per hash block this wave covers
                        // (sk_shift is wave-uniform and non-decreasing in i)
                        const uint64_t h = hs[rr];
                        int slot = -2;
                        double sgn = 0.0;
#pragma unroll
                        for (int i = 0; i < MAXA; ++i) {
                            if (i == 0 || sk_shift[i] != sk_shift[i - 1]) {
                                const unsigned b = (unsigned)(h >> sk_shift[i]) & 0xffu;
                                slot = (int)(((b >> 1) * (unsigned)sk_B) >> 7);
                                sgn = (b & 1u) ? -1.0 : 1.0;
                            }
                            const double coef = (slot == sk_slot[i]) ? sgn : 0.0;
#pragma unroll
                            for (int c = 0; c < W; ++c) acc[i][c] = fma(coef, x[c], acc[i][c]);
                        }
                    } else if constexpr (RED == RED_SKETCH_DENSE) {
                        const double* th = a.theta + row;
                        double tv[MAXA];
#pragma unroll
                        for (int i = 0; i < MAXA; ++i) {
                            const int al = a_lo + i;
                            tv[i] = (al < a.red_rows && row < n) ? th[(int64_t)al * a.ldtheta] : 0.0;
                        }
#pragma unroll
                        for (int i = 0; i < MAXA; ++i)
#pragma unroll
                            for (int c = 0; c < W; ++c) acc[i][c] += tv[i] * x[c];
                    }
                }
            }
            __syncthreads();
        }
    }

    if constexpr (RED == RED_PROJ) {
        // v_mfma_f64_16x16x4 output layout (measured on gfx950): D[i][j] of a tile sits in
        // lane j + 16 * (i % 4), element i / 4.  The waves' tiles are summed through LDS in
        // wave order.
        double* out = a.partials + (int64_t)blockIdx.x * a.part_stride;
        const int j = lane & 15;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (m >= ntiles) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) pred[(wave * 4 + r) * 64 + lane] = dacc[m][r];
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double v = 0.0;
                    for (int w2 = 0; w2 < C::NWAVE; ++w2) v += pred[(w2 * 4 + r) * 64 + lane];
                    const int col = 16 * m + (lane >> 4) + 4 * r;
                    if (col < a.red_rows && j < W) out[(a.red_row0 + col) + (int64_t)j * a.part_rows_total] = v;
                }
            }
            __syncthreads();
        }
    } else if constexpr (HAS_RED) {
        double* out = a.partials + (int64_t)blockIdx.x * a.part_stride;
#pragma unroll
        for (int i = 0; i < MAXA; ++i) {
            const int al = a_lo + i;
#pragma unroll
            for (int c = 0; c < W; ++c) {
                const double v = wave_sum(acc[i][c]);
                if (lane == 0 && al < a.red_rows)
                    out[(a.red_row0 + al) + (int64_t)c * a.part_rows_total] = v;
            }
        }
    }
}

using KernelPtr = void (*)(const PassArgs);

// The pass variants the orchestration launches: (reduction, update, solves, write).
template <int W, typename T>
KernelPtr select_w(const PassKey& k) {
    const int r = k.red;
    const bool u = k.upd, wr = k.write;
    const int t = k.ntrsm;
    if (!u && t == 0 && !wr) {
        if (r == RED_PROJ) return &pass_kernel<W, T, RED_PROJ, false, 0, false>;
        if (r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, false, 0, false>;
        if (r == RED_SKETCH_SPARSE) return &pass_kernel<W, T, RED_SKETCH_SPARSE, false, 0, false>;
        if (r == RED_SKETCH_DENSE) return &pass_kernel<W, T, RED_SKETCH_DENSE, false, 0, false>;
    }
    if (u && t == 0 && wr) {
        if (r == RED_NONE) return &pass_kernel<W, T, RED_NONE, true, 0, true>;
        if (r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, true, 0, true>;
        if (r == RED_SKETCH_SPARSE) return &pass_kernel<W, T, RED_SKETCH_SPARSE, true, 0, true>;
        if (r == RED_SKETCH_DENSE) return &pass_kernel<W, T, RED_SKETCH_DENSE, true, 0, true>;
    }
    if (!u && t == 1 && !wr && r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, false, 1, false>;
    if (!u && t == 2 && wr) {
        if (r == RED_PROJ) return &pass_kernel<W, T, RED_PROJ, false, 2, true>;
        if (r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, false, 2, true>;
    }
    if (r == RED_NONE && t == 1 && wr) {
        if (!u) return &pass_kernel<W, T, RED_NONE, false, 1, true>;
        return &pass_kernel<W, T, RED_NONE, true, 1, true>;
    }
    return nullptr;
}

template <int W>
int rows_w(int red) {
    switch (red) {
        case RED_PROJ: return Cfg<W, RED_PROJ>::ROWS;
        case RED_GRAM: return Cfg<W, RED_GRAM>::ROWS;
        case RED_SKETCH_SPARSE: return Cfg<W, RED_SKETCH_SPARSE>::ROWS;
        case RED_SKETCH_DENSE: return Cfg<W, RED_SKETCH_DENSE>::ROWS;
        default: return 0;
    }
}

template <int W>
int threads_w(int red) {
    switch (red) {
        case RED_SKETCH_SPARSE: return Cfg<W, RED_SKETCH_SPARSE>::NT;
        case RED_SKETCH_DENSE: return Cfg<W, RED_SKETCH_DENSE>::NT;
        case RED_PROJ: return Cfg<W, RED_PROJ>::NT;
        case RED_GRAM: return Cfg<W, RED_GRAM>::NT;
        default: return Cfg<W, RED_NONE>::NT;
    }
}

}  // namespace passk

// Per-width selectors, one translation unit each (pass_wNN.hip).
struct PassSel {
    passk::KernelPtr fn;
    int threads;  // workgroup size (= strip rows)
    int rows;     // reduction rows one launch can produce
};
PassSel select_pass_w1(const PassKey& k);
PassSel select_pass_w2(const PassKey& k);
PassSel select_pass_w3(const PassKey& k);
PassSel select_pass_w4(const PassKey& k);
PassSel select_pass_w5(const PassKey& k);
PassSel select_pass_w6(const PassKey& k);
PassSel select_pass_w7(const PassKey& k);
PassSel select_pass_w8(const PassKey& k);
PassSel select_pass_w9(const PassKey& k);
PassSel select_pass_w10(const PassKey& k);
PassSel select_pass_w11(const PassKey& k);
PassSel select_pass_w12(const PassKey& k);
PassSel select_pass_w13(const PassKey& k);
PassSel select_pass_w14(const PassKey& k);
PassSel select_pass_w15(const PassKey& k);
PassSel select_pass_w16(const PassKey& k);

}  // namespace sko
