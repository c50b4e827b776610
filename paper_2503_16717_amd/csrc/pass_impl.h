// Row-strip streaming pass kernel template for tall-skinny blocks on gfx950.
//
// One workgroup of 256 threads (4 waves of 64) walks strips of 256 consecutive rows
// (grid-stride over strips).  Phase A gives each thread one row: the block row is
// loaded with one coalesced 8-byte (or 4-byte) access per column, updated,
// triangular-solved and written back; the result is staged in LDS column-major.
// Phase B lets every lane own rows lane, lane+64, ... of the strip while each wave
// owns a slice of the reduction's output rows, so every tall operand is read from HBM
// exactly once and the per-lane accumulators stay in registers for the whole sweep.
// The workgroup's partial sums are combined across lanes with shuffles at the end.
#pragma once
#include "sko_internal.h"

namespace sko {
namespace passk {

constexpr int NT = kPassThreads;
constexpr int NWAVE = NT / 64;
constexpr int RPL = NT / 64;  // strip rows per lane in phase B

// Reduction rows per wave: about 40 double accumulators (80 VGPRs), and never fewer
// than needed for the W x W Gram matrix in one launch.
template <int W>
constexpr int maxa() {
    return (40 / W) > (W + NWAVE - 1) / NWAVE ? (40 / W) : (W + NWAVE - 1) / NWAVE;
}

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
__global__ void __launch_bounds__(NT) pass_kernel(const PassArgs a) {
    constexpr int MAXA = maxa<W>();
    constexpr bool HAS_RED = RED != RED_NONE;
    __shared__ double xs[HAS_RED ? W * NT : 1];
    __shared__ uint64_t hs[RED == RED_SKETCH_SPARSE ? NT : 1];
    __shared__ double sR[NTRSM > 0 ? NTRSM * W * W : 1];
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

    // Phase-B ownership: this wave accumulates reduction rows [a_lo, a_lo + MAXA).
    const int a_lo = wave * MAXA;
    double acc[HAS_RED ? MAXA : 1][W];
#pragma unroll
    for (int i = 0; i < (HAS_RED ? MAXA : 1); ++i)
#pragma unroll
        for (int c = 0; c < W; ++c) acc[i][c] = 0.0;

    // Sparse sketch: slot block t and slot j of each owned reduction row (wave-uniform).
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
                for (int c = 0; c < W; ++c) xs[c * NT + tid] = x[c];
            }
        }
        if constexpr (HAS_RED) {
            __syncthreads();
            // ---------------- phase B: lanes over rows, waves over output rows ----------------
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int rr = r * 64 + lane;
                const int64_t row = base + rr;
                double x[W];
#pragma unroll
                for (int c = 0; c < W; ++c) x[c] = xs[c * NT + rr];
                if constexpr (RED == RED_PROJ) {
                    const T* Qp = static_cast<const T*>(a.Qp) + row;
                    double q[MAXA];
#pragma unroll
                    for (int i = 0; i < MAXA; ++i) {
                        const int al = a_lo + i;
                        q[i] = (al < a.red_rows && row < n) ? ldv(Qp + (int64_t)al * a.ldqp) : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < MAXA; ++i)
#pragma unroll
                        for (int c = 0; c < W; ++c) acc[i][c] += q[i] * x[c];
                } else if constexpr (RED == RED_GRAM) {
#pragma unroll
                    for (int i = 0; i < MAXA; ++i) {
                        const int al = a_lo + i;
                        if (al < a.red_rows) {
                            const double xa = xs[(a.red_row0 + al) * NT + rr];
#pragma unroll
                            for (int c = 0; c < W; ++c) acc[i][c] += xa * x[c];
                        }
                    }
                } else if constexpr (RED == RED_SKETCH_SPARSE) {
                    const uint64_t h = hs[rr];
#pragma unroll
                    for (int i = 0; i < MAXA; ++i) {
                        const unsigned b = (unsigned)(h >> sk_shift[i]) & 0xffu;
                        const int slot = (int)(((b >> 1) * (unsigned)sk_B) >> 7);
                        const double coef = (slot == sk_slot[i]) ? ((b & 1u) ? -1.0 : 1.0) : 0.0;
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
            __syncthreads();
        }
    }

    if constexpr (HAS_RED) {
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

}  // namespace passk

// Per-width selectors, one translation unit each (pass_wNN.hip).
passk::KernelPtr select_pass_w1(const PassKey& k);
passk::KernelPtr select_pass_w2(const PassKey& k);
passk::KernelPtr select_pass_w3(const PassKey& k);
passk::KernelPtr select_pass_w4(const PassKey& k);
passk::KernelPtr select_pass_w5(const PassKey& k);
passk::KernelPtr select_pass_w6(const PassKey& k);
passk::KernelPtr select_pass_w7(const PassKey& k);
passk::KernelPtr select_pass_w8(const PassKey& k);
passk::KernelPtr select_pass_w9(const PassKey& k);
passk::KernelPtr select_pass_w10(const PassKey& k);
passk::KernelPtr select_pass_w11(const PassKey& k);
passk::KernelPtr select_pass_w12(const PassKey& k);
passk::KernelPtr select_pass_w13(const PassKey& k);
passk::KernelPtr select_pass_w14(const PassKey& k);
passk::KernelPtr select_pass_w15(const PassKey& k);
passk::KernelPtr select_pass_w16(const PassKey& k);

}  // namespace sko
