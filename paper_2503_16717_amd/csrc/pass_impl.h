// Row-strip streaming pass kernel template for tall-skinny blocks on gfx950.
//
// A workgroup (4 waves of 64) walks strips of consecutive rows (grid-stride over strips).
// Phase A gives each thread RPT consecutive rows (two for float storage, read and written
// as one 8-byte access per column, so a wave moves 512 bytes per load as it does for
// double storage; not for wide float blocks with triangular solves, which would not fit the
// registers): the rows are loaded with coalesced accesses, updated, triangular-solved
// and written back; the result is staged in LDS column-major (padded leading dimension,
// so column reads across lanes do not collide in the LDS banks).  Phase B computes the pass's one reduction from the staged strip:
//
//  * projection Q^T x and the sketches Theta^T x: FP64 MFMA (v_mfma_f64_16x16x4) tiles of
//    16 output rows.  The waves split the strip's 16-row groups; per group every lane
//    supplies 4 consecutive rows of one output row's operand (Q and a dense Theta are read
//    as one 32-byte piece per lane, so 16 lanes use each 128-byte line whole; the
//    sparse-sign Theta is decoded from the rows' hashes) and the matching 4 rows of x from
//    LDS, and issues 4 MFMAs per tile.  A 16 x 16 accumulator is 4 doubles per lane, so one
//    launch covers up to 16 * MT output rows; the waves' tiles are summed through LDS once
//    at the end.
//  * Gram x^T x: lanes own strip rows, waves own output rows, FP64 FMAs into register
//    accumulators.
//
// Every tall operand is read from HBM once per pass; partial sums stay in registers for the
// whole sweep and are written once per workgroup at the end.
#pragma once
#include <type_traits>
#include "batch.h"
#include "sko_internal.h"
#include "uniform.h"

namespace sko {
namespace passk {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Per-(width, reduction) launch configuration.
template <int W, int RED>
struct Cfg {
    static constexpr bool SK = RED == RED_SKETCH_SPARSE || RED == RED_SKETCH_DENSE;
    // reductions on MFMA tiles: the projection and both sketches
    static constexpr bool MF = RED == RED_PROJ || SK;
    static constexpr int NT = 256;
    static constexpr int NWAVE = NT / 64;
    // Gram: output rows per wave (accumulators per lane = MAXA * W), spread over all waves
    static constexpr int MAXA = (W + NWAVE - 1) / NWAVE;
    // MFMA tiles of 16 output rows held by every wave (a dense sketch up to 64 rows in one
    // launch; projections up to 128 previous columns); a sparse sketch covers 16 MT rows too,
    // on row masks (MT = 4: one sketch row per lane, 8: two).  Fewer tiles are instantiated
    // for launches that need fewer (more resident waves).
    static constexpr int MT = RED == RED_SKETCH_DENSE ? 4 : 8;
    static constexpr int ROWS = MF ? 16 * MT : NWAVE * MAXA;
};

// The tall operands stream through a pass once: loads and stores are non-temporal.
template <typename T>
__device__ __forceinline__ double ldv(const T* p) {
    return static_cast<double>(__builtin_nontemporal_load(p));
}
template <typename T>
__device__ __forceinline__ void stv(T* p, double v) {
    __builtin_nontemporal_store(static_cast<T>(v), p);
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

// Loads rows row0..row0+3 of one operand column (Q or a dense Theta) into av; rows at or
// beyond n read as zero.  `vec`: the column pointer is 32-byte aligned for every group.
template <typename TA>
__device__ __forceinline__ void load_col4(const TA* q, bool vec, bool full, int64_t row0, int64_t n,
                                          double av[4]) {
    if (vec && full) {
        if constexpr (sizeof(TA) == 8) {
            const double2 v0 = *reinterpret_cast<const double2*>(q);
            const double2 v1 = *reinterpret_cast<const double2*>(q + 2);
            av[0] = v0.x;
            av[1] = v0.y;
            av[2] = v1.x;
            av[3] = v1.y;
        } else {
            const float4 v = *reinterpret_cast<const float4*>(q);
            av[0] = v.x;
            av[1] = v.y;
            av[2] = v.z;
            av[3] = v.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = (row0 + u < n) ? ldv(q + u) : 0.0;
    }
}

// Rows row0..row0+R-1 of one column (zero at or beyond n); `vec`: R == 2 and the column
// start and leading dimension allow 2-element vector accesses.
template <int R, typename T>
__device__ __forceinline__ void load_rows(const T* col, bool vec, int64_t row0, int64_t n, double v[R]) {
    if constexpr (R == 2) {
        if (vec && row0 + 1 < n) {
            if constexpr (sizeof(T) == 8) {
                const double2 p = *reinterpret_cast<const double2*>(col + row0);
                v[0] = p.x;
                v[1] = p.y;
            } else {
                const float2 p = *reinterpret_cast<const float2*>(col + row0);
                v[0] = p.x;
                v[1] = p.y;
            }
            return;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (row0 + r < n) ? ldv(col + row0 + r) : 0.0;
}

template <int R, typename T>
__device__ __forceinline__ void store_rows(T* col, bool vec, int64_t row0, int64_t n, const double v[R]) {
    if constexpr (R == 2) {
        if (vec && row0 + 1 < n) {
            if constexpr (sizeof(T) == 8) {
                *reinterpret_cast<double2*>(col + row0) = double2{v[0], v[1]};
            } else {
                *reinterpret_cast<float2*>(col + row0) = float2{static_cast<float>(v[0]), static_cast<float>(v[1])};
            }
            return;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (row0 + r < n) stv(col + row0 + r, v[r]);
}

template <typename T>
__device__ __forceinline__ bool pair_aligned(const void* p, int64_t ld) {
    return p == nullptr || (((uintptr_t)p % (2 * sizeof(T))) == 0 && (ld % 2) == 0);
}

// Element types of a pass: TY the input block Y, TQ the basis operand (Qu of the update,
// Qp of the projection), TX the written block X.  Plain passes use one storage type for
// all three; the mixed-precision GMRES panel reads an FP64 panel against the FP32 basis.
template <typename TY_, typename TQ_, typename TX_>
struct Tys {
    using TY = TY_;
    using TQ = TQ_;
    using TX = TX_;
};

// One pass over the rows of `a` by workgroup wg of nwg.
template <int W, typename TS, int RED, bool UPD, int NTRSM, bool WRITE, int MTX>
__device__ __forceinline__ void pass_body(const PassArgs& a, const int wg, const int nwg) {
    using TY = typename TS::TY;
    using TQ = typename TS::TQ;
    using TX = typename TS::TX;
    using C = Cfg<W, RED>;
    constexpr int NT = C::NT;
    constexpr bool F32 = sizeof(TY) == 4 && sizeof(TQ) == 4 && sizeof(TX) == 4;
    // rows per thread in phase A: two for float storage (8-byte accesses), except for wide
    // blocks with triangular solves or updates, whose two rows would not fit the registers
    constexpr int RPT = (F32 && (W <= 8 || (NTRSM == 0 && !UPD))) ? 2 : 1;
    constexpr int STRIP = NT * RPT;
    constexpr int LDX = STRIP + 1;  // padded LDS leading dimension of the strip
    constexpr int RPL = STRIP / 64;
    constexpr int MAXA = C::MAXA;
    constexpr int MT = MTX > 0 ? MTX : C::MT;  // MFMA tiles held (fewer: more waves per SIMD)
    constexpr bool MF = C::MF;
    constexpr bool WAVE_LOCAL = C::SK;  // sketch tiles reduce each wave's own rows
    constexpr bool HAS_RED = RED != RED_NONE;
    constexpr bool GRAM = RED == RED_GRAM;
    // the strip in LDS, in the storage type: float storage reduces the rounded values it
    // stores (and halves the LDS)
    using XS = typename std::conditional<sizeof(typename std::conditional<WRITE, TX, TY>::type) == 4, float,
                                         double>::type;
    __shared__ XS xs[HAS_RED ? W * LDX : 1];
    __shared__ uint64_t hs[RED == RED_SKETCH_SPARSE ? STRIP : 1];
    __shared__ double pred[MF ? 4 * 64 * C::NWAVE : 1];  // cross-wave tile sums

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t n = a.n;

    // triangular factors (W x W, column-major) and update coefficients (pu x W)
    const CD gR0[2] = {as_uniform(a.R1), as_uniform(a.R2)};
    const CD gC0 = as_uniform(a.Cu);
    double rinv[NTRSM > 0 ? NTRSM * W : 1];
    if constexpr (NTRSM > 0) {
#pragma unroll
        for (int t = 0; t < NTRSM; ++t)
#pragma unroll
            for (int c = 0; c < W; ++c) rinv[t * W + c] = uniform_d(1.0 / gR0[t][c * W + c]);
    }

    // Gram: this wave accumulates output rows [a_lo, a_lo + MAXA)
    const int a_lo = wave * MAXA;
    double acc[GRAM ? MAXA : 1][W];
#pragma unroll
    for (int i = 0; i < (GRAM ? MAXA : 1); ++i)
#pragma unroll
        for (int c = 0; c < W; ++c) acc[i][c] = 0.0;
    // MFMA accumulators: tile m covers output rows 16m..16m+15 of this launch
    // The projection and dense sketch of blocks up to 12 columns run on v_mfma_f64_4x4x4 (four independent 4 x 4 x 4 blocks per instruction, the same FP64
    // rate as 16 x 16 x 4): a block covers 4 output rows x 4 columns of x, so narrow blocks
    // do not pay for 16 padded columns (three instructions of a quarter of the time instead
    // of one 16 x 16 x 4 for 11 columns).  Instruction (m, cb) holds the output rows
    // 16m..16m+15 (block b: rows 16m + 4b..+3) and the columns 4cb..4cb+3.  The A operand
    // uses the lane mapping of the 16 x 16 x 4 tile (lane l: output row 16m + l % 16, data
    // row l / 16), so the same pieces feed both forms.
    // sparse-sign sketches on row masks (no MFMA): lane l accumulates the launch's sketch rows
    // l and, for launches of up to 128 rows, l + 64
    constexpr bool SPM = RED == RED_SKETCH_SPARSE;
    constexpr int SPR = MT / 4;
    constexpr bool B4 = MF && !SPM && W <= 12;
    constexpr int CB = (W + 3) / 4;
    double4_t dacc[(MF && !SPM && !B4) ? MT : 1];
    double acc4[B4 ? MT * CB : 1];
#pragma unroll
    for (int i = 0; i < (B4 ? MT * CB : 1); ++i) acc4[i] = 0.0;
    const int ntiles = (a.red_rows + 15) / 16;
#pragma unroll
    for (int m = 0; m < (MF ? MT : 1); ++m) dacc[m] = double4_t{0.0, 0.0, 0.0, 0.0};

    // Sparse sketch on row masks (SPM): lane l accumulates sketch row g = red_row0 + l (and
    // g + 64), which is slot j of hash byte spm_t (none: spm_t = -1); byte b selects slot
    // floor((b >> 1) B / 128) of its B = k / zeta and carries the sign in bit 0.  Per 64 staged rows the wave forms,
    // for every byte t, the ballots of the bits of each row's slot and of its sign; a lane
    // keeps the rows whose slot bits all equal its own (spm_jn[i]: all ones where bit i of
    // spm_j is 0, so that ballot is inverted) for its own byte, then adds those rows into its
    // W sums in ascending row order.  Only the rows with a nonzero in the lane's sketch row
    // are touched: zeta W products per row instead of k W on MFMA blocks.
    constexpr int SPM_BITS = 7;  // slots per byte up to 128 (k <= 128)
    int spm_t[SPM ? SPR : 1], spm_nbits = 0;
    unsigned spm_jn[SPM ? SPR : 1][SPM ? SPM_BITS : 1];
    double sacc[SPM ? SPR : 1][SPM ? W : 1];
#pragma unroll
    for (int q = 0; q < (SPM ? SPR : 1); ++q)
#pragma unroll
        for (int c = 0; c < (SPM ? W : 1); ++c) sacc[q][c] = 0.0;
    if constexpr (SPM) {
        const int B = a.sk_k / a.sk_zeta;
        while ((1 << spm_nbits) < B) ++spm_nbits;
#pragma unroll
        for (int q = 0; q < SPR; ++q) {
            const int g = a.red_row0 + lane + 64 * q;
            const int t = g / B, j = g - t * B;
            spm_t[q] = (lane + 64 * q < a.red_rows && t < a.sk_zeta) ? t : -1;
#pragma unroll
            for (int i = 0; i < SPM_BITS; ++i) spm_jn[q][i] = ((j >> i) & 1) ? 0u : ~0u;
        }
    }

    // 2-row vector accesses need every tall operand's column starts 2-element aligned
    const bool vec = RPT == 2 && pair_aligned<TY>(a.Y, a.ldy) && (!UPD || pair_aligned<TQ>(a.Qu, a.ldqu)) &&
                     (!WRITE || pair_aligned<TX>(a.X, a.ldx));
    const int64_t nstrips = (n + STRIP - 1) / STRIP;
    for (int64_t s = wg; s < nstrips; s += nwg) {
        const int64_t base = s * STRIP;
        // wide blocks load the factor and coefficient entries again per strip (w(w-1)/2 per
        // factor would not fit the SGPRs for the whole sweep); narrow blocks may hold them
        CD gR[2] = {gR0[0], gR0[1]};
        CD gC = gC0;
        if constexpr (W >= 10) {
            gR[0] = per_strip(gR[0]);
            gR[1] = per_strip(gR[1]);
            gC = per_strip(gC);
        }
        // ---------------- phase A: RPT consecutive rows per thread ----------------
        if constexpr (RPT == 1)
        {
            const int64_t row = base + tid;
            double xa[1][W];
            double(&x)[W] = xa[0];
            if (row < n) {
                const TY* Y = static_cast<const TY*>(a.Y);
#pragma unroll
                for (int c = 0; c < W; ++c) x[c] = ldv(Y + row + c * a.ldy);
                if constexpr (UPD) update_rows<W, 1, TQ>(xa, static_cast<const TQ*>(a.Qu) + row, a.ldqu, a.pu, gC);
#pragma unroll
                for (int t = 0; t < NTRSM; ++t) {
                    const CD R = gR[t];
#pragma unroll
                    for (int c = 0; c < W; ++c) {
                        double v = x[c];
#pragma unroll
                        for (int q = 0; q < c; ++q) v -= x[q] * R[q + c * W];
                        x[c] = v * rinv[t * W + c];
                    }
                }
                if constexpr (WRITE) {
                    TX* X = static_cast<TX*>(a.X);
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
                for (int c = 0; c < W; ++c) xs[c * LDX + tid] = static_cast<XS>(x[c]);
            }
        }
        else
        {
            const int64_t row0 = base + (int64_t)RPT * tid;
            double x[RPT][W];
            if (row0 < n) {
                const TY* Y = static_cast<const TY*>(a.Y);
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    double v[RPT];
                    load_rows<RPT>(Y + (int64_t)c * a.ldy, vec, row0, n, v);
#pragma unroll
                    for (int r = 0; r < RPT; ++r) x[r][c] = v[r];
                }
                if constexpr (UPD) {
                  if (vec && row0 + RPT - 1 < n) {
                    update_rows<W, RPT, TQ>(x, static_cast<const TQ*>(a.Qu) + row0, a.ldqu, a.pu, gC);
                  } else {
                    const TQ* Q = static_cast<const TQ*>(a.Qu);
                    const int pu = a.pu;
                    int j = 0;
                    for (; j + 4 <= pu; j += 4) {
                        double q[4][RPT];
#pragma unroll
                        for (int u = 0; u < 4; ++u) load_rows<RPT>(Q + (int64_t)(j + u) * a.ldqu, vec, row0, n, q[u]);
#pragma unroll
                        for (int c = 0; c < W; ++c) {
                            const double c0 = gC[j + 0 + c * pu], c1 = gC[j + 1 + c * pu];
                            const double c2 = gC[j + 2 + c * pu], c3 = gC[j + 3 + c * pu];
#pragma unroll
                            for (int r = 0; r < RPT; ++r) {
                                double v = x[r][c];
                                v -= q[0][r] * c0;
                                v -= q[1][r] * c1;
                                v -= q[2][r] * c2;
                                v -= q[3][r] * c3;
                                x[r][c] = v;
                            }
                        }
                    }
                    for (; j < pu; ++j) {
                        double q[RPT];
                        load_rows<RPT>(Q + (int64_t)j * a.ldqu, vec, row0, n, q);
#pragma unroll
                        for (int c = 0; c < W; ++c) {
                            const double cj = gC[j + c * pu];
#pragma unroll
                            for (int r = 0; r < RPT; ++r) x[r][c] -= q[r] * cj;
                        }
                    }
                  }
                }
#pragma unroll
                for (int t = 0; t < NTRSM; ++t) {
                    const CD R = gR[t];
#pragma unroll
                    for (int c = 0; c < W; ++c) {
#pragma unroll
                        for (int r = 0; r < RPT; ++r) {
                            double v = x[r][c];
#pragma unroll
                            for (int q = 0; q < c; ++q) v -= x[r][q] * R[q + c * W];
                            x[r][c] = v * rinv[t * W + c];
                        }
                    }
                }
                if constexpr (WRITE) {
                    TX* X = static_cast<TX*>(a.X);
#pragma unroll
                    for (int c = 0; c < W; ++c) {
                        double v[RPT];
#pragma unroll
                        for (int r = 0; r < RPT; ++r) v[r] = x[r][c];
                        store_rows<RPT>(X + (int64_t)c * a.ldx, vec, row0, n, v);
                    }
                }
                // rows past n (a partial last pair) contribute zero to the reduction
#pragma unroll
                for (int r = 1; r < RPT; ++r)
                    if (row0 + r >= n)
#pragma unroll
                        for (int c = 0; c < W; ++c) x[r][c] = 0.0;
                if constexpr (RED == RED_SKETCH_SPARSE) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        hs[RPT * tid + r] = (row0 + r < n) ? splitmix64(a.sk_seed, (uint64_t)(row0 + r)) : 0;
                }
            } else {
#pragma unroll
                for (int r = 0; r < RPT; ++r)
#pragma unroll
                    for (int c = 0; c < W; ++c) x[r][c] = 0.0;
                if constexpr (RED == RED_SKETCH_SPARSE) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) hs[RPT * tid + r] = 0;
                }
            }
            if constexpr (HAS_RED) {
#pragma unroll
                for (int c = 0; c < W; ++c)
#pragma unroll
                    for (int r = 0; r < RPT; ++r) xs[c * LDX + RPT * tid + r] = static_cast<XS>(x[r][c]);
            }
        }
        if constexpr (HAS_RED) {
            // Sketches: each wave reduces the rows it staged itself, so only the wave's own LDS
            // writes must be visible (no workgroup barrier: the waves drift apart and one
            // wave's MFMA tiles overlap another's loads).  Projections and the Gram share the
            // whole strip across the waves (the projection's Q reads then cover each column's
            // strip segment at once, which the HBM pages favour).
            if constexpr (WAVE_LOCAL) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                __syncthreads();
            }
            if constexpr (SPM) {
                // ---------------- phase B, sparse-sign sketch on row masks ----------------
                constexpr int WROWS = STRIP / C::NWAVE;  // rows this wave staged (64 per thread row)
                const unsigned B = (unsigned)(a.sk_k / a.sk_zeta);
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int rb = wave * WROWS + u * 64;  // strip-local row of mask bit 0
                    const uint64_t h = hs[rb + lane];
                    const uint64_t vm = __ballot(base + rb + lane < n);
                    unsigned ml[SPR], mh[SPR], sl[SPR], sh[SPR];
#pragma unroll
                    for (int q = 0; q < SPR; ++q) ml[q] = mh[q] = sl[q] = sh[q] = 0u;
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        if (t < a.sk_zeta) {
                            const unsigned b8 = (unsigned)(h >> (8 * t)) & 0xffu;
                            const unsigned slot = ((b8 >> 1) * B) >> 7;
                            unsigned cl[SPR], ch[SPR];
#pragma unroll
                            for (int q = 0; q < SPR; ++q) cl[q] = ch[q] = ~0u;
#pragma unroll
                            for (int i = 0; i < SPM_BITS; ++i) {
                                if (i < spm_nbits) {
                                    const uint64_t bi = __ballot((slot >> i) & 1u);
#pragma unroll
                                    for (int q = 0; q < SPR; ++q) {
                                        cl[q] &= (unsigned)bi ^ spm_jn[q][i];
                                        ch[q] &= (unsigned)(bi >> 32) ^ spm_jn[q][i];
                                    }
                                }
                            }
                            const uint64_t sg = __ballot(b8 & 1u);
                            // keep this byte's masks only in the lanes whose sketch row it holds
#pragma unroll
                            for (int q = 0; q < SPR; ++q) {
                                const unsigned mine = t == spm_t[q] ? ~0u : 0u;
                                ml[q] |= cl[q] & mine;
                                mh[q] |= ch[q] & mine;
                                sl[q] |= (unsigned)sg & mine;
                                sh[q] |= (unsigned)(sg >> 32) & mine;
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < SPR; ++q) {
                        ml[q] &= (unsigned)vm;
                        mh[q] &= (unsigned)(vm >> 32);
                    }
                    // one sketch row per lane: each mask in two 32-row halves (the lowest set bit,
                    // its clearing and the sign are single 32-bit operations); two rows per lane:
                    // whole 64-row masks (four half loops would each run to their own longest
                    // half, and the sparser masks of larger sketches leave them short)
                    constexpr int NH = SPR == 1 ? 2 : 1;
#pragma unroll
                    for (int q = 0; q < SPR; ++q) {
#pragma unroll
                        for (int hf = 0; hf < NH; ++hf) {
                            using MW = typename std::conditional<NH == 2, unsigned, uint64_t>::type;
                            MW msk, sgm;
                            if constexpr (NH == 2) {
                                msk = hf ? mh[q] : ml[q];
                                sgm = hf ? sh[q] : sl[q];
                            } else {
                                msk = ((uint64_t)mh[q] << 32) | ml[q];
                                sgm = ((uint64_t)sh[q] << 32) | sl[q];
                            }
                            const int rh = rb + 32 * hf;
                            while (msk) {
                                const int bit = NH == 2 ? __builtin_ctz((unsigned)msk) : __builtin_ctzll((uint64_t)msk);
                                msk &= msk - 1u;
                                // +-1.0 from the row's sign bit for this byte
                                const unsigned sb = (unsigned)(sgm >> bit) & 1u;
                                const double sgn = __hiloint2double((int)((sb << 31) | 0x3FF00000u), 0);
#pragma unroll
                                for (int c = 0; c < W; ++c)
                                    sacc[q][c] = fma(sgn, (double)xs[c * LDX + rh + bit], sacc[q][c]);
                            }
                        }
                    }
                }
            } else if constexpr (MF) {
                // ---------------- phase B, MFMA tiles ----------------
                const int g = lane >> 4, ci = lane & 15;
                const TQ* Qp = static_cast<const TQ*>(a.Qp);
                const double* Th = a.theta;
                // 32-byte row pieces can be read as two 16-byte vectors when aligned
                bool vec = false;
                if constexpr (RED == RED_PROJ)
                    vec = (a.ldqp % 4) == 0 && ((uintptr_t)Qp % (4 * sizeof(TQ))) == 0;
                if constexpr (RED == RED_SKETCH_DENSE) vec = (a.ldtheta % 4) == 0 && ((uintptr_t)Th % 32) == 0;
                // rows per group: 16 (4 per lane), or 32 (8 per lane) for projections against an
                // FP32 basis on 4 x 4 x 4 blocks: a 4-byte piece load moves half the bytes of a
                // double one, so each lane loads two per column, as many bytes in flight as the
                // FP64 form (the staged operand stays in float until its MFMA)
                constexpr int UR = (RED == RED_PROJ && sizeof(TQ) == 4 && sizeof(XS) == 4 && B4) ? 8 : 4;
                constexpr int GR = 4 * UR;
                constexpr int GPW = STRIP / GR / C::NWAVE;  // row groups per wave
                static_assert(STRIP % (GR * C::NWAVE) == 0, "row groups must tile the strip");
                const int g0 = WAVE_LOCAL ? wave * GPW : wave, gstep = WAVE_LOCAL ? 1 : C::NWAVE;
                // not unrolled: the unrolled groups hold more loads and tiles at once and cost a
                // resident wave
#pragma unroll 1
                for (int gam = g0, it = 0; it < GPW; gam += gstep, ++it) {
                    const int r0 = gam * GR + UR * g;  // strip-local rows r0..r0+UR-1 for this lane
                    const bool full = base + r0 + 3 < n;
                    const bool full2 = base + r0 + UR - 1 < n;
                    // B operands: 16 x 16 x 4 tiles take column ci of the 4 rows; 4 x 4 x 4 blocks
                    // take column 4cb + lane % 4
                    double bv[B4 ? 1 : 4];
                    XS bq[B4 ? CB : 1][UR];
                    if constexpr (B4) {
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            const int col = 4 * cb + (lane & 3);
#pragma unroll
                            for (int u = 0; u < UR; ++u) bq[cb][u] = (col < W) ? xs[col * LDX + r0 + u] : XS(0);
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < 4; ++u) bv[u] = (ci < W) ? xs[ci * LDX + r0 + u] : 0.0;
                    }
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        if (m < ntiles) {
                            const int col = 16 * m + ci;
                            if constexpr (UR == 8) {
                                // the 8 pieces stay in float until their MFMA
                                float af[8];
#pragma unroll
                                for (int u = 0; u < 8; ++u) af[u] = 0.0f;
                                if (col < a.red_rows) {
                                    const float* qc = reinterpret_cast<const float*>(Qp) + (int64_t)col * a.ldqp + base + r0;
                                    if (vec && full2) {
                                        const float4 v0 = *reinterpret_cast<const float4*>(qc);
                                        const float4 v1 = *reinterpret_cast<const float4*>(qc + 4);
                                        af[0] = v0.x; af[1] = v0.y; af[2] = v0.z; af[3] = v0.w;
                                        af[4] = v1.x; af[5] = v1.y; af[6] = v1.z; af[7] = v1.w;
                                    } else {
#pragma unroll
                                        for (int u = 0; u < 8; ++u) af[u] = (base + r0 + u < n) ? qc[u] : 0.0f;
                                    }
                                }
#pragma unroll
                                for (int u = 0; u < 8; ++u)
#pragma unroll
                                    for (int cb = 0; cb < CB; ++cb)
                                        acc4[m * CB + cb] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                                            (double)af[u], (double)bq[cb][u], acc4[m * CB + cb], 0, 0, 0);
                                continue;
                            }
                            double av[4] = {0.0, 0.0, 0.0, 0.0};
                            if (col < a.red_rows) {
                                if constexpr (RED == RED_PROJ)
                                    load_col4(Qp + (int64_t)col * a.ldqp + base + r0, vec, full, base + r0, n, av);
                                else
                                    load_col4(Th + (int64_t)col * a.ldtheta + base + r0, vec, full, base + r0, n, av);
                            }
                            if constexpr (B4) {
#pragma unroll
                                for (int u = 0; u < 4; ++u)
#pragma unroll
                                    for (int cb = 0; cb < CB; ++cb)
                                        acc4[m * CB + cb] = __builtin_amdgcn_mfma_f64_4x4x4f64(
                                            av[u], (double)bq[cb][u], acc4[m * CB + cb], 0, 0, 0);
                            } else {
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    dacc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], dacc[m], 0, 0, 0);
                            }
                        }
                    }
                }
            } else if constexpr (GRAM) {
                // ---------------- phase B, lanes over rows, waves over output rows ----------------
#pragma unroll 2
                for (int r = 0; r < RPL; ++r) {
                    const int rr = r * 64 + lane;
                    double x[W];
#pragma unroll
                    for (int c = 0; c < W; ++c) x[c] = xs[c * LDX + rr];
#pragma unroll
                    for (int i = 0; i < MAXA; ++i) {
                        const int al = a_lo + i;
                        if (al < a.red_rows) {
                            const double xa = xs[(a.red_row0 + al) * LDX + rr];
#pragma unroll
                            for (int c = 0; c < W; ++c) acc[i][c] += xa * x[c];
                        }
                    }
                }
            }
            // the next strip's phase A overwrites the staged rows
            if constexpr (WAVE_LOCAL) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            } else {
                __syncthreads();
            }
        }
    }

    if constexpr (SPM) {
        // lane l holds sketch rows red_row0 + l + 64 q; the waves' sums are added through LDS in
        // wave order, four columns at a time
        double* out = a.partials + (int64_t)wg * a.part_stride;
#pragma unroll
        for (int q = 0; q < SPR; ++q) {
            const int r = lane + 64 * q;
#pragma unroll
            for (int c0 = 0; c0 < W; c0 += 4) {
#pragma unroll
                for (int cc = 0; cc < 4; ++cc)
                    if (c0 + cc < W) pred[(wave * 4 + cc) * 64 + lane] = sacc[q][c0 + cc];
                __syncthreads();
                if (wave == 0 && r < a.red_rows) {
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) {
                        if (c0 + cc < W) {
                            double v = 0.0;
                            for (int w2 = 0; w2 < C::NWAVE; ++w2) v += pred[(w2 * 4 + cc) * 64 + lane];
                            out[(a.red_row0 + r) + (int64_t)(c0 + cc) * a.part_rows_total] = v;
                        }
                    }
                }
                __syncthreads();
            }
        }
    } else if constexpr (B4) {
        // v_mfma_f64_4x4x4 output layout (measured on gfx950): D[i][j] of block b sits in lane
        // 4b + j + 16i, so lane l holds output row 16m + 4((l % 16) / 4) + l / 16 and column
        // 4cb + l % 4 of instruction (m, cb).  The waves' values are summed through LDS in wave
        // order.
        double* out = a.partials + (int64_t)wg * a.part_stride;
        const int srow = 4 * ((lane & 15) >> 2) + (lane >> 4);
        const int col = lane & 3;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (m >= ntiles) break;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) pred[(wave * 4 + cb) * 64 + lane] = acc4[m * CB + cb];
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    double v = 0.0;
                    for (int w2 = 0; w2 < C::NWAVE; ++w2) v += pred[(w2 * 4 + cb) * 64 + lane];
                    const int r = 16 * m + srow, c = 4 * cb + col;
                    if (r < a.red_rows && c < W) out[(a.red_row0 + r) + (int64_t)c * a.part_rows_total] = v;
                }
            }
            __syncthreads();
        }
    } else if constexpr (MF) {
        // v_mfma_f64_16x16x4 output layout (measured on gfx950): D[i][j] of a tile sits in
        // lane j + 16 * (i % 4), element i / 4.  The waves' tiles are summed through LDS in
        // wave order.
        double* out = a.partials + (int64_t)wg * a.part_stride;
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
    } else if constexpr (GRAM) {
        double* out = a.partials + (int64_t)wg * a.part_stride;
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

template <int W, typename T, int RED, bool UPD, int NTRSM, bool WRITE, int MTX = 0>
__global__ void __launch_bounds__((Cfg<W, RED>::NT)) pass_kernel(const PassArgs a) {
    pass_body<W, Tys<T, T, T>, RED, UPD, NTRSM, WRITE, MTX>(a, blockIdx.x, gridDim.x);
}

// FP64 panel (Y) against the FP32 basis (Q), written as TX.
template <int W, typename TX, int RED, bool UPD, int NTRSM, bool WRITE, int MTX = 0>
__global__ void __launch_bounds__((Cfg<W, RED>::NT)) pass_kernel_panel(const PassArgs a) {
    pass_body<W, Tys<double, float, TX>, RED, UPD, NTRSM, WRITE, MTX>(a, blockIdx.x, gridDim.x);
}

// Batched form: the template arguments are moved to the system of blockIdx.y.
template <int W, typename T, int RED, bool UPD, int NTRSM, bool WRITE, int MTX = 0>
__global__ void __launch_bounds__((Cfg<W, RED>::NT)) pass_kernel_batched(const PassArgs t, const BatchReloc br) {
    const int sys = batch_system(br);
    const BatchSys& d = br.sys[sys];
    PassArgs a = t;
    a.n = d.n;
    a.Y = batch_ptr(br, sys, d, t.Y);
    a.ldy = batch_ld(br, d, t.ldy);
    a.Qu = batch_ptr(br, sys, d, t.Qu);
    a.ldqu = batch_ld(br, d, t.ldqu);
    a.Cu = batch_ptr(br, sys, d, t.Cu);
    a.R1 = batch_ptr(br, sys, d, t.R1);
    a.R2 = batch_ptr(br, sys, d, t.R2);
    a.X = batch_ptr(br, sys, d, t.X);
    a.ldx = batch_ld(br, d, t.ldx);
    a.Qp = batch_ptr(br, sys, d, t.Qp);
    a.ldqp = batch_ld(br, d, t.ldqp);
    a.partials = batch_ptr(br, sys, d, t.partials);
    a.sk_seed = d.seed;
    pass_body<W, Tys<T, T, T>, RED, UPD, NTRSM, WRITE, MTX>(a, blockIdx.x, gridDim.x);
}

using KernelPtr = void (*)(const PassArgs);
using BatchedKernelPtr = void (*)(const PassArgs, const BatchReloc);

// The pass variants the orchestration launches: (reduction, update, solves, write).
template <int W, typename T>
KernelPtr select_w(const PassKey& k) {
    const int r = k.red;
    const bool u = k.upd, wr = k.write;
    const int t = k.ntrsm;
    // projections: the fewest accumulator tiles that hold the launch's rows
    const int mt = (k.tiles >= 1 && k.tiles <= 4) ? 4 : (k.tiles >= 5 && k.tiles <= 6) ? 6 : 8;
    if (!u && t == 0 && !wr) {
        if (r == RED_PROJ)
            return mt == 4   ? &pass_kernel<W, T, RED_PROJ, false, 0, false, 4>
                   : mt == 6 ? &pass_kernel<W, T, RED_PROJ, false, 0, false, 6>
                             : &pass_kernel<W, T, RED_PROJ, false, 0, false>;
        if (r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, false, 0, false>;
        if (r == RED_SKETCH_SPARSE)
            return mt == 4 ? &pass_kernel<W, T, RED_SKETCH_SPARSE, false, 0, false, 4>
                           : &pass_kernel<W, T, RED_SKETCH_SPARSE, false, 0, false>;
        if (r == RED_SKETCH_DENSE) return &pass_kernel<W, T, RED_SKETCH_DENSE, false, 0, false>;
    }
    if (u && t == 0 && wr) {
        if (r == RED_NONE) return &pass_kernel<W, T, RED_NONE, true, 0, true>;
        if (r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, true, 0, true>;
        if (r == RED_SKETCH_SPARSE)
            return mt == 4 ? &pass_kernel<W, T, RED_SKETCH_SPARSE, true, 0, true, 4>
                           : &pass_kernel<W, T, RED_SKETCH_SPARSE, true, 0, true>;
        if (r == RED_SKETCH_DENSE) return &pass_kernel<W, T, RED_SKETCH_DENSE, true, 0, true>;
    }
    if (!u && t == 1 && !wr && r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, false, 1, false>;
    if (!u && t == 2 && wr) {
        if (r == RED_PROJ)
            return mt == 4   ? &pass_kernel<W, T, RED_PROJ, false, 2, true, 4>
                   : mt == 6 ? &pass_kernel<W, T, RED_PROJ, false, 2, true, 6>
                             : &pass_kernel<W, T, RED_PROJ, false, 2, true>;
        if (r == RED_GRAM) return &pass_kernel<W, T, RED_GRAM, false, 2, true>;
    }
    if (r == RED_NONE && t == 1 && wr) {
        if (!u) return &pass_kernel<W, T, RED_NONE, false, 1, true>;
        return &pass_kernel<W, T, RED_NONE, true, 1, true>;
    }
    return nullptr;
}

// The variants of the mixed-precision GMRES panel step: panel 1 reads the FP64 panel
// against the FP32 basis and writes the panel (projection; update + sketch); panel 2 writes
// the finished columns into the FP32 basis (update + solve).
template <int W>
KernelPtr select_w_panel(const PassKey& k) {
    const int r = k.red;
    const bool u = k.upd, wr = k.write;
    const int t = k.ntrsm;
    const int mt = (k.tiles >= 1 && k.tiles <= 4) ? 4 : (k.tiles >= 5 && k.tiles <= 6) ? 6 : 8;
    if (k.panel == 1) {
        if (!u && t == 0 && !wr && r == RED_PROJ)
            return mt == 4   ? &pass_kernel_panel<W, double, RED_PROJ, false, 0, false, 4>
                   : mt == 6 ? &pass_kernel_panel<W, double, RED_PROJ, false, 0, false, 6>
                             : &pass_kernel_panel<W, double, RED_PROJ, false, 0, false>;
        if (u && t == 0 && wr) {
            if (r == RED_SKETCH_SPARSE)
                return mt == 4 ? &pass_kernel_panel<W, double, RED_SKETCH_SPARSE, true, 0, true, 4>
                               : &pass_kernel_panel<W, double, RED_SKETCH_SPARSE, true, 0, true>;
            if (r == RED_SKETCH_DENSE) return &pass_kernel_panel<W, double, RED_SKETCH_DENSE, true, 0, true>;
        }
    }
    if (k.panel == 2 && r == RED_NONE && t == 1 && wr)
        return u ? &pass_kernel_panel<W, float, RED_NONE, true, 1, true>
                 : &pass_kernel_panel<W, float, RED_NONE, false, 1, true>;
    return nullptr;
}

// The batched variants the lock-step two-stage solver launches.
template <int W, typename T>
BatchedKernelPtr select_w_batched(const PassKey& k) {
    const int r = k.red;
    const bool u = k.upd, wr = k.write;
    const int t = k.ntrsm;
    const bool few = k.tiles >= 1 && k.tiles <= 4;
    if (!u && t == 0 && !wr) {
        if (r == RED_PROJ)
            return few ? &pass_kernel_batched<W, T, RED_PROJ, false, 0, false, 4>
                       : &pass_kernel_batched<W, T, RED_PROJ, false, 0, false>;
        if (r == RED_SKETCH_SPARSE)
            return few ? &pass_kernel_batched<W, T, RED_SKETCH_SPARSE, false, 0, false, 4>
                       : &pass_kernel_batched<W, T, RED_SKETCH_SPARSE, false, 0, false>;
    }
    if (u && t == 0 && wr && r == RED_SKETCH_SPARSE)
        return few ? &pass_kernel_batched<W, T, RED_SKETCH_SPARSE, true, 0, true, 4>
                   : &pass_kernel_batched<W, T, RED_SKETCH_SPARSE, true, 0, true>;
    if (r == RED_NONE && t == 1 && wr) {
        if (!u) return &pass_kernel_batched<W, T, RED_NONE, false, 1, true>;
        return &pass_kernel_batched<W, T, RED_NONE, true, 1, true>;
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
    passk::BatchedKernelPtr fnb;  // batched form (null where not instantiated)
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
