// Batched launches: one kernel launch serves every active system of a batch of
// independent solves (blockIdx.y selects the system).
//
// The host builds each launch's arguments once, for a template system (system 0's
// addresses).  The kernel moves every pointer that lies in one of the template's regions
// to the same place in its own system's region:
//   * the Krylov basis (ld0 x columns, element size eb): same column and row of the
//     system's basis, whose leading dimension and row count differ per system;
//   * the small workspace, the partial sums and the reduction counters: equal-sized
//     regions laid out one after another, so the offset is sys * region size.
// Per-system scalars (row count, CSR operator, b, x, D^{-1}, sketch seed) come from the
// system table.
//
// The relocation is by address range, so it relies on one invariant: every pointer argument
// of a batched kernel is per-system data inside one of the four template regions, and data
// shared by all systems (the system table, the active list, the flat launch's block starts)
// travels in BatchReloc itself, never as a pointer argument.  batch_regions_disjoint checks
// on the host that the template regions overlap neither each other nor those shared arrays,
// so no shared datum can be taken for a template one.  Leading dimensions go through
// batch_ld only for tall operands (basis columns), never for the small dense arrays.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sko {

struct BatchSys {
    int64_t n;               // rows
    int64_t ld;              // basis leading dimension
    int64_t nnz;
    char* Q;                 // basis
    const int32_t* rowptr;
    const int32_t* colind;
    const double* val;       // A (FP64)
    const void* val_op;      // matrix-powers operator values (A D^{-1}, double or float)
    const double* b;
    double* x;
    const double* dinv;      // Jacobi D^{-1} or null
    uint64_t seed;           // sparse-sign sketch seed
    int32_t kupd;            // basis vectors in the solution update at a cycle end
    int32_t pad_;
};

struct BatchReloc {
    const BatchSys* sys;     // system table (device)
    const int* active;       // blockIdx.y -> system index (device)
    int nact;                // active systems = gridDim.y
    int eb;                  // basis element size (4 or 8)
    const char* q0;          // template basis and its extent
    int64_t q0_bytes;
    int64_t ld0;
    const char* ws0;         // template small workspace; system i's starts at ws0 + i * ws_bytes
    int64_t ws_bytes;
    const char* part0;       // template partial sums
    int64_t part_bytes;
    const char* cnt0;        // template reduction counters
    int64_t cnt_bytes;
    // Flat launches (one workgroup per `chunk` rows of a system, no idle workgroups): the
    // first workgroup of active slot j is blk0[j] (nact + 1 entries, device; blk0[nact] ==
    // nblk, the launch's grid).  Null: none set up.
    const int* blk0;
    int nblk;
    int chunk;
};

// Host check of the invariant above: the template regions of `br` are pairwise disjoint and
// disjoint from each of the `nshared` byte ranges [shared[i], shared[i] + shared_bytes[i]).
inline bool batch_regions_disjoint(const BatchReloc& br, const void* const* shared, const int64_t* shared_bytes,
                                   int nshared) {
    const char* lo[4] = {br.q0, br.ws0, br.part0, br.cnt0};
    const int64_t len[4] = {br.q0_bytes, br.ws_bytes, br.part_bytes, br.cnt_bytes};
    auto overlap = [](const char* a, int64_t na, const char* b, int64_t nb) {
        return a && b && na > 0 && nb > 0 && a < b + nb && b < a + na;
    };
    for (int i = 0; i < 4; ++i) {
        for (int j = i + 1; j < 4; ++j)
            if (overlap(lo[i], len[i], lo[j], len[j])) return false;
        for (int k = 0; k < nshared; ++k)
            if (overlap(lo[i], len[i], static_cast<const char*>(shared[k]), shared_bytes[k])) return false;
    }
    return true;
}

#ifdef __HIPCC__
// System served by this workgroup.
__device__ __forceinline__ int batch_system(const BatchReloc& br) { return br.active[blockIdx.y]; }

template <typename P>
__device__ __forceinline__ P* batch_ptr(const BatchReloc& br, int sys, const BatchSys& d, P* p) {
    if (!p) return p;
    const char* c = reinterpret_cast<const char*>(p);
    int64_t o = c - br.q0;
    if (o >= 0 && o < br.q0_bytes) {
        const int64_t e = o / br.eb;
        const int64_t col = e / br.ld0, row = e - col * br.ld0;
        return reinterpret_cast<P*>(d.Q + (col * d.ld + row) * br.eb);
    }
    o = c - br.ws0;
    if (o >= 0 && o < br.ws_bytes) return reinterpret_cast<P*>(const_cast<char*>(c) + (int64_t)sys * br.ws_bytes);
    o = c - br.part0;
    if (o >= 0 && o < br.part_bytes)
        return reinterpret_cast<P*>(const_cast<char*>(c) + (int64_t)sys * br.part_bytes);
    o = c - br.cnt0;
    if (o >= 0 && o < br.cnt_bytes) return reinterpret_cast<P*>(const_cast<char*>(c) + (int64_t)sys * br.cnt_bytes);
    return p;
}

// Active slot of this workgroup in a flat launch: the j with blk0[j] <= blockIdx.x <
// blk0[j + 1] (every active system has at least one workgroup).
__device__ __forceinline__ int flat_slot(const BatchReloc& br) {
    const int b = blockIdx.x;
    int lo = 0, hi = br.nact;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (br.blk0[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// A tall leading dimension of the template becomes the system's.
__device__ __forceinline__ int64_t batch_ld(const BatchReloc& br, const BatchSys& d, int64_t ld) {
    return ld == br.ld0 ? d.ld : ld;
}
#endif

}  // namespace sko
