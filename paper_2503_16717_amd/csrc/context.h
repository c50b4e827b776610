// Library context: device, stream and the reusable device workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "sko.h"
#include "sko_internal.h"

namespace sko {

// Event-timed per-kernel-kind statistics (sko_profile_enable / sko_profile_read).
struct Profiler {
    struct Stat {
        int64_t launches = 0;
        double ms = 0.0;
        double bytes = 0.0;
    };
    struct Pending {
        std::string name;
        double bytes;
        hipEvent_t e0, e1;
    };
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    std::map<std::string, Stat> stats;

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Bracket one launch: begin() before it, end() after it.
    int begin(const std::string& name, double bytes, hipStream_t st) {
        if (!on) return -1;
        Pending p{name, bytes, take(), take()};
        if (!p.e0 || !p.e1 || hipEventRecord(p.e0, st) != hipSuccess) return -1;
        pending.push_back(p);
        return (int)pending.size() - 1;
    }
    void end(int idx, hipStream_t st) {
        if (idx >= 0) (void)hipEventRecord(pending[idx].e1, st);
    }
    // After the stream has been synchronised: fold the pending launches into stats.
    void flush() {
        for (Pending& p : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
                Stat& s = stats[p.name];
                s.launches += 1;
                s.ms += ms;
                s.bytes += p.bytes;
            }
            pool.push_back(p.e0);
            pool.push_back(p.e1);
        }
        pending.clear();
    }
    void release() {
        for (Pending& p : pending) {
            pool.push_back(p.e0);
            pool.push_back(p.e1);
        }
        pending.clear();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

// Two HIP events destroyed on every return path.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() = default;
    EventPair(const EventPair&) = delete;
    EventPair& operator=(const EventPair&) = delete;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    hipError_t create() {
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        return hipEventCreate(&b);
    }
    // milliseconds between the two records (after b has completed)
    double ms() const {
        float v = 0.f;
        return hipEventElapsedTime(&v, a, b) == hipSuccess ? (double)v : 0.0;
    }
};

// Phase times of a solve (sko_gmres_opts::phase_timing): an event pair around each phase
// interval, folded into per-phase sums whenever the host has synchronised the stream.
struct PhaseTimer {
    enum { SPMV = 0, ORTH = 1, SMALL = 2, NPH = 3 };
    bool on = false;
    double ms[NPH] = {0.0, 0.0, 0.0};
    struct Pending {
        int ph;
        hipEvent_t e0, e1;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    int open = -1;  // phase of the interval in progress

    PhaseTimer() = default;
    PhaseTimer(const PhaseTimer&) = delete;
    PhaseTimer& operator=(const PhaseTimer&) = delete;
    ~PhaseTimer() {
        for (Pending& p : pending) {
            pool.push_back(p.e0);
            pool.push_back(p.e1);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
    // Start phase `ph` (ending the interval in progress, if another phase).
    void phase(int ph, hipStream_t st) {
        if (!on || ph == open) return;
        stop(st);
        hipEvent_t e0 = take(), e1 = take();
        if (!e0 || !e1 || hipEventRecord(e0, st) != hipSuccess) {
            if (e0) pool.push_back(e0);
            if (e1) pool.push_back(e1);
            return;
        }
        pending.push_back(Pending{ph, e0, e1});
        open = ph;
    }
    void stop(hipStream_t st) {
        if (!on || open < 0) return;
        (void)hipEventRecord(pending.back().e1, st);
        open = -1;
    }
    // Fold the recorded intervals into the sums; call after stop() and a synchronisation of
    // the stream.
    void flush() {
        if (!on) return;
        for (Pending& p : pending) {
            float v = 0.f;
            if (hipEventElapsedTime(&v, p.e0, p.e1) == hipSuccess) ms[p.ph] += v;
            pool.push_back(p.e0);
            pool.push_back(p.e1);
        }
        pending.clear();
    }
};

}  // namespace sko

struct sko_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int cus = 0;
    void* ws = nullptr;        // device workspace
    size_t ws_bytes = 0;
    int* status_host = nullptr;  // pinned host word for the breakdown status
    void* pinned = nullptr;      // pinned staging for small results copied to the host
    size_t pinned_bytes = 0;
    // four host words that kernels write directly (mapped, coherent pinned memory): the
    // one-stage GMRES block publishes its implicit residual and status word there, so no
    // copy launch follows each block.  zc_dev: the device's address of the same words.
    double* zc_host = nullptr;
    double* zc_dev = nullptr;
    sko::Profiler prof;
    // sko_autotune_orth: workgroups per CU per (pass kernel, log2 of its strip count)
    std::map<std::pair<const void*, int>, int> grid_wpc;
    // private stream on which launch graphs are captured (created on first use)
    hipStream_t cap_stream = nullptr;
};

namespace sko {

// Bump allocator over the context workspace, or over a fixed buffer (256-byte aligned
// slices).  Offsets are resolved against the context's workspace at use, so an arena may
// be laid out before the workspace has grown.
class Arena {
   public:
    explicit Arena(sko_ctx c) : c_(c) {}
    Arena(sko_ctx c, void* fixed) : c_(c), fixed_(fixed) {}
    size_t reserve(size_t bytes) {
        size_t off = (used_ + 255) & ~size_t(255);
        used_ = off + bytes;
        return off;
    }
    size_t used() const { return used_; }
    template <typename T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(static_cast<char*>(fixed_ ? fixed_ : c_->ws) + off);
    }

   private:
    sko_ctx c_;
    void* fixed_ = nullptr;
    size_t used_ = 0;
};

// Grow the context workspace to at least `bytes` (never shrinks).
inline sko_status ensure_workspace(sko_ctx c, size_t bytes) {
    if (c->ws_bytes >= bytes) return SKO_OK;
    if (c->ws) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return SKO_EDEVICE;
        (void)hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&c->ws, want) != hipSuccess) {
        c->ws = nullptr;
        return SKO_ENOMEM;
    }
    c->ws_bytes = want;
    return SKO_OK;
}

// Grow the pinned host staging buffer to at least `bytes`.
inline sko_status ensure_pinned(sko_ctx c, size_t bytes) {
    if (c->pinned_bytes >= bytes) return SKO_OK;
    if (c->pinned) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return SKO_EDEVICE;
        (void)hipHostFree(c->pinned);
        c->pinned = nullptr;
        c->pinned_bytes = 0;
    }
    if (hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        return SKO_ENOMEM;
    }
    c->pinned_bytes = bytes;
    return SKO_OK;
}

// The mapped host words kernels write results into (allocated once per context).
inline sko_status ensure_zerocopy(sko_ctx c) {
    if (c->zc_host) return SKO_OK;
    void* h = nullptr;
    if (hipHostMalloc(&h, 4 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return SKO_ENOMEM;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipHostFree(h);
        return SKO_EDEVICE;
    }
    c->zc_host = static_cast<double*>(h);
    c->zc_dev = static_cast<double*>(d);
    return SKO_OK;
}

#define SKO_HIP(call)                                  \
    do {                                               \
        if ((call) != hipSuccess) return SKO_EDEVICE;  \
    } while (0)

sko_status orth_blocks_impl(sko_ctx c, int64_t n, int32_t nb, int32_t w, const void* V, int64_t ldv,
                            void* Q, int64_t ldq, double* R, int64_t ldr, const sko_orth_opts* o,
                            int32_t* breakdown_col);
sko_status orth_block_impl(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq,
                           const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rp, double* Rd,
                           const sko_orth_opts* o, int32_t* breakdown_col);
sko_status orth_block_noalloc_impl(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq,
                                   const void* V, int64_t ldv, void* Qo, int64_t ldqo, double* Rp, double* Rd,
                                   const sko_orth_opts* o, int32_t* breakdown_col);
// Fixed no-allocation scratch of a device (noalloc.hip): noalloc_init once per device with
// that device current, at context creation; noalloc_scratch returns the device address
// (null before a successful noalloc_init).
constexpr size_t kNoallocScratchBytes = size_t(32) << 20;
sko_status noalloc_init(int device);
void* noalloc_scratch(int device);
sko_status sketch_apply_impl(sko_ctx c, int64_t n, int32_t w, const void* X, int64_t ldx, int32_t precision,
                             const sko_sketch* sk, double* Y, int64_t ldy);
sko_status autotune_orth_impl(sko_ctx c, int64_t n, int32_t nb, int32_t w, const sko_orth_opts* o);
sko_status gmres_impl(sko_ctx c, const sko_csr* A, const double* b, double* x, const sko_gmres_opts* o,
                      sko_gmres_info* info);
sko_status gmres_batched_impl(sko_ctx c, int32_t nsys, const sko_csr* A, const double* const* b,
                              double* const* x, const sko_gmres_opts* o, sko_gmres_info* infos);

}  // namespace sko
