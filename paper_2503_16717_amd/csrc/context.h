// Library context: device, stream and the reusable device workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>

#include "sko.h"
#include "sko_internal.h"

struct sko_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int cus = 0;
    void* ws = nullptr;        // device workspace
    size_t ws_bytes = 0;
    int* status_host = nullptr;  // pinned host word for the breakdown status
};

namespace sko {

// Bump allocator over the context workspace (256-byte aligned slices).
class Arena {
   public:
    explicit Arena(sko_ctx c) : c_(c) {}
    size_t reserve(size_t bytes) {
        size_t off = (used_ + 255) & ~size_t(255);
        used_ = off + bytes;
        return off;
    }
    size_t used() const { return used_; }
    template <typename T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(static_cast<char*>(c_->ws) + off);
    }

   private:
    sko_ctx c_;
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
sko_status gmres_impl(sko_ctx c, const sko_csr* A, const double* b, double* x, const sko_gmres_opts* o,
                      sko_gmres_info* info);
sko_status gmres_batched_impl(sko_ctx c, int32_t nsys, const sko_csr* A, const double* const* b,
                              double* const* x, const sko_gmres_opts* o, sko_gmres_info* infos);

}  // namespace sko
