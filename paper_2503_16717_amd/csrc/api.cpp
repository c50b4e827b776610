// C ABI entry points of libsko (declared in include/sko.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "context.h"

extern "C" {

sko_status sko_create(int device, void* hip_stream, sko_ctx* out) {
    if (!out) return SKO_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return SKO_EDEVICE;
    if (device < 0 || device >= count) return SKO_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SKO_EDEVICE;
    sko_ctx c = new (std::nothrow) sko_ctx_s();
    if (!c) return SKO_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        delete c;
        return SKO_EDEVICE;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->status_host), 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SKO_ENOMEM;
    }
    // device address of this device's fixed scratch (sko_orth_block_noalloc), once per device
    const sko_status ns = sko::noalloc_init(device);
    if (ns != SKO_OK) {
        (void)hipHostFree(c->status_host);
        delete c;
        return ns;
    }
    *out = c;
    return SKO_OK;
}

sko_status sko_destroy(sko_ctx c) {
    if (!c) return SKO_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->ws) (void)hipFree(c->ws);
    if (c->status_host) (void)hipHostFree(c->status_host);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->zc_host) (void)hipHostFree(c->zc_host);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->prof.release();
    delete c;
    return SKO_OK;
}

sko_status sko_set_stream(sko_ctx c, void* hip_stream) {
    if (!c) return SKO_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return SKO_OK;
}

const char* sko_strerror(sko_status s) {
    switch (s) {
        case SKO_OK: return "success";
        case SKO_EINVAL: return "invalid argument";
        case SKO_EDEVICE: return "HIP runtime error";
        case SKO_ENOMEM: return "out of device memory";
        case SKO_EBREAKDOWN: return "breakdown: non-positive Cholesky pivot or zero Householder diagonal";
        case SKO_ENOCONV: return "GMRES did not converge within maxiter";
        case SKO_EUNSUPPORTED: return "unsupported configuration";
        case SKO_ESCRATCH: return "request needs more device memory than the fixed no-allocation scratch holds";
    }
    return "unknown status";
}

sko_status sko_orth_block(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq, const void* V,
                          int64_t ldv, void* Q_out, int64_t ldqo, double* R_proj, double* R_diag,
                          const sko_orth_opts* opts, int32_t* breakdown_col) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::orth_block_impl(c, n, p, w, Q, ldq, V, ldv, Q_out, ldqo, R_proj, R_diag, opts, breakdown_col);
}

sko_status sko_orth_block_noalloc(sko_ctx c, int64_t n, int32_t p, int32_t w, const void* Q, int64_t ldq,
                                  const void* V, int64_t ldv, void* Q_out, int64_t ldqo, double* R_proj,
                                  double* R_diag, const sko_orth_opts* opts, int32_t* breakdown_col) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::orth_block_noalloc_impl(c, n, p, w, Q, ldq, V, ldv, Q_out, ldqo, R_proj, R_diag, opts,
                                        breakdown_col);
}

sko_status sko_orth_blocks(sko_ctx c, int64_t n, int32_t nb, int32_t w, const void* V, int64_t ldv, void* Q,
                           int64_t ldq, double* R, int64_t ldr, const sko_orth_opts* opts,
                           int32_t* breakdown_col) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::orth_blocks_impl(c, n, nb, w, V, ldv, Q, ldq, R, ldr, opts, breakdown_col);
}

sko_status sko_sketch_apply(sko_ctx c, int64_t n, int32_t w, const void* X, int64_t ldx, int32_t precision,
                            const sko_sketch* sketch, double* Y, int64_t ldy) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::sketch_apply_impl(c, n, w, X, ldx, precision, sketch, Y, ldy);
}

sko_status sko_gmres(sko_ctx c, const sko_csr* A, const double* b, double* x, const sko_gmres_opts* opts,
                     sko_gmres_info* info) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::gmres_impl(c, A, b, x, opts, info);
}

sko_status sko_gmres_batched(sko_ctx c, int32_t nsys, const sko_csr* A, const double* const* b, double* const* x,
                             const sko_gmres_opts* opts, sko_gmres_info* infos) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::gmres_batched_impl(c, nsys, A, b, x, opts, infos);
}

sko_status sko_autotune_orth(sko_ctx c, int64_t n, int32_t nb, int32_t w, const sko_orth_opts* opts) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    return sko::autotune_orth_impl(c, n, nb, w, opts);
}

sko_status sko_profile_enable(sko_ctx c, int enable) {
    if (!c) return SKO_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SKO_EDEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SKO_EDEVICE;
    c->prof.flush();
    if (enable) c->prof.stats.clear();
    c->prof.on = enable != 0;
    return SKO_OK;
}

int32_t sko_profile_read(sko_ctx c, sko_kernel_stat* out, int32_t max) {
    if (!c || max < 0 || (max > 0 && !out)) return -SKO_EINVAL;
    std::vector<std::pair<std::string, sko::Profiler::Stat>> v(c->prof.stats.begin(), c->prof.stats.end());
    std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.second.ms > b.second.ms; });
    const int32_t cnt = (int32_t)v.size();
    for (int32_t i = 0; i < cnt && i < max; ++i) {
        std::memset(&out[i], 0, sizeof(sko_kernel_stat));
        std::strncpy(out[i].name, v[i].first.c_str(), sizeof(out[i].name) - 1);
        out[i].launches = v[i].second.launches;
        out[i].total_ms = v[i].second.ms;
        out[i].bytes = v[i].second.bytes;
    }
    return cnt;
}

}  // extern "C"
