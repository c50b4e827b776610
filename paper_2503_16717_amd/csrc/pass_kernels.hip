// Dispatch and launch of the row-strip pass kernels (kernel template in pass_impl.h,
// instantiated per panel width in pass_wNN.hip).
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "pass_impl.h"

namespace sko {
namespace {

PassSel select_kernel(const PassKey& k) {
    switch (k.W) {
        case 1: return select_pass_w1(k);
        case 2: return select_pass_w2(k);
        case 3: return select_pass_w3(k);
        case 4: return select_pass_w4(k);
        case 5: return select_pass_w5(k);
        case 6: return select_pass_w6(k);
        case 7: return select_pass_w7(k);
        case 8: return select_pass_w8(k);
        case 9: return select_pass_w9(k);
        case 10: return select_pass_w10(k);
        case 11: return select_pass_w11(k);
        case 12: return select_pass_w12(k);
        case 13: return select_pass_w13(k);
        case 14: return select_pass_w14(k);
        case 15: return select_pass_w15(k);
        case 16: return select_pass_w16(k);
        default: return PassSel{nullptr, nullptr, 0, 0};
    }
}

}  // namespace

int pass_rows_per_launch(int W, int red) {
    PassKey k{W, false, red, false, 0, false};
    return select_kernel(k).rows;
}

int pass_strip_rows(const PassKey& key) { return select_kernel(key).threads; }

const void* pass_kernel_id(const PassKey& key) { return reinterpret_cast<const void*>(select_kernel(key).fn); }

// Resident workgroups of a pass kernel, queried once per (kernel, device): the occupancy
// query costs more than a launch.
int resident_grid(const void* kernel, int threads) {
    int dev = 0;
    if (!kernel || hipGetDevice(&dev) != hipSuccess) return -1;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    const std::pair<const void*, int> id{kernel, dev};
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = cache.find(id);
        if (it != cache.end()) return it->second;
    }
    int cus = 0, per_cu = 0;
    int res = -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) == hipSuccess && cus > 0)
        res = std::max(1, per_cu) * cus;
    std::lock_guard<std::mutex> lk(mu);
    cache[id] = res;
    return res;
}

int pass_grid_cap(const PassKey& key) {
    PassSel s = select_kernel(key);
    if (!s.fn) return 0;
    const int r = resident_grid(reinterpret_cast<const void*>(s.fn), s.threads);
    return r > 0 ? r : 0;
}

hipError_t launch_pass(const PassKey& key, const PassArgs& args, int grid, hipStream_t stream, const BatchReloc* br) {
    PassSel s = select_kernel(key);
    if (!s.fn || (br && !s.fnb)) return hipErrorInvalidValue;
    if (key.upd && args.pu * key.W > kMaxUpdCoef) return hipErrorInvalidValue;
    if (key.red != RED_NONE && args.red_rows > s.rows) return hipErrorInvalidValue;
    if (grid < 1) return hipErrorInvalidValue;
    if (br) {
        if (br->nact < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(s.fnb, dim3(grid, br->nact), dim3(s.threads), 0, stream, args, *br);
    } else {
        hipLaunchKernelGGL(s.fn, dim3(grid), dim3(s.threads), 0, stream, args);
    }
    return hipGetLastError();
}

}  // namespace sko
