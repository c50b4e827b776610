// Dispatch and launch of the row-strip pass kernels (kernel template in pass_impl.h,
// instantiated per panel width in pass_wNN.hip).
#include "pass_impl.h"

namespace sko {
namespace {

using passk::KernelPtr;

KernelPtr select_kernel(const PassKey& k) {
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
        default: return nullptr;
    }
}

constexpr int NT = kPassThreads;
constexpr int NWAVE = NT / 64;

}  // namespace

int pass_rows_per_launch(int W) {
    switch (W) {
#define SKO_W(w) case w: return NWAVE * passk::maxa<w>();
        SKO_W(1) SKO_W(2) SKO_W(3) SKO_W(4) SKO_W(5) SKO_W(6) SKO_W(7) SKO_W(8)
        SKO_W(9) SKO_W(10) SKO_W(11) SKO_W(12) SKO_W(13) SKO_W(14) SKO_W(15) SKO_W(16)
#undef SKO_W
        default: return 0;
    }
}

int pass_grid_cap(const PassKey& key) {
    KernelPtr f = select_kernel(key);
    if (!f) return 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f), NT, 0) !=
        hipSuccess)
        return 0;
    if (per_cu < 1) per_cu = 1;
    return per_cu * cus;
}

hipError_t launch_pass(const PassKey& key, const PassArgs& args, int grid, hipStream_t stream) {
    KernelPtr f = select_kernel(key);
    if (!f) return hipErrorInvalidValue;
    if (key.upd && args.pu * key.W > kMaxUpdCoef) return hipErrorInvalidValue;
    if (key.red != RED_NONE && args.red_rows > pass_rows_per_launch(key.W)) return hipErrorInvalidValue;
    if (grid < 1) return hipErrorInvalidValue;
    const size_t lds = key.upd ? sizeof(double) * (size_t)args.pu * key.W : 0;
    hipLaunchKernelGGL(f, dim3(grid), dim3(NT), lds, stream, args);
    return hipGetLastError();
}

}  // namespace sko
