// Pass kernels for panel width 16 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w16(const PassKey& k) {
    return k.f32 ? passk::select_w<16, float>(k) : passk::select_w<16, double>(k);
}
}  // namespace sko
