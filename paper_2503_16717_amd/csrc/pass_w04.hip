// Pass kernels for panel width 4 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w4(const PassKey& k) {
    return k.f32 ? passk::select_w<4, float>(k) : passk::select_w<4, double>(k);
}
}  // namespace sko
