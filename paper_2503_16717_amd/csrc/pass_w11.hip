// Pass kernels for panel width 11 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w11(const PassKey& k) {
    return k.f32 ? passk::select_w<11, float>(k) : passk::select_w<11, double>(k);
}
}  // namespace sko
