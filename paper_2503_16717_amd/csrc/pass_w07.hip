// Pass kernels for panel width 7 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w7(const PassKey& k) {
    return k.f32 ? passk::select_w<7, float>(k) : passk::select_w<7, double>(k);
}
}  // namespace sko
