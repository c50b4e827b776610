// Pass kernels for panel width 13 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w13(const PassKey& k) {
    return k.f32 ? passk::select_w<13, float>(k) : passk::select_w<13, double>(k);
}
}  // namespace sko
