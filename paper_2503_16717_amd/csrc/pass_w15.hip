// Pass kernels for panel width 15 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w15(const PassKey& k) {
    return k.f32 ? passk::select_w<15, float>(k) : passk::select_w<15, double>(k);
}
}  // namespace sko
