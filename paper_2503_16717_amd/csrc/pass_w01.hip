// Pass kernels for panel width 1 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w1(const PassKey& k) {
    return k.f32 ? passk::select_w<1, float>(k) : passk::select_w<1, double>(k);
}
}  // namespace sko
