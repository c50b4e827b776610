// Pass kernels for panel width 2 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w2(const PassKey& k) {
    return k.f32 ? passk::select_w<2, float>(k) : passk::select_w<2, double>(k);
}
}  // namespace sko
