// Pass kernels for panel width 5 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w5(const PassKey& k) {
    return k.f32 ? passk::select_w<5, float>(k) : passk::select_w<5, double>(k);
}
}  // namespace sko
