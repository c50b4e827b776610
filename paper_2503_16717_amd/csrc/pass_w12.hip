// Pass kernels for panel width 12 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w12(const PassKey& k) {
    return k.f32 ? passk::select_w<12, float>(k) : passk::select_w<12, double>(k);
}
}  // namespace sko
