// Pass kernels for panel width 6 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w6(const PassKey& k) {
    return k.f32 ? passk::select_w<6, float>(k) : passk::select_w<6, double>(k);
}
}  // namespace sko
