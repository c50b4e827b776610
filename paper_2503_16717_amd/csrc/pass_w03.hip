// Pass kernels for panel width 3 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w3(const PassKey& k) {
    return k.f32 ? passk::select_w<3, float>(k) : passk::select_w<3, double>(k);
}
}  // namespace sko
