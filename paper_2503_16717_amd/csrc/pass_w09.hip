// Pass kernels for panel width 9 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w9(const PassKey& k) {
    return k.f32 ? passk::select_w<9, float>(k) : passk::select_w<9, double>(k);
}
}  // namespace sko
