// Pass kernels for panel width 8 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w8(const PassKey& k) {
    return k.f32 ? passk::select_w<8, float>(k) : passk::select_w<8, double>(k);
}
}  // namespace sko
