// Pass kernels for panel width 10 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w10(const PassKey& k) {
    return k.f32 ? passk::select_w<10, float>(k) : passk::select_w<10, double>(k);
}
}  // namespace sko
