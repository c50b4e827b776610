// Pass kernels for panel width 14 (double and float storage).
#include "pass_impl.h"

namespace sko {
passk::KernelPtr select_pass_w14(const PassKey& k) {
    return k.f32 ? passk::select_w<14, float>(k) : passk::select_w<14, double>(k);
}
}  // namespace sko
