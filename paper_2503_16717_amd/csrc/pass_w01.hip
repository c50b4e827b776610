// Pass kernels for panel width 1 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w1(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<1>(k)
                   : k.f32 ? passk::select_w<1, float>(k) : passk::select_w<1, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<1, float>(k) : passk::select_w_batched<1, double>(k);
    s.threads = passk::threads_w<1>(k.red);
    s.rows = passk::rows_w<1>(k.red);
    return s;
}
}  // namespace sko
