// Pass kernels for panel width 11 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w11(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<11>(k)
                   : k.f32 ? passk::select_w<11, float>(k) : passk::select_w<11, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<11, float>(k) : passk::select_w_batched<11, double>(k);
    s.threads = passk::threads_w<11>(k.red);
    s.rows = passk::rows_w<11>(k.red);
    return s;
}
}  // namespace sko
