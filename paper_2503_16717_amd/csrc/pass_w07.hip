// Pass kernels for panel width 7 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w7(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<7>(k)
                   : k.f32 ? passk::select_w<7, float>(k) : passk::select_w<7, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<7, float>(k) : passk::select_w_batched<7, double>(k);
    s.threads = passk::threads_w<7>(k.red);
    s.rows = passk::rows_w<7>(k.red);
    return s;
}
}  // namespace sko
