// Pass kernels for panel width 4 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w4(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<4>(k)
                   : k.f32 ? passk::select_w<4, float>(k) : passk::select_w<4, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<4, float>(k) : passk::select_w_batched<4, double>(k);
    s.threads = passk::threads_w<4>(k.red);
    s.rows = passk::rows_w<4>(k.red);
    return s;
}
}  // namespace sko
