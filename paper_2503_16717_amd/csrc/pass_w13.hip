// Pass kernels for panel width 13 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w13(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<13>(k)
                   : k.f32 ? passk::select_w<13, float>(k) : passk::select_w<13, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<13, float>(k) : passk::select_w_batched<13, double>(k);
    s.threads = passk::threads_w<13>(k.red);
    s.rows = passk::rows_w<13>(k.red);
    return s;
}
}  // namespace sko
