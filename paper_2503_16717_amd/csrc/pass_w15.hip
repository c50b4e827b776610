// Pass kernels for panel width 15 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w15(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<15>(k)
                   : k.f32 ? passk::select_w<15, float>(k) : passk::select_w<15, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<15, float>(k) : passk::select_w_batched<15, double>(k);
    s.threads = passk::threads_w<15>(k.red);
    s.rows = passk::rows_w<15>(k.red);
    return s;
}
}  // namespace sko
