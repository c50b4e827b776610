// Pass kernels for panel width 2 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w2(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<2>(k)
                   : k.f32 ? passk::select_w<2, float>(k) : passk::select_w<2, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<2, float>(k) : passk::select_w_batched<2, double>(k);
    s.threads = passk::threads_w<2>(k.red);
    s.rows = passk::rows_w<2>(k.red);
    return s;
}
}  // namespace sko
