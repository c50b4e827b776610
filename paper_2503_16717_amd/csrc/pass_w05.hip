// Pass kernels for panel width 5 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w5(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<5>(k)
                   : k.f32 ? passk::select_w<5, float>(k) : passk::select_w<5, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<5, float>(k) : passk::select_w_batched<5, double>(k);
    s.threads = passk::threads_w<5>(k.red);
    s.rows = passk::rows_w<5>(k.red);
    return s;
}
}  // namespace sko
