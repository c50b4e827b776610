// Pass kernels for panel width 10 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w10(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<10>(k)
                   : k.f32 ? passk::select_w<10, float>(k) : passk::select_w<10, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<10, float>(k) : passk::select_w_batched<10, double>(k);
    s.threads = passk::threads_w<10>(k.red);
    s.rows = passk::rows_w<10>(k.red);
    return s;
}
}  // namespace sko
