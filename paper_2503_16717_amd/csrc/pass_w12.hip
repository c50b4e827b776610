// Pass kernels for panel width 12 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w12(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<12>(k)
                   : k.f32 ? passk::select_w<12, float>(k) : passk::select_w<12, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<12, float>(k) : passk::select_w_batched<12, double>(k);
    s.threads = passk::threads_w<12>(k.red);
    s.rows = passk::rows_w<12>(k.red);
    return s;
}
}  // namespace sko
