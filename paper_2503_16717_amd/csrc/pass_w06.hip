// Pass kernels for panel width 6 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w6(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<6>(k)
                   : k.f32 ? passk::select_w<6, float>(k) : passk::select_w<6, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<6, float>(k) : passk::select_w_batched<6, double>(k);
    s.threads = passk::threads_w<6>(k.red);
    s.rows = passk::rows_w<6>(k.red);
    return s;
}
}  // namespace sko
