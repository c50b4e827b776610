// Pass kernels for panel width 3 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w3(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<3>(k)
                   : k.f32 ? passk::select_w<3, float>(k) : passk::select_w<3, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<3, float>(k) : passk::select_w_batched<3, double>(k);
    s.threads = passk::threads_w<3>(k.red);
    s.rows = passk::rows_w<3>(k.red);
    return s;
}
}  // namespace sko
