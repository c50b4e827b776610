// Pass kernels for panel width 16 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w16(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<16>(k)
                   : k.f32 ? passk::select_w<16, float>(k) : passk::select_w<16, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<16, float>(k) : passk::select_w_batched<16, double>(k);
    s.threads = passk::threads_w<16>(k.red);
    s.rows = passk::rows_w<16>(k.red);
    return s;
}
}  // namespace sko
