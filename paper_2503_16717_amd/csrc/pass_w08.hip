// Pass kernels for panel width 8 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w8(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<8>(k)
                   : k.f32 ? passk::select_w<8, float>(k) : passk::select_w<8, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<8, float>(k) : passk::select_w_batched<8, double>(k);
    s.threads = passk::threads_w<8>(k.red);
    s.rows = passk::rows_w<8>(k.red);
    return s;
}
}  // namespace sko
