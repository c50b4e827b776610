// Pass kernels for panel width 9 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w9(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<9>(k)
                   : k.f32 ? passk::select_w<9, float>(k) : passk::select_w<9, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<9, float>(k) : passk::select_w_batched<9, double>(k);
    s.threads = passk::threads_w<9>(k.red);
    s.rows = passk::rows_w<9>(k.red);
    return s;
}
}  // namespace sko
