// Pass kernels for panel width 14 (double and float storage).
#include "pass_impl.h"

namespace sko {
PassSel select_pass_w14(const PassKey& k) {
    PassSel s;
    s.fn = k.panel ? passk::select_w_panel<14>(k)
                   : k.f32 ? passk::select_w<14, float>(k) : passk::select_w<14, double>(k);
    s.fnb = k.panel ? nullptr
                    : k.f32 ? passk::select_w_batched<14, float>(k) : passk::select_w_batched<14, double>(k);
    s.threads = passk::threads_w<14>(k.red);
    s.rows = passk::rows_w<14>(k.red);
    return s;
}
}  // namespace sko
