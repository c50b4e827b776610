// Restarted s-step GMRES on the device (Fig. 1; two-stage Fig. 5).
#include "context.h"

namespace sko {

sko_status gmres_impl(sko_ctx, const sko_csr*, const double*, double*, const sko_gmres_opts*, sko_gmres_info* info) {
    if (info) *info = sko_gmres_info{};
    return SKO_EUNSUPPORTED;
}

sko_status gmres_batched_impl(sko_ctx, int32_t, const sko_csr*, const double* const*, double* const*,
                              const sko_gmres_opts*, sko_gmres_info*) {
    return SKO_EUNSUPPORTED;
}

}  // namespace sko
