// Adjoint of the flux stage instantiated for the double bulk type.
#include "gks_flux_vjp.h"

namespace gks {
template hipError_t launch_flux_vjp_t<double>(const DevMesh &, const AdjFlux &, const Params &, double, int,
                                          hipStream_t);
}  // namespace gks
