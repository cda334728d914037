// Kernel B (gas-kinetic flux) instantiated for the float bulk type.
#include "gks_flux_kernel.h"

namespace gks {
template hipError_t launch_flux_t<float>(const DevMesh &, const DevState &, const Params &, double, const double *,
                                     int, hipStream_t);
}  // namespace gks
