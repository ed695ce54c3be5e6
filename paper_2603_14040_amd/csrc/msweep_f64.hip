// double instantiation of the multi-sweep Gauss-Seidel tile launcher.
#include "msweep.h"

namespace tph {
template hipError_t launch_gs_tile<double>(const Geom&, const Geom&, int, int, int, int, const double*, const double*,
                                        double*, double*, const double*, const double*, const double*, const double*,
                                        const double*, const double*, double*, double*, double, hipStream_t,
                                        hipEvent_t, hipEvent_t);
}  // namespace tph
