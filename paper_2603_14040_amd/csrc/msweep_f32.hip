// float instantiation of the multi-sweep Gauss-Seidel tile launcher.
#include "msweep.h"

namespace tph {
template hipError_t launch_gs_tile<float>(const Geom&, const Geom&, int, int, int, int, const float*, const float*,
                                        float*, float*, const float*, const float*, const float*, const float*,
                                        const float*, const float*, float*, float*, float, hipStream_t,
                                        hipEvent_t, hipEvent_t);
}  // namespace tph
