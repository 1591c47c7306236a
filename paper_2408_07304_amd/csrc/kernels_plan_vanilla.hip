// Persistent mixed-shape kernel, vanilla scheme, and the scheme dispatch.
#include "kernels_plan.h"

namespace zinc {

hipError_t launch_plan_zinc(const PlanDev& d, const double* slots, uint64_t* ct, hipStream_t s);

hipError_t launch_plan(const PlanDev& d, int scheme, const double* slots, uint64_t* ct, hipStream_t s) {
    if (scheme == ZINC_SCHEME_ZINC) return launch_plan_zinc(d, slots, ct, s);
    return launch_plan_scheme<ZINC_SCHEME_VANILLA>(d, slots, ct, s);
}

}  // namespace zinc
