// Persistent mixed-shape kernel, Zinc scheme (a translation unit of its own so
// that the two schemes compile in parallel).
#include "kernels_plan.h"

namespace zinc {

hipError_t launch_plan_zinc(const PlanDev& d, const double* slots, uint64_t* ct, hipStream_t s) {
    return launch_plan_scheme<ZINC_SCHEME_ZINC>(d, slots, ct, s);
}

}  // namespace zinc
