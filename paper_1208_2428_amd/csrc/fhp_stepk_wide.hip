// fhp_stepk_wide.hip -- the temporally blocked pass (kernel in fhp_stepk.h)
// for state buffers of 4 GiB and more: one buffer resource per plane.
#include "fhp_stepk.h"

namespace fhp {

hipError_t launch_stepk_wide(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                             const StepkArgs& a, uint32_t rules, hipStream_t st) {
    return launch_depth<true>(K, in, out, L, a, rules, st);
}

}  // namespace fhp
