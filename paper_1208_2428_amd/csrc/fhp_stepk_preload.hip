// fhp_stepk_preload.hip -- the temporally blocked pass (kernel in fhp_stepk.h)
// with the rows of its pipeline fill loaded at once, for launches of at most
// one wave per SIMD (its own translation unit so that it compiles in parallel).
#include "fhp_stepk.h"

namespace fhp {

hipError_t launch_stepk_preload(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                                const StepkArgs& a, uint32_t rules, bool one_wave,
                                hipStream_t st) {
    if (one_wave) return launch_depth<false, true, true>(K, in, out, L, a, rules, st);
    return launch_depth<false, false, true>(K, in, out, L, a, rules, st);
}

}  // namespace fhp
