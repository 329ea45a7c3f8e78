// fhp_stepk_wave.hip -- the temporally blocked pass (kernel in fhp_stepk.h)
// for rows of a power of two words up to 64: one wave per band, carries
// between lanes by DPP (its own translation unit so that it compiles in
// parallel).
#include "fhp_stepk.h"

namespace fhp {

hipError_t launch_stepk_wave(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                             const StepkArgs& a, uint32_t rules, hipStream_t st) {
    return launch_depth<false, true>(K, in, out, L, a, rules, st);
}

}  // namespace fhp
