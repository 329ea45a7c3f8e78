// fhp_stepk_k5.hip -- the depth-5 pass of the temporally blocked kernel
// (fhp_stepk.h) with carries through LDS and rows streamed two ahead, for state
// buffers below 4 GiB: the pass of wide lattices such as 16384 x 16384.  Its
// own translation unit, so that it can be compiled with the backend's
// instruction-level-parallelism schedule (build.py), which measured 2.2%
// faster on 16384^2 at the same two waves per SIMD (238 VGPRs) but 4% slower
// for the depth-4 and one-wave passes of smaller lattices.
#include "fhp_stepk.h"

namespace fhp {

hipError_t launch_stepk_k5(const uint64_t* in, uint64_t* out, const Lattice& L, const StepkArgs& a,
                           uint32_t rules, hipStream_t st) {
    return launch_k2<false, 5>(in, out, L, a, rules, st);
}

}  // namespace fhp
