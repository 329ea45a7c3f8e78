// fhp_stepk.hip -- the temporally blocked pass (kernel in fhp_stepk.h) for
// state buffers below 4 GiB, and the dispatch by depth, rule set and buffer
// size.
#include "fhp_stepk.h"

namespace fhp {

hipError_t launch_stepk(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                        const Dyn& D, uint64_t t, uint32_t T, hipStream_t st) {
    StepkArgs a;
    a.H = L.H;
    a.wd = L.wd;
    a.T = (T + 1) & ~1u;  // even, so that y0 is even
    a.walls = L.walls;
    a.ps = L.ps;
    a.t0 = t;
    a.key_chir = D.key_chir;
    a.key_force = D.key_force;
    a.thr_force = D.thr_force;
    a.chi_and = (D.chir_mode == FHP_CHIR_HASH) ? ~0u : 0u;
    a.chi_or = (D.chir_mode == FHP_CHIR_ONE) ? ~0u : 0u;
    if (planes_wide(L.ps)) return launch_stepk_wide(K, in, out, L, a, D.rules, st);
    if (L.wd == 64) return launch_stepk_wave(K, in, out, L, a, D.rules, st);
    return launch_depth<false>(K, in, out, L, a, D.rules, st);
}

}  // namespace fhp
