// fhp_stepk.hip -- the temporally blocked pass (kernel in fhp_stepk.h) for
// state buffers below 4 GiB, and the dispatch by depth, rule set and buffer
// size.
#include "fhp_stepk.h"

namespace fhp {

hipError_t launch_stepk(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                        const Dyn& D, uint64_t t, uint32_t T, uint32_t simds, hipStream_t st) {
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
    // Contiguous runs of bands per XCD (band_of) where bands are one wave or
    // less and short, so that each row is read by several neighbouring bands:
    // on 4096^2 at K = 5 +19%, +8%, +6%, +4% and +1% for 2-, 4-, 6-, 8- and
    // 16-row bands, on 2048^2 +5% to +9%.  Taller bands lose by it (32-row
    // bands of a 4096 x 65536 lattice -25%, 16384^2 at 16 and 32 rows -10% and
    // -8%), and rows of 128 words gain nothing at 4 or 8 rows.
    a.xcd_runs = (L.wd <= 64 && a.T <= 8) ? 1u : 0u;
    if (planes_wide(L.ps)) return launch_stepk_wide(K, in, out, L, a, D.rules, st);
    // At most one wave per SIMD: nothing hides a wave's load latency, and the
    // preloaded pipeline fill pays: on 4096^2 +8% at K = 3 and +11% at K = 5
    // (4-row bands), on 2048^2 +5%.  With two waves per SIMD the other wave
    // hides it and the preload costs 1-5% (16384^2, 8192^2, 4096 x 65536).
    const uint64_t waves = (uint64_t)((L.H + a.T - 1) / a.T) * ((L.wd + 63) / 64);
    // Rows of a power of two words up to 64 run one wave per band with DPP
    // carries (the row repeated across the wave); other widths exchange
    // carries through LDS.
    const bool one_wave = 64 % L.wd == 0;
    if (waves <= simds) return launch_stepk_preload(K, in, out, L, a, D.rules, one_wave, st);
    if (one_wave) return launch_stepk_wave(K, in, out, L, a, D.rules, st);
    if (K == 5) return launch_stepk_k5(in, out, L, a, D.rules, st);
    return launch_depth<false, false, false, 4>(K, in, out, L, a, D.rules, st);
}

}  // namespace fhp
