// fhp_stepk.h -- temporally blocked FHP update: K time steps per pass over
// HBM (K = 1..FHP_MAX_DEPTH).
//
// Decomposition.  A workgroup owns a band of T consecutive rows (T even) and
// the full lattice width: thread w holds 64-node word w of every row it
// touches, so the periodic wrap in x needs no halo words.  The band sweeps
// downwards through rows y0-K .. y0+T+K-1 of the input buffer, one row per
// iteration.  Level 0 is the loaded row; level l (1..K) is the state after l
// steps, and its row rho = r - l is computed as soon as level l-1 has
// produced rows rho-1, rho and rho+1 (pull streaming reads exactly those).
// Each level keeps the last two rows of the level below it in registers, so
// every input row is read from HBM once per band and only the 2K halo rows
// are read twice (by the neighbouring bands).  Level K rows y0 .. y0+T-1 are
// stored.  The first 2K iterations fill the pipeline; after that every
// iteration produces one row of every level.
//
// Horizontal carries.  A 1-node shift of a word needs one bit of the
// neighbouring word: bit 63 of the left word for rotl1, bit 0 of the right
// word for rotr1.  After a row is produced each thread publishes in LDS the
// four 32-bit halves of its word that its neighbours will shift in over the
// row's life (which four depends on the row's parity), the workgroup
// synchronises, and each thread reads its two neighbours' halves (wrapping at
// the row ends).  Every shift is then two funnel shifts (v_alignbit) with no
// bit packing.  Two LDS slots alternate so that one barrier per exchange
// suffices.  Rows of 64 words, or of a power of two fewer repeated across
// the 64 lanes (ONE_WAVE), are one wave per band, and the halves move between
// neighbouring lanes by DPP rotations instead, with no LDS and no barrier.
//
// Loads.  Rows are loaded two iterations ahead of their use.  Launches of at
// most one wave per SIMD (PRELOAD), where no other wave hides a load's
// latency, load the 2K + 2 rows of the pipeline fill at once.
//
// Row parity.  Odd rows are shifted by +1/2, so which planes shift depends on
// the parity of the destination row.  With y0 and H even it equals the
// parity of (i + K + l) for iteration i and level l; the sweep is unrolled by
// two so that parity is a compile-time constant in every level.
//
// Time: level l of a pass starting at t0 applies step t0 + l - 1 (hash
// counters use that t and the absolute row index, so results do not depend
// on K or on the band height).
#pragma once

#include "fhp_device.h"
#include "fhp_internal.h"
#include "fhp_sweep.h"

namespace fhp {

struct StepkArgs {
    uint32_t H, wd;        // rows, words per row
    uint32_t T;            // band height (even)
    uint32_t walls;        // rows 0 and H-1 solid
    uint64_t ps;           // plane stride in words
    uint64_t t0;           // steps done before this pass
    uint64_t key_chir, key_force, thr_force;
    uint32_t chi_and, chi_or;  // chirality word = (hash & chi_and) | chi_or, per 32-bit half
    uint32_t xcd_runs;         // give each XCD a contiguous run of bands (see band_of)
};

namespace {

// Band processed by workgroup b of nb.  Workgroups are dispatched round-robin
// over the 8 XCDs (b to XCD b mod 8).  With `runs` set, XCD x instead takes a
// contiguous run of bands, so that the halo rows a band shares with its
// neighbours are read through one L2.
__device__ inline uint32_t band_of(uint32_t b, uint32_t nb, uint32_t runs) {
    if (!runs) return b;
    const uint32_t q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

constexpr size_t kStepkLdsBytes = 2 * 4 * kMaxBlockedWords * sizeof(uint32_t);

// ONE_WAVE: rows of wd words, wd a power of two up to 64, one wave per band:
// lane l holds word l mod wd, so that the row repeats 64 / wd times across
// the wave and a rotation of the whole wave by one lane brings every lane its
// periodic neighbour; the carries move by DPP (gather_wave) instead of through
// LDS.  Only the first copy stores.
// PRELOAD: the 2K + 2 rows of the pipeline fill are loaded at once, for
// launches of at most one wave per SIMD (see launch_stepk).
template <int K, bool FORCE, bool MASK, int RULES, bool WIDE, bool ONE_WAVE = false,
          bool PRELOAD = false>
__global__ void __launch_bounds__(512) k_stepk(const uint64_t* __restrict__ in,
                                                uint64_t* __restrict__ out,
                                                const uint64_t* __restrict__ S, StepkArgs a) {
    extern __shared__ uint32_t xch[];  // 2 slots x 4 halves x kMaxBlockedWords entries
    const uint32_t lane = threadIdx.x;
    const bool valid = lane < a.wd;
    const uint32_t w = ONE_WAVE ? (lane & (a.wd - 1)) : (valid ? lane : 0);
    const uint32_t wl = w ? w - 1 : a.wd - 1;
    const uint32_t wr = (w + 1 == a.wd) ? 0 : w + 1;
    const uint32_t H = a.H;
    const uint32_t y0 = band_of(blockIdx.x, gridDim.x, a.xcd_runs) * a.T;
    const uint32_t rows = min(a.T, H - y0);
    const int n_iter = (int)rows + 2 * K;
    const uint64_t base_chi = word_base(a.key_chir, w);
    const uint64_t base_frc = word_base(a.key_force, w);
    uint32_t chi_and = a.chi_and;  // kept in a vector register (see chir_word)
    asm("" : "+v"(chi_and));

    auto wrap_row = [&](int r) __attribute__((always_inline)) -> uint32_t {
        int m = r % (int)H;
        return (uint32_t)(m < 0 ? m + (int)H : m);
    };
    // Byte offset of word w of row y within a plane (planes are < 4 GiB).
    auto offset = [&](uint32_t y) __attribute__((always_inline)) -> uint32_t { return (y * a.wd + w) * 8u; };
    const uint32_t plane_bytes = H * a.wd * 8u;
    const Planes<WIDE> pin(in, a.ps, plane_bytes), pout(out, a.ps, plane_bytes);
    const __amdgpu_buffer_rsrc_t rs = region_rsrc(S, plane_bytes);
    // Issues the loads of row y; wall rows are applied when the row is
    // consumed, so that nothing waits on these loads before the next row.
    auto load = [&](uint32_t y, Row& x) __attribute__((always_inline)) {
        const uint32_t off = offset(y);
#pragma unroll
        for (int c = 0; c < 7; c++) x.p[c] = pin.load(c, off);
        if (MASK) x.s = buf_load64(rs, off, 0);
    };
    uint32_t slot = 0;

    // Level l keeps two rows of level l-1: rho-1 (only planes 3, 4 and one
    // neighbour half are read again) and rho (everything).  Flat arrays indexed by
    // compile-time levels stay in registers.
    uint64_t a3[K + 1], a4[K + 1], bp[K + 1][7], bs[K + 1];
    uint32_t ac[K + 1], b2[K + 1], b5[K + 1], bq[K + 1];
    auto push = [&](auto lc, const Row& x) __attribute__((always_inline)) {
        constexpr int l = decltype(lc)::value;
        a3[l] = bp[l][3];
        a4[l] = bp[l][4];
        ac[l] = bq[l];
#pragma unroll
        for (int c = 0; c < 7; c++) bp[l][c] = x.p[c];
        bs[l] = x.s;
        b2[l] = x.c[1];
        b5[l] = x.c[2];
        bq[l] = x.c[3];
    };
    // Rows are loaded two ahead of the sweep (nxt, nxt2).  With PRELOAD the
    // rows of the whole pipeline fill are loaded before it instead: the fill
    // iterations run few levels, so a wave that has its SIMD to itself would
    // otherwise wait out most of each load's latency there.
    constexpr int kPre = PRELOAD ? 2 * K + 2 : 2;
    Row pre[kPre];
    static_for<0, kPre - 1>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        load(wrap_row((int)y0 - K + j), pre[j]);
    });
    Row nxt = pre[kPre - 2], nxt2 = pre[kPre - 1];

    // Row bookkeeping, in scalar registers and kept incrementally (a wave that
    // has its SIMD to itself issues every scalar instruction in place of a
    // vector one).  Before iteration i, whose row is r = y0 - K + i,
    // yq[j] = (r + 1 - j) mod H and hq[j] = row_term(0, yq[j]); an iteration
    // shifts both windows by one and appends row r + 2.  Level l then computes
    // row yq[2 + l], whose hash counter term is tq[l] + hq[2 + l].
    constexpr int kWin = K + 3;
    uint32_t yq[kWin];
    uint64_t hq[kWin], tq[K + 1];
    static_for<0, kWin - 1>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        yq[j] = wrap_row((int)y0 - K + 1 - j);
        hq[j] = row_term(0, yq[j]);
    });
    static_for<1, K>([&](auto lc) __attribute__((always_inline)) {
        constexpr int l = decltype(lc)::value;
        tq[l] = row_term(a.t0 + (uint64_t)(l - 1), 0);
    });
    const uint64_t row_step = row_term(0, 1);

    // One sweep iteration.  FULL: every level is active (i >= 2K).  PAR: i & 1.
    // X: the row of level 0 in the preloaded fill; otherwise it is taken from
    // the prefetch queue.
    auto body = [&](int i, auto full_c, auto par_c, Row X) __attribute__((always_inline)) {
        constexpr bool FULL = decltype(full_c)::value;
        constexpr int PAR = decltype(par_c)::value;
        static_for<1, kWin - 1>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = kWin - decltype(jc)::value;
            yq[j] = yq[j - 1];
            hq[j] = hq[j - 1];
        });
        yq[0] = (yq[1] + 1 == H) ? 0u : yq[1] + 1;
        hq[0] = yq[0] ? hq[1] + row_step : 0ull;
        const uint32_t y = yq[2];
        if constexpr (FULL || !PRELOAD) {
            X = nxt;
            nxt = nxt2;
            // prefetch two rows ahead (the last iterations reload their own row)
            load((i + 2 < n_iter) ? yq[0] : y, nxt2);
        }
        const uint64_t wall = (a.walls && (y == 0 || y == H - 1)) ? ~0ull : 0ull;  // uniform
        X.s = MASK ? (X.s | wall) : wall;
        // The hash words of the next level do not depend on the exchange, so
        // they are formed between publishing a row and the barrier.
        uint64_t chi = 0, coin = 0;
        uint32_t up = 0;
        auto hashes = [&](auto hc) __attribute__((always_inline)) {
            constexpr int l = decltype(hc)::value;
            const uint64_t R = in_sgprs(tq[l] + hq[2 + l]);
            chi = chir_word(mix64(base_chi + R), chi_and, a.chi_or);
            if (FORCE) {
                const uint64_t hf = mix64(base_frc + R);
                coin = coin_bit(hf);
                up = coin_up(hf, a.thr_force);
            }
        };
        constexpr bool odd0 = ((PAR + K) & 1) != 0;  // y0 even: parity of y
        if constexpr (ONE_WAVE) {
            if (FULL || i >= 2) hashes(std::integral_constant<int, 1>{});
            gather_wave<odd0>(X);
        } else {
            publish<odd0>(xch, slot, kMaxBlockedWords, lane, X);
            if (FULL || i >= 2) hashes(std::integral_constant<int, 1>{});
            gather<odd0>(xch, slot, kMaxBlockedWords, wl, wr, X);
        }
        bool have = true;  // X holds a new row of level l-1
        static_for<1, K>([&](auto lc) __attribute__((always_inline)) {
            constexpr int l = decltype(lc)::value;
            if (!FULL) {
                if (!have) return;
                if (i < 2 * l) {
                    push(lc, X);
                    have = false;
                    return;
                }
            }
            const uint32_t rho = yq[2 + l];
            constexpr bool odd = ((PAR + K + l) & 1) != 0;  // parity of rho
            uint64_t n[7];
            stream_in<odd>(a3[l], a4[l], ac[l], bp[l], b2[l], b5[l], X, n);
            const uint64_t sw = bs[l];
            Row Y;
            update<RULES>(n, sw, chi, coin, up, Y.p);
            Y.s = sw;
            push(lc, X);
            if constexpr (l < K) {
                if constexpr (ONE_WAVE) {
                    if (FULL || i >= 2 * (l + 1)) hashes(std::integral_constant<int, l + 1>{});
                    gather_wave<odd>(Y);
                } else {
                    publish<odd>(xch, slot, kMaxBlockedWords, lane, Y);
                    if (FULL || i >= 2 * (l + 1)) hashes(std::integral_constant<int, l + 1>{});
                    gather<odd>(xch, slot, kMaxBlockedWords, wl, wr, Y);
                }
                X = Y;
            } else if (valid) {
                const uint32_t off = offset(rho);
#pragma unroll
                for (int c = 0; c < 7; c++) pout.store(c, off, Y.p[c]);
            }
        });
    };

    using F = std::false_type;
    using T = std::true_type;
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    // pipeline fill (n_iter >= 2K + 2)
    static_for<0, K - 1>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = 2 * decltype(jc)::value;
        body(j, F{}, P0{}, pre[PRELOAD ? j : 0]);
        body(j + 1, F{}, P1{}, pre[PRELOAD ? j + 1 : 0]);
    });
    int i = 2 * K;
    // Steady state, six rows per trip: a row's planes 3 and 4 stay live for
    // three iterations, and with two iterations per trip the compiler
    // rotates them through registers with moves (about 6 per word and level).
    for (; i + 6 <= n_iter; i += 6) {
        body(i, T{}, P0{}, nxt);
        body(i + 1, T{}, P1{}, nxt);
        body(i + 2, T{}, P0{}, nxt);
        body(i + 3, T{}, P1{}, nxt);
        body(i + 4, T{}, P0{}, nxt);
        body(i + 5, T{}, P1{}, nxt);
    }
    // The last 0, 2 or 4 rows (rows is even, so n_iter - 2K is even).  At
    // depths up to 3 in straight-line code: no loop back-edge, so no rotating
    // moves (bands of 4 rows run all their full iterations here; 3% faster on
    // 4096^2 and 2048^2).  Deeper passes, and FHP-III, would spill there.
    if constexpr (K <= 3 && RULES != kRulesFHP3) {
        if (n_iter - i == 4) {
            body(i, T{}, P0{}, nxt);
            body(i + 1, T{}, P1{}, nxt);
            body(i + 2, T{}, P0{}, nxt);
            body(i + 3, T{}, P1{}, nxt);
        } else if (n_iter - i == 2) {
            body(i, T{}, P0{}, nxt);
            body(i + 1, T{}, P1{}, nxt);
        }
    } else {
        for (; i < n_iter; i += 2) {
            body(i, T{}, P0{}, nxt);
            body(i + 1, T{}, P1{}, nxt);
        }
    }
}

template <bool WIDE, int K, bool FORCE, bool MASK, int RULES = kRulesFHP2, bool ONE_WAVE = false,
          bool PRELOAD = false>
hipError_t launch_k(const uint64_t* in, uint64_t* out, const Lattice& L, const StepkArgs& a,
                    hipStream_t st) {
    const uint32_t nt = (L.wd + 63) / 64 * 64;
    const uint32_t bands = (L.H + a.T - 1) / a.T;
    if constexpr (ONE_WAVE) {
        if (L.wd == 0 || 64 % L.wd != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_stepk<K, FORCE, MASK, RULES, WIDE, true, PRELOAD>), dim3(bands),
                           dim3(64), 0, st, in, out, L.S, a);
    } else {
        hipLaunchKernelGGL((k_stepk<K, FORCE, MASK, RULES, WIDE, false, PRELOAD>), dim3(bands),
                           dim3(nt), kStepkLdsBytes, st, in, out, L.S, a);
    }
    return hipGetLastError();
}

// FHP-II has a kernel for every combination of forcing and obstacles; the
// other rule sets use the forcing variant (a zero rate draws no coin).
template <bool WIDE, int K, bool OW = false, bool PL = false>
hipError_t launch_k2(const uint64_t* in, uint64_t* out, const Lattice& L, const StepkArgs& a,
                     uint32_t rules, hipStream_t st) {
    const bool force = a.thr_force != 0, mask = L.S != nullptr;
    if (rules == kRulesFHP1)
        return mask ? launch_k<WIDE, K, true, true, kRulesFHP1, OW, PL>(in, out, L, a, st)
                    : launch_k<WIDE, K, true, false, kRulesFHP1, OW, PL>(in, out, L, a, st);
    if (rules == kRulesFHP3) {
        if constexpr (K <= kMaxDepthFHP3)
            return mask ? launch_k<WIDE, K, true, true, kRulesFHP3, OW, PL>(in, out, L, a, st)
                        : launch_k<WIDE, K, true, false, kRulesFHP3, OW, PL>(in, out, L, a, st);
        return hipErrorInvalidValue;
    }
    if (force) return mask ? launch_k<WIDE, K, true, true, kRulesFHP2, OW, PL>(in, out, L, a, st)
                           : launch_k<WIDE, K, true, false, kRulesFHP2, OW, PL>(in, out, L, a, st);
    return mask ? launch_k<WIDE, K, false, true, kRulesFHP2, OW, PL>(in, out, L, a, st)
                : launch_k<WIDE, K, false, false, kRulesFHP2, OW, PL>(in, out, L, a, st);
}

// Launches the pass of depth K for buffers of the given width class
// (OW: the one-wave kernel for rows of a power of two words up to 64; PL: the
// preloaded fill).  KMAX: the deepest pass this instantiation launches (deeper
// ones are left to another translation unit).
template <bool WIDE, bool OW = false, bool PL = false, int KMAX = 5>
hipError_t launch_depth(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L, const StepkArgs& a,
                        uint32_t rules, hipStream_t st) {
    switch (K) {
        case 1: return launch_k2<WIDE, 1, OW, PL>(in, out, L, a, rules, st);
        case 2: return launch_k2<WIDE, 2, OW, PL>(in, out, L, a, rules, st);
        case 3: return launch_k2<WIDE, 3, OW, PL>(in, out, L, a, rules, st);
        case 4: return launch_k2<WIDE, 4, OW, PL>(in, out, L, a, rules, st);
        case 5:
            if constexpr (KMAX >= 5) return launch_k2<WIDE, 5, OW, PL>(in, out, L, a, rules, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// The pass for buffers of seven planes above 4 GiB (fhp_stepk_wide.hip, its
// own translation unit so that the two halves compile in parallel).
hipError_t launch_stepk_wide(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                             const StepkArgs& a, uint32_t rules, hipStream_t st);
// The depth-5 pass with LDS carries and the streamed fill, for state buffers
// below 4 GiB (fhp_stepk_k5.hip, compiled with its own instruction schedule).
hipError_t launch_stepk_k5(const uint64_t* in, uint64_t* out, const Lattice& L, const StepkArgs& a,
                           uint32_t rules, hipStream_t st);
// The pass for rows of a power of two words up to 64, one wave per band
// (fhp_stepk_wave.hip).
hipError_t launch_stepk_wave(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                             const StepkArgs& a, uint32_t rules, hipStream_t st);
// The passes with the preloaded pipeline fill, for launches of at most one
// wave per SIMD (fhp_stepk_preload.hip); one_wave as for launch_stepk_wave.
hipError_t launch_stepk_preload(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                                const StepkArgs& a, uint32_t rules, bool one_wave,
                                hipStream_t st);

}  // namespace fhp
