// fhp_device.h -- per-word FHP arithmetic shared by the gfx950 kernels.
//
// Every function works on 64 nodes at once: bit b of a uint64 word is node
// x = 64w + b of one row, and a node's seven channels live in seven such words
// (bit-planes).  All functions are pure bit logic; they compile for the device
// and for the host (the host build is used only to check them exhaustively).
//
// Model: arXiv:1208.2428, Sec. 2 (seven channels, motion then scattering,
// bounce-back at boundary nodes, forcing by exchanging bits 2 and 5).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FHP_HD __host__ __device__ __forceinline__

namespace fhp {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kTagInit = 1, kTagChir = 2, kTagForce = 3;

// SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
FHP_HD uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Output number n+1 of SplitMix64 started from state key.
FHP_HD uint64_t hash64(uint64_t key, uint64_t n) { return mix64(key + (n + 1) * kGamma); }

// Hash counter of (t, row, 64-node word): t*2^40 + y*2^20 + w.
FHP_HD uint64_t counter(uint64_t t, uint64_t y, uint64_t w) { return (t << 40) + (y << 20) + w; }

// The same hash split into a per-word and a per-row part, so that a kernel
// forms the SplitMix64 state with one 64-bit add:
//   key + (t*2^40 + y*2^20 + w + 1)*gamma = word_base(key, w) + row_term(t, y)  (mod 2^64).
FHP_HD uint64_t word_base(uint64_t key, uint64_t w) { return key + (w + 1) * kGamma; }
FHP_HD uint64_t row_term(uint64_t t, uint64_t y) { return ((t << 40) + (y << 20)) * kGamma; }

// Three-input bit function: bit i of the result is bit (a_i b_i c_i) of the
// truth table TT, i.e. TT = f(0xF0, 0xCC, 0xAA).  One v_bitop3_b32 on gfx950.
constexpr uint32_t kA = 0xF0, kB = 0xCC, kC = 0xAA;

template <uint32_t TT>
FHP_HD uint32_t lop3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT & 0xFF);
#else
    uint32_t r = 0;
    for (uint32_t i = 0; i < 8; i++)
        if ((TT >> i) & 1) r |= ((i & 4) ? a : ~a) & ((i & 2) ? b : ~b) & ((i & 1) ? c : ~c);
    return r;
#endif
}

FHP_HD uint32_t mux3(uint32_t s, uint32_t x, uint32_t y) {  // s ? x : y
    return lop3<(kA & kB) | (~kA & kC)>(s, x, y);
}
FHP_HD uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    return lop3<(kA & kB) | (kA & kC) | (kB & kC)>(a, b, c);
}
FHP_HD uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return lop3<kA ^ kB ^ kC>(a, b, c); }
FHP_HD uint32_t or3(uint32_t a, uint32_t b, uint32_t c) { return lop3<kA | kB | kC>(a, b, c); }

// Rule sets (the values of fhp_params.rules).
constexpr int kRulesFHP2 = 0, kRulesFHP1 = 1, kRulesFHP3 = 2;

// Particle counts of the six moving channels of 32 nodes, by parity class:
// even class (0, 2, 4) count = 2 ce + se, odd class (1, 3, 5) = 2 co + so;
// total n = n0 + 2 n1 + 4 n2; pp = a head-on pair is present; eq024 =
// channels 0, 2, 4 all equal.
struct Counts {
    uint32_t se, ce, so, co, n0, n1, n2, pp, eq024;
};

FHP_HD Counts counts(const uint32_t a[7]) {
    Counts K;
    K.se = xor3(a[0], a[2], a[4]);
    K.ce = maj3(a[0], a[2], a[4]);
    K.so = xor3(a[1], a[3], a[5]);
    K.co = maj3(a[1], a[3], a[5]);
    K.n0 = K.se ^ K.so;
    const uint32_t c0 = K.se & K.so;
    K.n1 = xor3(K.ce, K.co, c0);
    K.n2 = maj3(K.ce, K.co, c0);
    uint32_t pp = a[0] & a[3];
    pp = lop3<kA | (kB & kC)>(pp, a[1], a[4]);
    K.pp = lop3<kA | (kB & kC)>(pp, a[2], a[5]);
    K.eq024 = lop3<(kA & kB & kC) | (~kA & ~kB & ~kC)>(a[0], a[2], a[4]);
    return K;
}

// Collision of 32 nodes after streaming (fluid nodes) and bounce-back (solid
// nodes), FHP-II or FHP-I.  a[0..5] moving channels, a[6] rest, s solid, chi
// chirality.
//
// Every colliding state maps each output channel j to a function of the two
// channels next to it, A = a_{j-1} and B = a_{j+1} (indices mod 6):
//   R1 head-on pair alone (rest particle a spectator): the pair turns by
//      +60 deg (chi = 1) or -60 deg (chi = 0): o_j = chi ? A : B;
//   R2 {0,2,4} <-> {1,3,5} (FHP-II: without rest particle): o_j = A (= B);
//   R3 (FHP-II only) one particle c plus rest -> {c-1, c+1}: o_j = A | B,
//      and {c-1, c+1} without rest -> c plus rest: o_j = A & B; i.e.
//      o_j = maj(rest, A, B), and the rest bit flips.
// Both forms are "A where A = B, else Z": Z = (chi XNOR A) for R1/R2 and
// Z = rest for R3.  The rule that applies comes from the number of moving
// particles: R1 = (n = 2) & (an opposite pair present); R3 = rest ? (n = 1) :
// ((n = 2) & both particles in one class, i.e. at 120 deg); R2 = (n = 3),
// channels 0, 2, 4 equal (and no rest for FHP-II).  The rule masks ignore
// the solid bit: a solid node takes the bounced channel j+3 in the last
// select whatever its rule mask says, and keeps its rest bit.
template <int RULES>
FHP_HD void collide_fhp12(const uint32_t a[7], const Counts& K, uint32_t s, uint32_t chi,
                          uint32_t o[7]) {
    const uint32_t r = a[6];
    const uint32_t is2 = lop3<~kA & kB & ~kC>(K.n0, K.n1, K.n2);
    const uint32_t is3 = K.n0 & K.n1;  // n = 7 cannot occur
    uint32_t c12, c3, zc;
    if constexpr (RULES == kRulesFHP1) {
        const uint32_t tri = is3 & K.eq024;                                   // R2
        c12 = lop3<((kA & kB) | kC) & 0xFF>(is2, K.pp, tri);                  // R1 or R2
        c3 = 0;
        zc = ~chi;
    } else {
        const uint32_t tri = lop3<kA & kB & ~kC>(is3, K.eq024, r);          // R2
        c12 = lop3<((kA & kB) | kC) & 0xFF>(is2, K.pp, tri);                  // R1 or R2
        const uint32_t is1 = lop3<kA & ~kB & ~kC>(K.n0, K.n1, K.n2);
        const uint32_t f3 = is2 & ~K.se;                                      // two at 120 deg
        c3 = lop3<(kA & kB) | (~kA & kC)>(r, is1, f3);                      // R3: r ? n = 1 : f3
        zc = lop3<(kA & ~kB) | (~kA & kC)>(c12, chi, r);                    // c12 ? ~chi : r
    }
    const uint32_t any = c12 | c3;                                          // a rule applies
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const uint32_t am = a[(j + 5) % 6], ap = a[(j + 1) % 6];
        const uint32_t z = lop3<kA ^ (kB & kC)>(zc, c12, am);             // zc ^ (c12 & A)
        const uint32_t sp = lop3<(((kA ^ kB) & kC) | (~(kA ^ kB) & kA)) & 0xFF>(am, ap, z);
        const uint32_t fl = mux3(any, sp, a[j]);                           // fluid: collide or keep
        o[j] = mux3(s, a[(j + 3) % 6], fl);                                // solid: bounce back
    }
    o[6] = lop3<kA ^ (kB & ~kC)>(r, c3, s);                               // r ^ (c3 & ~s)
}

// FHP-II collision of 32 nodes with the rule masks formed from the class
// counts alone (19 operations where counts() + collide_fhp12 take 21).  With
// e, o the particle counts of the even and odd class (se/ce, so/co their
// parity and carry bits) and x = se ^ so (the total is odd):
//   R1, a head-on pair alone: e = o = 1 and an opposite pair present;
//   R2, three in one class without rest: e, o in {0, 3} and x (e != o);
//   R3: with rest, one particle (x and no carry); without rest, two
//       particles in one class (no parity bit, exactly one carry).
// The per-channel outputs are those of collide_fhp12.
FHP_HD void collide_fhp2(const uint32_t a[7], uint32_t s, uint32_t chi, uint32_t o[7]) {
    const uint32_t r = a[6];
    const uint32_t se = xor3(a[0], a[2], a[4]), ce = maj3(a[0], a[2], a[4]);
    const uint32_t so = xor3(a[1], a[3], a[5]), co = maj3(a[1], a[3], a[5]);
    const uint32_t x = se ^ so;
    const uint32_t one = lop3<kA & ~kB & ~kC>(x, ce, co);          // one particle
    const uint32_t two_cls = lop3<~kA & ~kB & kC>(se, so, ce ^ co);  // two in one class
    const uint32_t c3 = mux3(r, one, two_cls);                       // R3
    uint32_t pp = a[0] & a[3];
    pp = lop3<kA | (kB & kC)>(pp, a[1], a[4]);
    pp = lop3<kA | (kB & kC)>(pp, a[2], a[5]);                      // an opposite pair
    const uint32_t e1o1 = lop3<kA & kB & ~kC>(se, so, ce);          // with ~co: e = o = 1
    const uint32_t r1 = lop3<kA & ~kB & kC>(e1o1, co, pp);          // R1
    const uint32_t w = lop3<kA & ~(kB ^ kC)>(x, se, ce);            // x, e in {0, 3}
    const uint32_t r2 = lop3<kA & ~(kB ^ kC)>(w, so, co);           // and o in {0, 3}
    const uint32_t c12 = lop3<kA | (kB & ~kC)>(r1, r2, r);          // R1 or R2 (no rest)
    const uint32_t zc = lop3<(kA & ~kB) | (~kA & kC)>(c12, chi, r); // c12 ? ~chi : r
    const uint32_t any = c12 | c3;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const uint32_t am = a[(j + 5) % 6], ap = a[(j + 1) % 6];
        const uint32_t z = lop3<kA ^ (kB & kC)>(zc, c12, am);
        const uint32_t sp = lop3<(((kA ^ kB) & kC) | (~(kA ^ kB) & kA)) & 0xFF>(am, ap, z);
        const uint32_t fl = mux3(any, sp, a[j]);
        o[j] = mux3(s, a[(j + 3) % 6], fl);
    }
    o[6] = lop3<kA ^ (kB & ~kC)>(r, c3, s);
}

// Collision-saturated FHP-III.  Nodes of mass >= 4 are handled through their
// complement (particle-hole duality: T(s) = ~T(~s)), so the rules below act
// on mass <= 3 only: FHP-II, plus for every spectator position j the cycle
// A_j -> B_j -> C_j -> A_j (chi = 1; reversed for chi = 0) with
//   A_j = {j, j+1, j+4}, B_j = {j, j+2, j+5}, C_j = {j+1, j+5} + rest.
// Bounce-back commutes with the complement, so solid nodes need no care.
FHP_HD void collide_fhp3(const uint32_t a[7], uint32_t s, uint32_t chi, uint32_t o[7]) {
    const Counts K0 = counts(a);
    // mass = n + rest >= 4  <=>  n >= 4, or n = 3 with a rest particle
    const uint32_t cm = lop3<(kA & kB & kC)>(K0.n0, K0.n1, a[6]) | K0.n2;
    uint32_t b[7];
#pragma unroll
    for (int c = 0; c < 7; c++) b[c] = a[c] ^ cm;
    // Counts of the complemented state from those of a: a class of three
    // channels with e particles has 3 - e after the complement, which flips
    // both bits of e (so the parity of the total is unchanged).
    Counts K;
    K.se = K0.se ^ cm;
    K.ce = K0.ce ^ cm;
    K.so = K0.so ^ cm;
    K.co = K0.co ^ cm;
    K.n0 = K0.n0;
    const uint32_t c0 = K.se & K.so;
    K.n1 = xor3(K.ce, K.co, c0);
    K.n2 = maj3(K.ce, K.co, c0);
    // head-on pairs (k, k+3) one by one: the three-cycles need them singly
    const uint32_t P0 = b[0] & b[3], P1 = b[1] & b[4], P2 = b[2] & b[5];
    K.pp = or3(P0, P1, P2);
    K.eq024 = lop3<(kA & kB & kC) | (~kA & ~kB & ~kC)>(b[0], b[2], b[4]);
    uint32_t ob[7];
    collide_fhp12<kRulesFHP2>(b, K, s, chi, ob);
    const uint32_t rb = b[6];
    const uint32_t is3 = K.n0 & K.n1;
    const uint32_t is2 = lop3<~kA & kB & ~kC>(K.n0, K.n1, K.n2);
    // three moving with a head-on pair, no rest; two at 120 deg plus rest
    const uint32_t p3 = lop3<kA & ~kB & ~kC>(is3 & K.pp, rb, s);
    const uint32_t p2 = lop3<kA & ~kB & kC>(is2, K.se, rb) & ~s;
    // A_j holds the pair (j+1, j+4) and B_j the pair (j+2, j+5), each with
    // particle j: q[k] marks the p3 nodes whose pair is (k, k+3)
    const uint32_t q[3] = {p3 & P0, p3 & P1, p3 & P2};
    // Results of the cycles, gathered per channel: channel c collects A_c,
    // A_{c-1}, A_{c+2}, B_c, B_{c-2}, B_{c+1}, C_{c-1}, C_{c+1}; the rest bit
    // every C.  A_j and B_{j+2} both add to channel j+4, so each A_j waits two
    // steps for its partner; the C_j pair up for the rest bit.
    uint32_t nw[7] = {0, 0, 0, 0, 0, 0, 0};
    uint32_t tA_hold[6] = {0, 0, 0, 0, 0, 0};
    uint32_t tC_prev = 0;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const int j1 = (j + 1) % 6, j2 = (j + 2) % 6, j5 = (j + 5) % 6;
        const uint32_t iA = q[(j + 1) % 3] & b[j];
        const uint32_t iB = q[(j + 2) % 3] & b[j];
        const uint32_t iC = lop3<kA & kB & kC>(p2, b[j1], b[j5]);
        const uint32_t tA = mux3(chi, iC, iB);  // nodes whose result is A_j = {j, j+1, j+4}
        const uint32_t tB = mux3(chi, iA, iC);  // B_j = {j, j+2, j+5}
        const uint32_t tC = mux3(chi, iB, iA);  // C_j = {j+1, j+5} + rest
        nw[j] = or3(nw[j], tA, tB);
        nw[j1] = or3(nw[j1], tA, tC);
        nw[j5] = or3(nw[j5], tB, tC);
        tA_hold[j] = tA;
        // channel j+2 = (j-2)+4: A_{j-2} with B_j (A_{j-2} of j < 2 waits for the wrap)
        if (j >= 2) nw[j2] = or3(nw[j2], tA_hold[j - 2], tB);
        else nw[j2] |= tB;
        if (j & 1) nw[6] = or3(nw[6], tC_prev, tC);
        else tC_prev = tC;
    }
    // A_4 and A_5 add to channels 2 and 3
    nw[2] |= tA_hold[4];
    nw[3] |= tA_hold[5];
    const uint32_t cyc = p3 | p2;
#pragma unroll
    for (int k = 0; k < 7; k++) o[k] = lop3<(kA & ~kB) | kC>(ob[k], cyc, nw[k]) ^ cm;
}

// Update of 32 nodes after streaming: collision (fluid) or bounce-back
// (solid) of rule set RULES, then forcing: bits 5 -> 2 where the coin is up,
// on fluid nodes with o5 set and o2 clear.  coin has at most one bit; up is
// all ones (the coin counts) or zero (it does not).
template <int RULES = kRulesFHP2>
FHP_HD void update32(const uint32_t a[7], uint32_t s, uint32_t chi, uint32_t coin, uint32_t up,
                     uint32_t o[7]) {
    if constexpr (RULES == kRulesFHP3) {
        collide_fhp3(a, s, chi, o);
    } else if constexpr (RULES == kRulesFHP2) {
        collide_fhp2(a, s, chi, o);
    } else {
        collide_fhp12<RULES>(a, counts(a), s, chi, o);
    }
    const uint32_t cf = lop3<kA & ~kB & kC>(coin, s, up);
    const uint32_t o5 = lop3<kA & ~(kB & ~kC)>(o[5], cf, o[2]);
    const uint32_t o2 = lop3<kA | (kB & kC)>(o[2], cf, o[5]);
    o[5] = o5;
    o[2] = o2;
}

// 64-node version: the two 32-bit halves independently.
template <int RULES = kRulesFHP2>
FHP_HD void update(const uint64_t a[7], uint64_t solid, uint64_t chi, uint64_t coin, uint32_t up,
                   uint64_t o[7]) {
    uint32_t lo[7], hi[7], olo[7], ohi[7];
    for (int c = 0; c < 7; c++) {
        lo[c] = (uint32_t)a[c];
        hi[c] = (uint32_t)(a[c] >> 32);
    }
    update32<RULES>(lo, (uint32_t)solid, (uint32_t)chi, (uint32_t)coin, up, olo);
#if defined(__HIP_DEVICE_COMPILE__)
    // The halves are independent; interleaving them buys no speed on a
    // wave-serial SIMD but nearly doubles the live values (FHP-II at depth 4:
    // 243 VGPRs interleaved, 188 apart).  An empty asm that makes the high
    // inputs depend on the low result keeps them apart.
#pragma unroll
    for (int c = 0; c < 7; c++) asm volatile("" : "+v"(hi[c]) : "v"(olo[c]));
#endif
    update32<RULES>(hi, (uint32_t)(solid >> 32), (uint32_t)(chi >> 32), (uint32_t)(coin >> 32), up,
                    ohi);
    for (int c = 0; c < 7; c++) o[c] = ((uint64_t)ohi[c] << 32) | olo[c];
}

// The same with a coin word that is up wherever it has a bit.
template <int RULES = kRulesFHP2>
FHP_HD void update(const uint64_t a[7], uint64_t solid, uint64_t chi, uint64_t coin, uint64_t o[7]) {
    update<RULES>(a, solid, chi, coin, ~0u, o);
}

// Forcing coin of one 64-node word, h = H(key_force, counter): the coin of
// node h>>58 is up when (h mod 2^32) < thr, thr = floor(f * 2^38) < 2^32.
// The blocked kernels keep it as that node's bit (coin_bit) and a mask that
// is all ones when the coin is up (coin_up); the forcing step folds the mask
// into a bit function it evaluates anyway.
FHP_HD uint64_t coin_bit(uint64_t h) { return 1ull << (h >> 58); }
FHP_HD uint32_t coin_up(uint64_t h, uint64_t thr) { return ((uint32_t)h < (uint32_t)thr) ? ~0u : 0u; }
FHP_HD uint64_t coin_word(uint64_t h, uint64_t thr) { return coin_up(h, thr) ? coin_bit(h) : 0ull; }

// Chirality word of a chirality mode: (h & m_and) | m_or on each 32-bit half
// (m_and, m_or are all ones or all zeros).  With m_and in a vector register
// each half is one three-input bit function.
FHP_HD uint64_t chir_word(uint64_t h, uint32_t m_and, uint32_t m_or) {
    const uint32_t lo = lop3<(kA & kB) | kC>((uint32_t)h, m_and, m_or);
    const uint32_t hi = lop3<(kA & kB) | kC>((uint32_t)(h >> 32), m_and, m_or);
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace fhp
