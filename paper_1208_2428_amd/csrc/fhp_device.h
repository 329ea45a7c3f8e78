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

// FHP-II collision of 64 fluid nodes.  a[0..5] are the moving channels after
// streaming, a[6] the rest channel, chi the chirality word.  Written as flip
// masks: every rule moves the node between two states, so each output channel
// is its input XOR the OR of the rules that touch it.  Indices are mod 6 for
// channels and mod 3 for opposite pairs (pair j = channels j and j+3).
//   R1 head-on pair j alone (no other moving particle): channels j, j+3 empty
//      and the pair turned by +60 deg (chi=1) or -60 deg (chi=0) filled;
//   R2 {0,2,4} <-> {1,3,5} with no rest particle: all six moving channels flip;
//   R3 pattern (rest, c-1, c, c+1) = (1,0,1,0) or (0,1,0,1) with c+2, c+3,
//      c+4 empty: channels c-1, c, c+1 and the rest channel flip.
FHP_HD void collide(const uint64_t a[7], uint64_t chi, uint64_t o[7]) {
    const uint64_t r = a[6];
    uint64_t q[3], d[3], x[3];
    for (int j = 0; j < 3; j++) {
        q[j] = ~(a[j] | a[j + 3]);  // pair empty
        x[j] = a[j] ^ a[j + 3];     // exactly one of the pair
    }
    for (int j = 0; j < 3; j++)     // head-on pair j and nothing else moving
        d[j] = (a[j] & a[j + 3]) & q[(j + 1) % 3] & q[(j + 2) % 3];
    // R2: one particle per pair and channels 0, 2, 4 equal, no rest particle.
    const uint64_t eq024 = ~((a[0] ^ a[2]) | (a[0] ^ a[4]));
    const uint64_t tri = ~r & x[0] & x[1] & x[2] & eq024;
    // R1 flips per pair: the source pair, plus the target pair chosen by chi.
    uint64_t f1[3];
    for (int j = 0; j < 3; j++) {
        const uint64_t tgt = (chi & d[(j + 2) % 3]) | (~chi & d[(j + 1) % 3]);
        f1[j] = d[j] | tgt | tri;
    }
    // R3: g[c] marks nodes where the (c-1, c, c+1, rest) exchange applies.
    uint64_t g[6];
    for (int c = 0; c < 6; c++) {
        const int cm = (c + 5) % 6, cp = (c + 1) % 6;
        const uint64_t far_empty = ~(a[(c + 2) % 6] | a[(c + 3) % 6] | a[(c + 4) % 6]);
        g[c] = far_empty & (r ^ a[cm]) & (a[c] ^ a[cm]) & (a[c] ^ a[cp]);
    }
    uint64_t gany = 0;
    for (int c = 0; c < 6; c++) {
        o[c] = a[c] ^ f1[c % 3] ^ (g[(c + 5) % 6] | g[c] | g[(c + 1) % 6]);
        gany |= g[c];
    }
    o[6] = r ^ gany;
}

// Full per-word update after streaming: collision on fluid nodes, bounce-back
// c_i -> c_{i+3} on solid nodes (rest particle kept), then the forcing swap
// of bits 5 -> 2 on fluid nodes selected by `coin` (one bit at most).
FHP_HD void update(const uint64_t a[7], uint64_t solid, uint64_t chi, uint64_t coin,
                   uint64_t o[7]) {
    uint64_t c[7];
    collide(a, chi, c);
    for (int i = 0; i < 6; i++) o[i] = (solid & a[(i + 3) % 6]) | (~solid & c[i]);
    o[6] = (solid & a[6]) | (~solid & c[6]);
    const uint64_t m = coin & ~solid & o[5] & ~o[2];
    o[5] ^= m;
    o[2] ^= m;
}

// Forcing coin word: h = H(key_force, counter); the coin of node h>>58 is up
// when (h mod 2^32) < thr, thr = floor(f * 2^38) < 2^32.
FHP_HD uint64_t coin_word(uint64_t h, uint64_t thr) {
    return ((h & 0xffffffffull) < thr) ? (1ull << (h >> 58)) : 0ull;
}

}  // namespace fhp
