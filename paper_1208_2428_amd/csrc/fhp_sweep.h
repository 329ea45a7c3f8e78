// fhp_sweep.h -- pieces shared by the temporally blocked kernels (one lattice,
// and many lattices in one persistent launch): a row of one level held by one
// thread, the horizontal carry exchange, and the pull streaming of one level.
//
// Streaming (arXiv:1208.2428, Sec. 2, motion step; odd rows shifted by +1/2,
// c_i at (i-2)*60 degrees): the particle arriving with velocity c_i comes from
// the neighbour at -c_i.  rotl1 (towards larger x) takes the bit of node x-1,
// rotr1 takes node x+1:
//   c2 (E):  row y,   rotl1            c5 (W):  row y,   rotr1
//   c3 (NE): row y-1, rotl1 if y even  c4 (NW): row y-1, rotr1 if y odd
//   c0 (SW): row y+1, rotr1 if y odd   c1 (SE): row y+1, rotl1 if y even
#pragma once

#include <type_traits>

#include "fhp_device.h"

namespace fhp {

// One row of one level, as seen by one thread (one 64-node word).
struct Row {
    uint64_t p[7];  // planes
    uint64_t s;     // solid word (obstacles + wall rows)
    uint32_t c;     // carry-in bits: bit 0..2 = bit 63 of the left word's planes 1, 2, 3;
                    // bit 8..10 = bit 0 of the right word's planes 0, 4, 5
};

__device__ __forceinline__ uint64_t rotl1(uint64_t v, uint32_t cin) { return (v << 1) | cin; }
__device__ __forceinline__ uint64_t rotr1(uint64_t v, uint32_t cin) {
    return (v >> 1) | ((uint64_t)cin << 63);
}

// Calls f(integral_constant<int, I>) for I = L .. N.
template <int L, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (L <= N) {
        f(std::integral_constant<int, L>{});
        static_for<L + 1, N>(f);
    }
}

// Workgroup barrier that orders LDS traffic only: global loads issued for the
// next row stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The bits a row's word gives to its neighbours: bit 63 of planes 1, 2, 3
// (sources of rotl1 for the word on its right) and bit 0 of planes 0, 4, 5
// (sources of rotr1 for the word on its left).
__device__ __forceinline__ uint32_t carry_out(const Row& x) {
    return (uint32_t)(x.p[1] >> 63) | ((uint32_t)(x.p[2] >> 63) << 1) |
           ((uint32_t)(x.p[3] >> 63) << 2) | ((uint32_t)(x.p[0] & 1) << 8) |
           ((uint32_t)(x.p[4] & 1) << 9) | ((uint32_t)(x.p[5] & 1) << 10);
}

// Publishes x's carry bits in LDS slot `slot`, synchronises the workgroup and
// gathers the carry-in bits from the words at lanes wl (left) and wr (right).
__device__ __forceinline__ void exchange(uint32_t* xch, uint32_t& slot, uint32_t nt,
                                         uint32_t lane, uint32_t wl, uint32_t wr, Row& x) {
    uint32_t* buf = xch + slot * nt;
    buf[lane] = carry_out(x);
    lds_barrier();
    x.c = (buf[wl] & 0x7u) | (buf[wr] & 0x700u);
    slot ^= 1;
}

// Pull streaming of one destination row of parity ODD from the level below:
// rows rho-1 (planes 3, 4 and carries ac), rho (bp, carries bc) and rho+1 (x).
template <bool ODD>
__device__ __forceinline__ void stream_in(uint64_t a3, uint64_t a4, uint32_t ac, const uint64_t* bp,
                                          uint32_t bc, const Row& x, uint64_t n[7]) {
    if (ODD) {
        n[3] = a3;
        n[4] = rotr1(a4, (ac >> 9) & 1);
        n[0] = rotr1(x.p[0], (x.c >> 8) & 1);
        n[1] = x.p[1];
    } else {
        n[3] = rotl1(a3, (ac >> 2) & 1);
        n[4] = a4;
        n[0] = x.p[0];
        n[1] = rotl1(x.p[1], x.c & 1);
    }
    n[2] = rotl1(bp[2], (bc >> 1) & 1);
    n[5] = rotr1(bp[5], (bc >> 10) & 1);
    n[6] = bp[6];
}

}  // namespace fhp
