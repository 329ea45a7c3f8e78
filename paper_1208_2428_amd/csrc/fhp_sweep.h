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

// One row of one level, as seen by one thread (one 64-node word).  A 1-node
// shift of a word needs one bit of a neighbouring word: bit 63 of the left
// word for rotl1 (its high half, whose bit 31 is that bit), bit 0 of the right
// word for rotr1 (its low half).  Over its life a row of parity P is rotated
// in four planes:
//   as the row below its destination (dest y = row - 1): plane 0 (rotr1) if
//       the row is even, plane 1 (rotl1) if odd;
//   as the destination row: planes 2 (rotl1) and 5 (rotr1);
//   as the row above (dest y = row + 1): plane 4 (rotr1) if even, plane 3
//       (rotl1) if odd.
// c[0..3] hold the neighbour halves for these four uses, in this order.
struct Row {
    uint64_t p[7];  // planes
    uint64_t s;     // solid word (obstacles + wall rows)
    uint32_t c[4];  // neighbour halves: as row below, planes 2 and 5, as row above
};

__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }

// v shifted one node towards larger x; left_hi = high half of the left word.
__device__ __forceinline__ uint64_t rotl1(uint64_t v, uint32_t left_hi) {
    const uint32_t lo = __builtin_amdgcn_alignbit(lo32(v), left_hi, 31);
    const uint32_t hi = __builtin_amdgcn_alignbit(hi32(v), lo32(v), 31);
    return ((uint64_t)hi << 32) | lo;
}
// v shifted one node towards smaller x; right_lo = low half of the right word.
__device__ __forceinline__ uint64_t rotr1(uint64_t v, uint32_t right_lo) {
    const uint32_t lo = __builtin_amdgcn_alignbit(hi32(v), lo32(v), 1);
    const uint32_t hi = __builtin_amdgcn_alignbit(right_lo, hi32(v), 1);
    return ((uint64_t)hi << 32) | lo;
}

// Calls f(integral_constant<int, I>) for I = L .. N.
template <int L, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (L <= N) {
        f(std::integral_constant<int, L>{});
        static_for<L + 1, N>(f);
    }
}

// Pins a wave-uniform 64-bit value in scalar registers.  Left alone, the
// compiler folds the row term's multiply into a vector multiply-add with the
// per-word hash base (two vector instructions per hash instead of one add).
__device__ __forceinline__ uint64_t in_sgprs(uint64_t v) {
    asm("" : "+s"(v));
    return v;
}

// A region of num_bytes bytes at p as a buffer resource (gfx9 layout, 32-bit
// data format).  Accesses take a 32-bit byte offset in a vector register and
// one in a scalar register; the hardware returns zero for loads and drops
// stores beyond num_bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t region_rsrc(const void* p, uint32_t num_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)num_bytes, 0x00020000);
}
__device__ __forceinline__ uint64_t buf_load64(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0);
    return ((uint64_t)v[1] << 32) | v[0];
}
// Stores of a pass's output rows carry the non-temporal hint (nt): the rows
// are not read again in this launch, and streaming them out instead of
// keeping them dirty in the L2 made the 16384^2 pass 3.4% faster and the
// pass-shaped copy 1.44x faster.
constexpr int kStoreNT = 2;  // cache-policy bits of a buffer store: nt
__device__ __forceinline__ void buf_store64(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff,
                                            uint64_t x) {
    __attribute__((ext_vector_type(2))) uint32_t v;
    v[0] = (uint32_t)x;
    v[1] = (uint32_t)(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, (int)soff, kStoreNT);
}

// The seven planes of one state buffer (plane stride ps words, planes of
// plane_bytes bytes), accessed by plane and by the byte offset of a word
// within its plane.  An access is then a buffer resource in scalar registers
// plus that 32-bit offset; with plain pointers the compiler forms a 64-bit
// vector address per plane and row.  WIDE = false: the whole buffer is below
// 4 GiB, one resource, and the plane is a scalar offset.  WIDE = true: one
// resource per plane (every plane is below 4 GiB).
template <bool WIDE>
struct Planes;

template <>
struct Planes<false> {
    __amdgpu_buffer_rsrc_t r;
    uint32_t ps8;
    __device__ __forceinline__ Planes(const uint64_t* base, uint64_t ps, uint32_t) {
        r = region_rsrc(base, (uint32_t)(7 * ps * 8));
        ps8 = (uint32_t)(ps * 8);
    }
    __device__ __forceinline__ uint64_t load(int c, uint32_t off) const { return buf_load64(r, off, c * ps8); }
    __device__ __forceinline__ void store(int c, uint32_t off, uint64_t x) const {
        buf_store64(r, off, c * ps8, x);
    }
};

template <>
struct Planes<true> {
    __amdgpu_buffer_rsrc_t r[7];
    __device__ __forceinline__ Planes(const uint64_t* base, uint64_t ps, uint32_t plane_bytes) {
#pragma unroll
        for (int c = 0; c < 7; c++) r[c] = region_rsrc(base + c * ps, plane_bytes);
    }
    __device__ __forceinline__ uint64_t load(int c, uint32_t off) const { return buf_load64(r[c], off, 0); }
    __device__ __forceinline__ void store(int c, uint32_t off, uint64_t x) const {
        buf_store64(r[c], off, 0, x);
    }
};

// True when a buffer of seven planes of stride ps words needs a resource per
// plane.
inline bool planes_wide(uint64_t ps) { return 7 * ps * 8 > 0xffffffffull; }

// Workgroup barrier that orders LDS traffic only: global loads issued for the
// next row stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The carry exchange lives in LDS as two slots of four 32-bit arrays (one per
// published half) of `stride` entries each: a lane's four halves are 4-byte
// words `stride` apart, so that lanes reading consecutive neighbours hit
// consecutive banks (16-byte entries per lane made every read a 4-way bank
// conflict).

// Publishes the halves of x that the neighbouring words will need (for a row
// of parity ODD) in LDS slot `slot`.
template <bool ODD>
__device__ __forceinline__ void publish(uint32_t* xch, uint32_t slot, uint32_t stride, uint32_t lane,
                                        const Row& x) {
    uint32_t* buf = xch + slot * 4 * stride + lane;
    buf[0] = ODD ? hi32(x.p[1]) : lo32(x.p[0]);
    buf[stride] = hi32(x.p[2]);
    buf[2 * stride] = lo32(x.p[5]);
    buf[3 * stride] = ODD ? hi32(x.p[3]) : lo32(x.p[4]);
}

// Synchronises the workgroup and gathers x's neighbour halves from what the
// words at lanes wl (left) and wr (right) published; the next exchange uses
// the other slot.
template <bool ODD>
__device__ __forceinline__ void gather(const uint32_t* xch, uint32_t& slot, uint32_t stride, uint32_t wl,
                                       uint32_t wr, Row& x) {
    const uint32_t* buf = xch + slot * 4 * stride;
    lds_barrier();
    const uint32_t n = ODD ? wl : wr;  // the side planes 0/1 and 3/4 shift in from
    x.c[0] = buf[n];
    x.c[1] = buf[stride + wl];
    x.c[2] = buf[2 * stride + wr];
    x.c[3] = buf[3 * stride + n];
    slot ^= 1;
}

// Rows held by a single wave (64 words, lane = word, or fewer words repeated
// across the wave): the neighbour halves come from the adjacent lanes through
// DPP wave rotations, with no LDS and no barrier.  wave_ror:1 hands each lane
// the value of the lane below it (lane 0 gets lane 63's: the periodic wrap of
// the row), wave_rol:1 the value of the lane above it.
__device__ __forceinline__ uint32_t from_left_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13C, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t from_right_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x134, 0xf, 0xf, false);
}

// gather() for a row held by one wave.
template <bool ODD>
__device__ __forceinline__ void gather_wave(Row& x) {
    x.c[0] = ODD ? from_left_lane(hi32(x.p[1])) : from_right_lane(lo32(x.p[0]));
    x.c[1] = from_left_lane(hi32(x.p[2]));
    x.c[2] = from_right_lane(lo32(x.p[5]));
    x.c[3] = ODD ? from_left_lane(hi32(x.p[3])) : from_right_lane(lo32(x.p[4]));
}

template <bool ODD>
__device__ __forceinline__ void exchange(uint32_t* xch, uint32_t& slot, uint32_t stride, uint32_t lane,
                                         uint32_t wl, uint32_t wr, Row& x) {
    publish<ODD>(xch, slot, stride, lane, x);
    gather<ODD>(xch, slot, stride, wl, wr, x);
}

// Pull streaming of one destination row of parity ODD from the level below:
// rows y-1 (planes 3, 4 and its neighbour half as the row above, ac), y (bp,
// neighbour halves of planes 2 and 5, b2 and b5) and y+1 (x).
template <bool ODD>
__device__ __forceinline__ void stream_in(uint64_t a3, uint64_t a4, uint32_t ac, const uint64_t* bp,
                                          uint32_t b2, uint32_t b5, const Row& x, uint64_t n[7]) {
    if (ODD) {  // row y-1 even, row y+1 even
        n[3] = a3;
        n[4] = rotr1(a4, ac);
        n[0] = rotr1(x.p[0], x.c[0]);
        n[1] = x.p[1];
    } else {  // row y-1 odd, row y+1 odd
        n[3] = rotl1(a3, ac);
        n[4] = a4;
        n[0] = x.p[0];
        n[1] = rotl1(x.p[1], x.c[0]);
    }
    n[2] = rotl1(bp[2], b2);
    n[5] = rotr1(bp[5], b5);
    n[6] = bp[6];
}

}  // namespace fhp
