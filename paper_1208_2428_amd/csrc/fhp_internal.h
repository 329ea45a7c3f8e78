// fhp_internal.h -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fhp.h"

namespace fhp {

// Geometry and buffers of one lattice on the device.
//   planes: 7 bit-planes, plane c at planes + c*ps, word (y, w) at y*wd + w.
struct Lattice {
    uint32_t W = 0, H = 0, wd = 0;  // width in nodes, height, words per row (W/64)
    size_t ps = 0;                  // plane stride in words (>= H*wd, 256-byte multiple)
    uint32_t walls = 0;             // rows 0 and H-1 solid
    const uint64_t* S = nullptr;    // obstacle plane (H*wd words); nullptr = none
};

// Per-simulation constants of the dynamics.
struct Dyn {
    uint64_t key_chir = 0, key_force = 0;
    uint64_t thr_force = 0;  // floor(f * 2^38)
    uint32_t chir_mode = 0;  // FHP_CHIR_*
};

// Kernel launchers (fhp_kernels.hip).  All enqueue on `st` and return the HIP
// launch status.
hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t st);
hipError_t launch_pack(const uint8_t* bytes, uint32_t row0, uint32_t rows, const Lattice& L,
                       uint64_t* planes, uint64_t* S, int mask_only, hipStream_t st);
hipError_t launch_unpack(const uint64_t* planes, const Lattice& L, uint32_t row0, uint32_t rows,
                         uint8_t* bytes, hipStream_t st);
hipError_t launch_init(uint64_t* planes, const Lattice& L, uint64_t key_init, uint64_t thr_fill,
                       hipStream_t st);
hipError_t launch_or_reduce(const uint64_t* p, size_t n, uint64_t* acc, hipStream_t st);
hipError_t launch_observe_global(const uint64_t* planes, const Lattice& L, uint64_t* acc,
                                 hipStream_t st);
hipError_t launch_observe_blocks(const uint64_t* planes, const Lattice& L, uint32_t b,
                                 uint32_t brow0, uint32_t brows, int32_t* out, hipStream_t st);
hipError_t launch_digest(const uint64_t* planes, const Lattice& L, uint64_t* acc, hipStream_t st);
hipError_t launch_step1(const uint64_t* in, uint64_t* out, const Lattice& L, const Dyn& D,
                        uint64_t t, hipStream_t st);
// K steps in one pass (fhp_stepk.hip); bands of T rows, one workgroup per band.
// Needs L.wd <= kMaxBlockedWords.
hipError_t launch_stepk(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                        const Dyn& D, uint64_t t, uint32_t T, hipStream_t st);
constexpr uint32_t kMaxBlockedWords = 512;

}  // namespace fhp
