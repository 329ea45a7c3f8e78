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
    uint32_t rules = 0;      // FHP_RULES_*
};

// FHP-III's collision holds many more live values than FHP-II's; with more
// than three levels in registers the blocked kernel would spill, so passes
// of an FHP-III lattice are at most three steps deep.
constexpr uint32_t kMaxDepthFHP3 = 3;

// Workspace layout of one lattice: [buffer 0: 7 planes][buffer 1: 7 planes]
// [S plane][aux].
struct Layout {
    size_t plane_words;  // padded words per plane
    size_t buf_words;    // 7 planes
    size_t s_off, aux_off, total_bytes;
};

constexpr uint64_t kTimeLimit = 1ull << 24;  // t*2^40 must stay below 2^64
constexpr size_t kAuxWords = 512;            // reduction scratch (words)
constexpr uint32_t kMaxBlockedWords = 512;   // widest row of the blocked kernels (words)

// Error reporting: sets the calling thread's message, returns the code.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define FHP_HIP_TRY(expr, what)                                 \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return ::fhp::hip_fail(e_, what); \
    } while (0)

// Host-side fault injection for tests of the error paths, from the
// environment variable FHP_FAULT, read once per process:
//   "launch@N": single-lattice step launches after the first N fail with
//               hipErrorLaunchFailure without reaching the device;
//   "alloc":    the pinned staging buffer of batches and pools is not
//               allocated (hipErrorOutOfMemory).
// Unset or empty: no faults.  The GPU never sees an injected fault.
bool fault_launch();  // true when this launch is to fail (counts launches)
bool fault_alloc();

int validate(const fhp_params* p);
Layout layout_for(uint32_t W, uint32_t H);
uint32_t default_depth(uint32_t H, uint32_t wd, uint32_t simds);
uint32_t default_band(uint32_t H, uint32_t wd, uint32_t simds);
// Hash keys, forcing threshold and modes of the dynamics of *p.
Dyn dyn_for(const fhp_params* p);
// SIMDs of the current device (4 per compute unit).
uint32_t device_simds();

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
hipError_t launch_observe_rows(const uint64_t* planes, const Lattice& L, uint32_t row0,
                               uint32_t rows, int64_t* out, hipStream_t st);
hipError_t launch_observe_blocks(const uint64_t* planes, const Lattice& L, uint32_t b,
                                 uint32_t brow0, uint32_t brows, uint32_t bx0, uint32_t nbx,
                                 int32_t* out, hipStream_t st);
hipError_t launch_digest(const uint64_t* planes, const Lattice& L, uint64_t* acc, hipStream_t st);
hipError_t launch_step1(const uint64_t* in, uint64_t* out, const Lattice& L, const Dyn& D,
                        uint64_t t, hipStream_t st);
// K steps in one pass (fhp_stepk.hip); bands of T rows, one workgroup per band,
// on a device of `simds` SIMDs.  Needs L.wd <= kMaxBlockedWords.
hipError_t launch_stepk(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                        const Dyn& D, uint64_t t, uint32_t T, uint32_t simds, hipStream_t st);

}  // namespace fhp

// One lattice.  A standalone simulation owns no device memory (the caller owns
// the workspace); a batch member is a view into the batch workspace
// (owner != nullptr), released with the batch.
struct fhp_sim {
    fhp_params p;
    fhp::Lattice L;  // L.S is set per launch from has_mask
    fhp::Dyn D;
    fhp::Layout lay;
    uint64_t* buf[2];
    uint64_t* S;
    uint64_t* aux;
    int cur;         // buffer holding the current state
    uint64_t t;      // steps completed
    uint32_t depth;  // temporal-block depth K
    uint32_t band;   // rows per workgroup of the blocked kernel (0 = default)
    uint32_t simds;  // SIMDs of the device the simulation runs on (4 per CU)
    int has_mask;
    hipStream_t st;
    void* owner;     // batch that owns this view, or nullptr
    int* changed;    // set to 1 when the state or time is changed through this handle
};

namespace fhp {

// Fills in a simulation whose planes start at `planes` (layout `lay`) with
// reduction scratch `aux`, uploads the mask and writes the initial state.
// Synchronises the stream when `sync` is set or a mask is given; otherwise the
// initial state is only enqueued.
int sim_setup(fhp_sim* s, const fhp_params* p, uint64_t* planes, const Layout& lay,
              uint64_t* aux, hipStream_t st, bool sync = true);
Lattice lattice_of(const fhp_sim* s);

}  // namespace fhp
