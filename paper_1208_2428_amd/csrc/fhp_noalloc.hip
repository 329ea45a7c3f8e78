// fhp_noalloc.hip -- fhp_step_noalloc: the time step of fhp_step for callers
// that cannot allocate device memory (declared in include/fhp.h).
//
// The state lives in the caller's two plane buffers (input and output); the
// only other memory a run of several passes needs, the buffer between passes,
// is the file-scope device array `scratch` below.  Nothing here allocates:
// the array's device address is looked up once per device and every call on
// that device uses that same array.
#include <mutex>

#include "fhp_internal.h"

namespace fhp {
namespace {

constexpr size_t kScratchBytes = FHP_NOALLOC_MAX_STATE_BYTES;
constexpr int kMaxDevices = 64;

// Intermediate state between passes (one buffer of seven planes).  Every
// device the library runs on holds its own copy until the process ends.
static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch`, per device

// Device address of this device's `scratch` (looked up on the device's first
// call, with the device current).  In host code the array's name is only a
// stand-in for the symbol, never an address a kernel may use.
int scratch_ptr(uint64_t** out) {
    int dev = 0;
    FHP_HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FHP_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        FHP_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FHP_E_DEVICE, "scratch has no device address");
        g_scratch[dev] = p;
    }
    *out = (uint64_t*)g_scratch[dev];
    return FHP_OK;
}

bool overlap(const void* a, const void* b, size_t n) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + n && y < x + n;
}

}  // namespace
}  // namespace fhp

using namespace fhp;

extern "C" int fhp_step_noalloc(const fhp_params* p, const uint64_t* dev_in, uint64_t* dev_out,
                                const uint64_t* dev_solid, uint64_t t, uint64_t n, uint32_t depth,
                                void* hip_stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (p->solid)
        return fail(FHP_E_INVAL, "params.solid must be NULL: obstacles come as a device plane");
    if (!dev_in || !dev_out || ((uintptr_t)dev_in & 255) || ((uintptr_t)dev_out & 255) ||
        ((uintptr_t)dev_solid & 7))
        return fail(FHP_E_INVAL, "state buffers must be non-NULL 256-byte aligned device pointers");
    const uint32_t wd = p->width / 64;
    const size_t plane_words = (size_t)p->height * wd;
    const size_t state_bytes = 7 * plane_words * sizeof(uint64_t);
    if (state_bytes > kScratchBytes)
        return fail(FHP_E_NOMEM, "state of %zu bytes (%u x %u): fhp_step_noalloc takes at most %zu",
                    state_bytes, p->width, p->height, kScratchBytes);
    if (overlap(dev_in, dev_out, state_bytes))
        return fail(FHP_E_INVAL, "input and output state buffers overlap");
    if (depth > FHP_MAX_DEPTH) return fail(FHP_E_INVAL, "depth %u above %u", depth, FHP_MAX_DEPTH);
    if (depth > 1 && wd > kMaxBlockedWords)
        return fail(FHP_E_INVAL, "depth %u needs width <= %u", depth, 64 * kMaxBlockedWords);
    if (t >= kTimeLimit || n >= kTimeLimit || t + n >= kTimeLimit)
        return fail(FHP_E_STATE, "time %llu + %llu would reach 2^24", (unsigned long long)t,
                    (unsigned long long)n);
    uint64_t* mid = nullptr;
    rc = scratch_ptr(&mid);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    if (n == 0) {
        FHP_HIP_TRY(hipMemcpyAsync(dev_out, dev_in, state_bytes, hipMemcpyDeviceToDevice, st),
                    "copy");
        return FHP_OK;
    }

    Lattice L;
    L.W = p->width;
    L.H = p->height;
    L.wd = wd;
    L.ps = plane_words;
    L.walls = p->walls == FHP_WALLS_CHANNEL;
    L.S = dev_solid;
    const Dyn D = dyn_for(p);
    const uint32_t simds = device_simds();
    uint32_t K = depth ? depth : default_depth(L.H, wd, simds);
    if (D.rules == FHP_RULES_FHP3 && K > kMaxDepthFHP3) K = kMaxDepthFHP3;
    const uint32_t T = default_band(L.H, wd, simds);
    // Passes of K steps (the last one shorter), alternating between dev_out
    // and the scratch buffer so that the last pass writes dev_out.
    uint64_t passes = (n + K - 1) / K;
    const uint64_t* src = dev_in;
    while (n > 0) {
        const uint32_t k = n >= K ? K : (uint32_t)n;
        uint64_t* dst = (passes % 2 == 1) ? dev_out : mid;
        if (k == 1)
            FHP_HIP_TRY(launch_step1(src, dst, L, D, t, st), "step");
        else
            FHP_HIP_TRY(launch_stepk(k, src, dst, L, D, t, T, simds, st), "step");
        src = dst;
        t += k;
        n -= k;
        passes--;
    }
    return FHP_OK;
}
