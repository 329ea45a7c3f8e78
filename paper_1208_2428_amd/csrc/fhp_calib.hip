// fhp_calib.hip -- streaming reference kernels (include/fhp_calib.h).
//
// k_calib_pass makes the memory accesses of one blocked pass of the step
// kernel and nothing else: a workgroup per band of rows, one thread per 64-bit
// word of the full row width, the rows of the band (plus `halo` rows above and
// below) swept top to bottom with the next row's loads issued before the
// current row is used, seven planes through one buffer resource, the obstacle
// plane through another, and the band's own rows of seven planes stored.  Its
// bandwidth is therefore what a pass of that shape reaches when the
// arithmetic costs nothing.  k_calib_flat streams a flat buffer in 16-byte
// pieces per thread: the device's plain streaming bandwidth.
#include "../../include/fhp_calib.h"
#include "fhp_internal.h"
#include "fhp_sweep.h"

namespace fhp {
namespace {

struct CalibArgs {
    uint32_t wd, H, T, halo;
    uint64_t ps;
};

template <int MODE, bool MASK>
__global__ void __launch_bounds__(512) k_calib_pass(const uint64_t* __restrict__ in,
                                                     uint64_t* __restrict__ out,
                                                     const uint64_t* __restrict__ S, CalibArgs a) {
    const uint32_t lane = threadIdx.x;
    const bool valid = lane < a.wd;
    const uint32_t w = valid ? lane : 0;
    const uint32_t H = a.H;
    const uint32_t y0 = blockIdx.x * a.T;
    const uint32_t rows = min(a.T, H - y0);
    const int halo = (int)a.halo;
    const int n_iter = (int)rows + 2 * halo;
    const uint32_t plane_bytes = H * a.wd * 8u;
    const Planes<false> pin(in, a.ps, plane_bytes), pout(out, a.ps, plane_bytes);
    const __amdgpu_buffer_rsrc_t rs = region_rsrc(S, plane_bytes);
    auto wrap_row = [&](int r) -> uint32_t {
        int m = r % (int)H;
        return (uint32_t)(m < 0 ? m + (int)H : m);
    };
    auto offset = [&](uint32_t y) -> uint32_t { return (y * a.wd + w) * 8u; };

    if constexpr (MODE == FHP_CALIB_WRITE) {
        for (uint32_t i = 0; i < rows; i++) {
            const uint32_t off = offset(y0 + i);
            if (valid) {
#pragma unroll
                for (int c = 0; c < 7; c++) pout.store(c, off, (uint64_t)(off + c));
            }
        }
        return;
    } else {
        uint64_t nxt[8], cur[8];
        auto load = [&](uint32_t y, uint64_t* x) {
            const uint32_t off = offset(y);
#pragma unroll
            for (int c = 0; c < 7; c++) x[c] = pin.load(c, off);
            x[7] = MASK ? buf_load64(rs, off, 0) : 0;
        };
        uint64_t acc = 0;
        load(wrap_row((int)y0 - halo), nxt);
        for (int i = 0; i < n_iter; i++) {
#pragma unroll
            for (int c = 0; c < 8; c++) cur[c] = nxt[c];
            const int r = (int)y0 - halo + i;
            if (i + 1 < n_iter) load(wrap_row(r + 1), nxt);
            if constexpr (MODE == FHP_CALIB_COPY) {
                if (valid && i >= halo && i < halo + (int)rows) {
                    const uint32_t off = offset((uint32_t)r);
#pragma unroll
                    for (int c = 0; c < 7; c++) pout.store(c, off, cur[c] ^ cur[7]);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 8; c++) acc ^= cur[c];
            }
        }
        if constexpr (MODE == FHP_CALIB_READ) {
            if (valid) out[(size_t)blockIdx.x * a.wd + w] = acc;
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_calib_flat(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (MODE == FHP_CALIB_WRITE) {
        const uint4 v = make_uint4((uint32_t)gid, 1u, 2u, 3u);
        for (size_t i = gid; i < n; i += stride) dst[i] = v;
    } else {
        uint4 acc = make_uint4(0, 0, 0, 0);
        size_t i = gid;
        // four 16-byte loads in flight per thread
        for (; i + 3 * stride < n; i += 4 * stride) {
            uint4 v[4];
#pragma unroll
            for (int k = 0; k < 4; k++) v[k] = src[i + k * stride];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                if constexpr (MODE == FHP_CALIB_COPY) {
                    dst[i + k * stride] = v[k];
                } else {
                    acc.x ^= v[k].x;
                    acc.y ^= v[k].y;
                    acc.z ^= v[k].z;
                    acc.w ^= v[k].w;
                }
            }
        }
        for (; i < n; i += stride) {
            const uint4 v = src[i];
            if constexpr (MODE == FHP_CALIB_COPY) {
                dst[i] = v;
            } else {
                acc.x ^= v.x;
                acc.y ^= v.y;
                acc.z ^= v.z;
                acc.w ^= v.w;
            }
        }
        if constexpr (MODE == FHP_CALIB_READ) dst[gid] = acc;
    }
}

template <int MODE>
hipError_t launch_pass(const uint64_t* in, uint64_t* out, const uint64_t* S, const CalibArgs& a,
                       hipStream_t st) {
    const uint32_t nt = (a.wd + 63) / 64 * 64;
    const uint32_t bands = (a.H + a.T - 1) / a.T;
    if (S)
        hipLaunchKernelGGL((k_calib_pass<MODE, true>), dim3(bands), dim3(nt), 0, st, in, out, S, a);
    else
        hipLaunchKernelGGL((k_calib_pass<MODE, false>), dim3(bands), dim3(nt), 0, st, in, out, S, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace fhp

using namespace fhp;

extern "C" int fhp_calib_pass(int mode, const uint64_t* in, uint64_t* out, const uint64_t* mask,
                              uint32_t wd, uint32_t H, uint64_t plane_stride, uint32_t band,
                              uint32_t halo, void* hip_stream) {
    if (mode < FHP_CALIB_COPY || mode > FHP_CALIB_WRITE) return fail(FHP_E_INVAL, "calib mode %d unknown", mode);
    if (wd == 0 || wd > kMaxBlockedWords) return fail(FHP_E_INVAL, "wd %u outside 1..%u", wd, kMaxBlockedWords);
    if (H == 0 || band == 0) return fail(FHP_E_INVAL, "H and band must be positive");
    if (halo > 8 || halo > H) return fail(FHP_E_INVAL, "halo %u outside 0..min(8, H)", halo);
    if (plane_stride < (uint64_t)H * wd) return fail(FHP_E_INVAL, "plane stride below H * wd");
    if (7 * plane_stride * 8 > 0xffffffffull) return fail(FHP_E_INVAL, "seven planes reach 4 GiB");
    if (!out || (mode != FHP_CALIB_WRITE && !in)) return fail(FHP_E_INVAL, "NULL buffer");
    if (mode == FHP_CALIB_READ && (uint64_t)((H + band - 1) / band) * wd > 7 * plane_stride)
        return fail(FHP_E_INVAL, "output too small for the per-thread words");
    CalibArgs a{wd, H, band, halo, plane_stride};
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    const uint64_t* S = (mode == FHP_CALIB_WRITE) ? nullptr : mask;
    switch (mode) {
        case FHP_CALIB_COPY: e = launch_pass<FHP_CALIB_COPY>(in, out, S, a, st); break;
        case FHP_CALIB_READ: e = launch_pass<FHP_CALIB_READ>(in, out, S, a, st); break;
        default: e = launch_pass<FHP_CALIB_WRITE>(in, out, S, a, st); break;
    }
    return e == hipSuccess ? FHP_OK : hip_fail(e, "calib pass launch");
}

extern "C" int fhp_calib_flat(int mode, const void* src, void* dst, size_t bytes, uint32_t blocks,
                              uint32_t* blocks_used, void* hip_stream) {
    if (mode < FHP_CALIB_COPY || mode > FHP_CALIB_WRITE) return fail(FHP_E_INVAL, "calib mode %d unknown", mode);
    if (bytes == 0 || bytes % 16) return fail(FHP_E_INVAL, "bytes must be a positive multiple of 16");
    if (!dst || (mode != FHP_CALIB_WRITE && !src)) return fail(FHP_E_INVAL, "NULL buffer");
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(FHP_E_INVAL, "buffers must be 16-byte aligned");
    if (blocks == 0) blocks = device_simds() * 2;  // 8 workgroups of 256 threads per CU
    if (blocks_used) *blocks_used = blocks;
    const size_t n = bytes / 16;
    hipStream_t st = (hipStream_t)hip_stream;
    const uint4* s = (const uint4*)src;
    uint4* d = (uint4*)dst;
    switch (mode) {
        case FHP_CALIB_COPY: hipLaunchKernelGGL(k_calib_flat<FHP_CALIB_COPY>, dim3(blocks), dim3(256), 0, st, s, d, n); break;
        case FHP_CALIB_READ: hipLaunchKernelGGL(k_calib_flat<FHP_CALIB_READ>, dim3(blocks), dim3(256), 0, st, s, d, n); break;
        default: hipLaunchKernelGGL(k_calib_flat<FHP_CALIB_WRITE>, dim3(blocks), dim3(256), 0, st, s, d, n); break;
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FHP_OK : hip_fail(e, "calib flat launch");
}
