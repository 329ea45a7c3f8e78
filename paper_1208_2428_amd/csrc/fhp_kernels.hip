// fhp_kernels.hip -- gfx950 kernels of the FHP library: layout conversion,
// initial state, observables and the one-step (k = 1) update.
//
// Layout: 7 bit-planes of uint64 words per buffer; bit b of word (y, w) is
// node x = 64w + b of row y (arXiv:1208.2428, Sec. 2 stores one byte per node;
// here channel c of 64 nodes is one word, so one 64-bit logic op updates 64
// nodes).  The obstacle plane S has the same shape; wall rows are computed from
// y and never stored.
#include "fhp_device.h"
#include "fhp_internal.h"

namespace fhp {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t solid_word(const Lattice& L, uint32_t y, size_t idx) {
    uint64_t s = L.S ? L.S[idx] : 0ull;
    if (L.walls && (y == 0 || y == L.H - 1)) s = ~0ull;
    return s;
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(uint64_t* p, size_t n, uint64_t v) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// bytes -> bit-planes.  One wave per 64-node word: lane b reads node 64w+b and
// a wave ballot gathers bit c of the 64 nodes into plane c's word.
// mask_only: every nonzero byte is an obstacle (S only).  Otherwise bits 0-6
// go to the 7 planes and bit 7 to S.
__global__ void __launch_bounds__(kBlock) k_pack(const uint8_t* __restrict__ bytes, uint32_t row0,
                                                 uint32_t rows, Lattice L,
                                                 uint64_t* __restrict__ planes,
                                                 uint64_t* __restrict__ S, int mask_only) {
    const uint32_t lane = threadIdx.x & 63;
    const size_t word = ((size_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (word >= (size_t)rows * L.wd) return;  // whole wave exits together
    const uint32_t ry = (uint32_t)(word / L.wd), w = (uint32_t)(word % L.wd);
    const uint8_t v = bytes[(size_t)ry * L.W + 64u * w + lane];
    const size_t idx = (size_t)(row0 + ry) * L.wd + w;
    if (mask_only) {
        const uint64_t m = __ballot(v != 0);
        if (lane == 0) S[idx] = m;
        return;
    }
    uint64_t words[8];
#pragma unroll
    for (int c = 0; c < 8; c++) words[c] = __ballot((v >> c) & 1);
    if (lane < 7) planes[(size_t)lane * L.ps + idx] = words[lane];
    if (lane == 7) S[idx] = words[7];
}

// bit-planes -> bytes (bit 7 = obstacle or wall row).
__global__ void __launch_bounds__(kBlock) k_unpack(const uint64_t* __restrict__ planes, Lattice L,
                                                   uint32_t row0, uint32_t rows,
                                                   uint8_t* __restrict__ bytes) {
    const uint32_t lane = threadIdx.x & 63;
    const size_t word = ((size_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    if (word >= (size_t)rows * L.wd) return;
    const uint32_t ry = (uint32_t)(word / L.wd), w = (uint32_t)(word % L.wd);
    const uint32_t y = row0 + ry;
    const size_t idx = (size_t)y * L.wd + w;
    uint32_t v = 0;
#pragma unroll
    for (int c = 0; c < 7; c++) v |= (uint32_t)((planes[(size_t)c * L.ps + idx] >> lane) & 1) << c;
    v |= (uint32_t)((solid_word(L, y, idx) >> lane) & 1) << 7;
    bytes[(size_t)ry * L.W + 64u * w + lane] = (uint8_t)v;
}

// Initial state: fluid node bit c set iff
// (H(key_init, c*2^40 + y*2^20 + x) >> 32) < thr_fill; solid nodes empty.
__global__ void __launch_bounds__(kBlock) k_init(uint64_t* __restrict__ planes, Lattice L,
                                                 uint64_t key_init, uint64_t thr_fill) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)L.H * L.wd) return;
    const uint32_t y = (uint32_t)(idx / L.wd), w = (uint32_t)(idx % L.wd);
    const uint64_t fluid = ~solid_word(L, y, idx);
    for (uint64_t c = 0; c < 7; c++) {
        uint64_t word = 0;
        const uint64_t base = (c << 40) + ((uint64_t)y << 20) + 64ull * w;
        for (uint32_t b = 0; b < 64; b++) {
            const uint64_t h = hash64(key_init, base + b);
            word |= (uint64_t)((h >> 32) < thr_fill) << b;
        }
        planes[c * L.ps + idx] = word & fluid;
    }
}

__global__ void __launch_bounds__(kBlock) k_or_reduce(const uint64_t* __restrict__ p, size_t n,
                                                      unsigned long long* acc) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t v = 0;
    for (; i < n; i += (size_t)gridDim.x * kBlock) v |= p[i];
    // wave-level OR, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicOr(acc, (unsigned long long)v);
}

// Momentum of channel c in units (1/2, sqrt(3)/2); c_i at (i-2)*60 degrees.
__constant__ int kPx[7] = {-1, 1, 2, 1, -1, -2, 0};
__constant__ int kPy[7] = {-1, -1, 0, 1, 1, 0, 0};

// acc[0..10] += mass, p_x, p_y, count of channels 0..6, solid nodes.
__global__ void __launch_bounds__(kBlock) k_observe_global(const uint64_t* __restrict__ planes,
                                                           Lattice L, unsigned long long* acc) {
    __shared__ long long part[kBlock / 64][11];
    long long v[11] = {0};
    const size_t n = (size_t)L.H * L.wd;
    for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * kBlock) {
        const uint32_t y = (uint32_t)(idx / L.wd);
        for (int c = 0; c < 7; c++) {
            const long long k = __popcll(planes[(size_t)c * L.ps + idx]);
            v[0] += k;
            v[1] += kPx[c] * k;
            v[2] += kPy[c] * k;
            v[3 + c] += k;
        }
        v[10] += __popcll(solid_word(L, y, idx));
    }
    for (int j = 0; j < 11; j++)
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int j = 0; j < 11; j++) part[wave][j] = v[j];
    __syncthreads();
    if (threadIdx.x < 11) {
        long long s = 0;
        for (int k = 0; k < kBlock / 64; k++) s += part[k][threadIdx.x];
        atomicAdd(acc + threadIdx.x, (unsigned long long)s);
    }
}

// Block sums over b x b node blocks: one thread per output block (by, bx),
// for block rows brow0 .. brow0 + brows - 1 and block columns bx0 .. bx0 +
// nbx - 1, written row-major (nbx blocks per row).  b divides 64 (a block is
// a b-bit field of one word) or is a multiple of 64 (a block spans b/64
// whole words).
__global__ void __launch_bounds__(kBlock) k_observe_blocks(const uint64_t* __restrict__ planes,
                                                           Lattice L, uint32_t b, uint32_t brow0,
                                                           uint32_t brows, uint32_t bx0, uint32_t nbx,
                                                           int32_t* __restrict__ out) {
    const size_t o = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (o >= (size_t)brows * nbx) return;
    const uint32_t by = brow0 + (uint32_t)(o / nbx), bx = bx0 + (uint32_t)(o % nbx);
    const uint32_t y0 = by * b, y1 = min(L.H, y0 + b);
    int32_t rho = 0, px = 0, py = 0;
    uint32_t w0, w1;
    uint64_t field;
    if (b < 64) {
        w0 = (bx * b) >> 6;
        w1 = w0 + 1;
        field = ((1ull << b) - 1) << ((bx * b) & 63);
    } else {
        w0 = bx * (b >> 6);
        w1 = min(L.wd, w0 + (b >> 6));
        field = ~0ull;
    }
    for (uint32_t y = y0; y < y1; y++)
        for (uint32_t w = w0; w < w1; w++) {
            const size_t idx = (size_t)y * L.wd + w;
            for (int c = 0; c < 7; c++) {
                const int32_t k = __popcll(planes[(size_t)c * L.ps + idx] & field);
                rho += k;
                px += kPx[c] * k;
                py += kPy[c] * k;
            }
        }
    int32_t* dst = out + o * 3;
    dst[0] = rho;
    dst[1] = px;
    dst[2] = py;
}

// Row sums of (rho, p_x, p_y) for rows row0 .. row0 + rows - 1: one workgroup
// per row at a time, threads over the row's words, then a workgroup sum.
__global__ void __launch_bounds__(kBlock) k_observe_rows(const uint64_t* __restrict__ planes,
                                                         Lattice L, uint32_t row0, uint32_t rows,
                                                         int64_t* __restrict__ out) {
    __shared__ int32_t part[3][kBlock / 64];
    for (uint32_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const size_t base = (size_t)(row0 + r) * L.wd;
        int32_t v[3] = {0, 0, 0};
        for (uint32_t w = threadIdx.x; w < L.wd; w += kBlock)
            for (int c = 0; c < 7; c++) {
                const int32_t k = __popcll(planes[(size_t)c * L.ps + base + w]);
                v[0] += k;
                v[1] += kPx[c] * k;
                v[2] += kPy[c] * k;
            }
        for (int i = 0; i < 3; i++) {
            for (int d = 32; d > 0; d >>= 1) v[i] += __shfl_xor(v[i], d);
            if ((threadIdx.x & 63) == 0) part[i][threadIdx.x >> 6] = v[i];
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            int64_t sum = 0;
            for (int k = 0; k < kBlock / 64; k++) sum += part[threadIdx.x][k];
            out[(size_t)r * 3 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

// acc[0] += sum over planes c = 0..7, words (y, w) of H(word, c*2^40 + y*2^20 + w).
__global__ void __launch_bounds__(kBlock) k_digest(const uint64_t* __restrict__ planes, Lattice L,
                                                   unsigned long long* acc) {
    uint64_t d = 0;
    const size_t n = (size_t)L.H * L.wd;
    for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * kBlock) {
        const uint32_t y = (uint32_t)(idx / L.wd), w = (uint32_t)(idx % L.wd);
        for (uint64_t c = 0; c < 7; c++) d += hash64(planes[c * L.ps + idx], counter(c, y, w));
        d += hash64(solid_word(L, y, idx), counter(7, y, w));
    }
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(acc, (unsigned long long)d);
}

// One time step t -> t+1, one thread per 64-node word (y, w).
// Motion in pull form (odd rows shifted by +1/2, c_i at (i-2)*60 deg): the
// particle arriving with velocity c_i comes from the neighbour at -c_i.
// rotl1 (shift towards larger x) takes bit x-1, rotr1 takes bit x+1:
//   c2 (E):  row y, rotl1          c5 (W):  row y, rotr1
//   c3 (NE): row y-1, rotl1 if y even       c4 (NW): row y-1, rotr1 if y odd
//   c0 (SW): row y+1, rotr1 if y odd        c1 (SE): row y+1, rotl1 if y even
// The carry bit of a shifted word comes from the neighbouring word of the
// same row (periodic in x).  Then collision / bounce-back / forcing.
template <int RULES>
__global__ void __launch_bounds__(kBlock) k_step1(const uint64_t* __restrict__ in,
                                                  uint64_t* __restrict__ out, Lattice L, Dyn D,
                                                  uint64_t t) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)L.H * L.wd) return;
    const uint32_t y = (uint32_t)(idx / L.wd), w = (uint32_t)(idx % L.wd);
    const uint32_t ym = y ? y - 1 : L.H - 1, yp = (y + 1 == L.H) ? 0 : y + 1;
    const uint32_t wl = w ? w - 1 : L.wd - 1, wr = (w + 1 == L.wd) ? 0 : w + 1;
    const size_t ps = L.ps;
    const size_t rm = (size_t)ym * L.wd, r0 = (size_t)y * L.wd, rp = (size_t)yp * L.wd;

    uint64_t a[7];
    a[2] = (in[2 * ps + r0 + w] << 1) | (in[2 * ps + r0 + wl] >> 63);
    a[5] = (in[5 * ps + r0 + w] >> 1) | (in[5 * ps + r0 + wr] << 63);
    a[6] = in[6 * ps + r0 + w];
    if ((y & 1) == 0) {
        a[3] = (in[3 * ps + rm + w] << 1) | (in[3 * ps + rm + wl] >> 63);
        a[4] = in[4 * ps + rm + w];
        a[0] = in[0 * ps + rp + w];
        a[1] = (in[1 * ps + rp + w] << 1) | (in[1 * ps + rp + wl] >> 63);
    } else {
        a[3] = in[3 * ps + rm + w];
        a[4] = (in[4 * ps + rm + w] >> 1) | (in[4 * ps + rm + wr] << 63);
        a[0] = (in[0 * ps + rp + w] >> 1) | (in[0 * ps + rp + wr] << 63);
        a[1] = in[1 * ps + rp + w];
    }
    const uint64_t solid = solid_word(L, y, idx);
    const uint64_t ctr = counter(t, y, w);
    uint64_t chi;
    if (D.chir_mode == FHP_CHIR_HASH) chi = hash64(D.key_chir, ctr);
    else chi = (D.chir_mode == FHP_CHIR_ONE) ? ~0ull : 0ull;
    const uint64_t coin = D.thr_force ? coin_word(hash64(D.key_force, ctr), D.thr_force) : 0ull;
    uint64_t o[7];
    update<RULES>(a, solid, chi, coin, o);
#pragma unroll
    for (int c = 0; c < 7; c++) out[c * ps + idx] = o[c];
}

unsigned grid_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
unsigned grid_capped(size_t n) {
    const size_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g < 4096 ? (g ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t st) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_pack(const uint8_t* bytes, uint32_t row0, uint32_t rows, const Lattice& L,
                       uint64_t* planes, uint64_t* S, int mask_only, hipStream_t st) {
    const size_t threads = (size_t)rows * L.wd * 64;
    if (!threads) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(threads)), dim3(kBlock), 0, st, bytes, row0, rows, L,
                       planes, S, mask_only);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint64_t* planes, const Lattice& L, uint32_t row0, uint32_t rows,
                         uint8_t* bytes, hipStream_t st) {
    const size_t threads = (size_t)rows * L.wd * 64;
    if (!threads) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(threads)), dim3(kBlock), 0, st, planes, L, row0,
                       rows, bytes);
    return hipGetLastError();
}

hipError_t launch_init(uint64_t* planes, const Lattice& L, uint64_t key_init, uint64_t thr_fill,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(grid_for((size_t)L.H * L.wd)), dim3(kBlock), 0, st, planes, L,
                       key_init, thr_fill);
    return hipGetLastError();
}

hipError_t launch_or_reduce(const uint64_t* p, size_t n, uint64_t* acc, hipStream_t st) {
    hipLaunchKernelGGL(k_or_reduce, dim3(grid_capped(n)), dim3(kBlock), 0, st, p, n,
                       (unsigned long long*)acc);
    return hipGetLastError();
}

hipError_t launch_observe_global(const uint64_t* planes, const Lattice& L, uint64_t* acc,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_observe_global, dim3(grid_capped((size_t)L.H * L.wd)), dim3(kBlock), 0,
                       st, planes, L, (unsigned long long*)acc);
    return hipGetLastError();
}

hipError_t launch_observe_blocks(const uint64_t* planes, const Lattice& L, uint32_t b,
                                 uint32_t brow0, uint32_t brows, uint32_t bx0, uint32_t nbx,
                                 int32_t* out, hipStream_t st) {
    const size_t n = (size_t)brows * nbx;
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_observe_blocks, dim3(grid_for(n)), dim3(kBlock), 0, st, planes, L, b,
                       brow0, brows, bx0, nbx, out);
    return hipGetLastError();
}

hipError_t launch_observe_rows(const uint64_t* planes, const Lattice& L, uint32_t row0,
                               uint32_t rows, int64_t* out, hipStream_t st) {
    if (!rows) return hipSuccess;
    hipLaunchKernelGGL(k_observe_rows, dim3(rows < 4096 ? rows : 4096), dim3(kBlock), 0, st,
                       planes, L, row0, rows, out);
    return hipGetLastError();
}

hipError_t launch_digest(const uint64_t* planes, const Lattice& L, uint64_t* acc, hipStream_t st) {
    hipLaunchKernelGGL(k_digest, dim3(grid_capped((size_t)L.H * L.wd)), dim3(kBlock), 0, st,
                       planes, L, (unsigned long long*)acc);
    return hipGetLastError();
}

hipError_t launch_step1(const uint64_t* in, uint64_t* out, const Lattice& L, const Dyn& D,
                        uint64_t t, hipStream_t st) {
    const dim3 grid(grid_for((size_t)L.H * L.wd));
    if (D.rules == kRulesFHP1)
        hipLaunchKernelGGL(k_step1<kRulesFHP1>, grid, dim3(kBlock), 0, st, in, out, L, D, t);
    else if (D.rules == kRulesFHP3)
        hipLaunchKernelGGL(k_step1<kRulesFHP3>, grid, dim3(kBlock), 0, st, in, out, L, D, t);
    else
        hipLaunchKernelGGL(k_step1<kRulesFHP2>, grid, dim3(kBlock), 0, st, in, out, L, D, t);
    return hipGetLastError();
}

}  // namespace fhp
