// fhp_stepk.hip -- temporally blocked FHP update: K time steps per pass over
// HBM (K = 1..FHP_MAX_DEPTH).
//
// Decomposition.  A workgroup owns a band of T consecutive rows and the full
// lattice width: thread w holds 64-node word w of every row it touches, so
// the periodic wrap in x needs no halo words.  The band sweeps downwards
// through rows y0-K .. y0+T+K-1 of the input buffer, one row per iteration.
// Level 0 is the loaded row; level l (1..K) is the state after l steps, and
// its row rho = r - l is computed as soon as level l-1 has produced rows
// rho-1, rho and rho+1 (pull streaming reads exactly those).  Each level
// keeps the last two rows of the level below it in registers, so every input
// row is read from HBM once per band and only the 2K halo rows are read twice
// (by the neighbouring bands).  Level K rows y0 .. y0+T-1 are stored.
//
// Horizontal carries.  A 1-node shift of a word needs one bit of the
// neighbouring word: bit 63 of the left word for rotl1, bit 0 of the right
// word for rotr1.  After a row is produced each thread publishes those bits of
// the six moving planes in one LDS dword, the workgroup synchronises, and
// each thread reads its two neighbours' dwords (wrapping at the row ends).
// Two LDS slots alternate so that one barrier per exchange suffices.
//
// Time: level l of a pass starting at t0 applies step t0 + l - 1 (hash
// counters use that t and the absolute row index, so results do not depend
// on K or on the band size).
#include "fhp_device.h"
#include "fhp_internal.h"

namespace fhp {
namespace {

// One row of one level, as seen by one thread.
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

// Workgroup barrier that orders LDS traffic only: global loads issued for the
// next row stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int K>
__global__ void __launch_bounds__(512) k_stepk(const uint64_t* __restrict__ in,
                                                uint64_t* __restrict__ out, Lattice L, Dyn D,
                                                uint64_t t0, uint32_t T) {
    extern __shared__ uint32_t xch[];  // 2 slots x blockDim.x dwords
    const uint32_t nt = blockDim.x;
    const uint32_t lane = threadIdx.x;
    const bool valid = lane < L.wd;
    const uint32_t w = valid ? lane : 0;
    const uint32_t wl = w ? w - 1 : L.wd - 1;
    const uint32_t wr = (w + 1 == L.wd) ? 0 : w + 1;
    const uint32_t H = L.H;
    const uint32_t y0 = blockIdx.x * T;
    const uint32_t rows = min(T, H - y0);
    const int n_iter = (int)rows + 2 * K;
    const size_t ps = L.ps;

    auto wrap_row = [&](int r) -> uint32_t {
        int m = r % (int)H;
        return (uint32_t)(m < 0 ? m + (int)H : m);
    };
    // Issues the loads of row y; the wall rows are applied when the row is
    // consumed, so that nothing waits on these loads before the next row.
    auto load = [&](uint32_t y, Row& x) {
        const size_t base = (size_t)y * L.wd + w;
#pragma unroll
        for (int c = 0; c < 7; c++) x.p[c] = in[c * ps + base];
        x.s = L.S ? L.S[base] : 0ull;
    };
    uint32_t slot = 0;
    auto exchange = [&](Row& x) {
        const uint32_t bits = (uint32_t)(x.p[1] >> 63) | ((uint32_t)(x.p[2] >> 63) << 1) |
                              ((uint32_t)(x.p[3] >> 63) << 2) | ((uint32_t)(x.p[0] & 1) << 8) |
                              ((uint32_t)(x.p[4] & 1) << 9) | ((uint32_t)(x.p[5] & 1) << 10);
        uint32_t* buf = xch + slot * nt;
        buf[lane] = bits;
        lds_barrier();
        x.c = (buf[wl] & 0x7u) | (buf[wr] & 0x700u);
        slot ^= 1;
    };

    Row A[K + 1], B[K + 1];  // level l input rows rho-1 (A) and rho (B), from level l-1
    Row nxt;
    load(wrap_row((int)y0 - K), nxt);
    for (int i = 0; i < n_iter; i++) {
        const int r = (int)y0 - K + i;
        Row X = nxt;
        if (i + 1 < n_iter) load(wrap_row(r + 1), nxt);
        {
            const uint32_t y = wrap_row(r);
            if (L.walls && (y == 0 || y == H - 1)) X.s = ~0ull;
        }
        exchange(X);
        bool have = true;  // X holds a new row of level l-1
#pragma unroll
        for (int l = 1; l <= K; l++) {
            if (!have) break;
            if (i >= 2 * l) {
                const uint32_t rho = wrap_row(r - l);
                const bool odd = rho & 1;
                const Row& a = A[l];
                const Row& b = B[l];
                uint64_t n[7];
                n[3] = odd ? a.p[3] : rotl1(a.p[3], (a.c >> 2) & 1);
                n[4] = odd ? rotr1(a.p[4], (a.c >> 9) & 1) : a.p[4];
                n[2] = rotl1(b.p[2], (b.c >> 1) & 1);
                n[5] = rotr1(b.p[5], (b.c >> 10) & 1);
                n[6] = b.p[6];
                n[0] = odd ? rotr1(X.p[0], (X.c >> 8) & 1) : X.p[0];
                n[1] = odd ? X.p[1] : rotl1(X.p[1], X.c & 1);
                const uint64_t tl = t0 + (uint64_t)(l - 1);
                const uint64_t ctr = counter(tl, rho, w);
                uint64_t chi;
                if (D.chir_mode == FHP_CHIR_HASH) chi = hash64(D.key_chir, ctr);
                else chi = (D.chir_mode == FHP_CHIR_ONE) ? ~0ull : 0ull;
                const uint64_t coin =
                    D.thr_force ? coin_word(hash64(D.key_force, ctr), D.thr_force) : 0ull;
                Row Y;
                update(n, b.s, chi, coin, Y.p);
                Y.s = b.s;
                A[l] = B[l];
                B[l] = X;
                if (l < K) {
                    exchange(Y);
                    X = Y;
                } else if (valid) {
                    const size_t base = (size_t)rho * L.wd + w;
#pragma unroll
                    for (int c = 0; c < 7; c++) out[c * ps + base] = Y.p[c];
                }
            } else {
                A[l] = B[l];
                B[l] = X;
                have = false;
            }
        }
    }
}

template <int K>
hipError_t launch_k(const uint64_t* in, uint64_t* out, const Lattice& L, const Dyn& D, uint64_t t,
                    uint32_t T, hipStream_t st) {
    const uint32_t nt = (L.wd + 63) / 64 * 64;
    const uint32_t bands = (L.H + T - 1) / T;
    hipLaunchKernelGGL(k_stepk<K>, dim3(bands), dim3(nt), 2 * nt * sizeof(uint32_t), st, in, out,
                       L, D, t, T);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stepk(uint32_t K, const uint64_t* in, uint64_t* out, const Lattice& L,
                        const Dyn& D, uint64_t t, uint32_t T, hipStream_t st) {
    switch (K) {
        case 1: return launch_k<1>(in, out, L, D, t, T, st);
        case 2: return launch_k<2>(in, out, L, D, t, T, st);
        case 3: return launch_k<3>(in, out, L, D, t, T, st);
        case 4: return launch_k<4>(in, out, L, D, t, T, st);
        case 5: return launch_k<5>(in, out, L, D, t, T, st);
        case 6: return launch_k<6>(in, out, L, D, t, T, st);
        case 7: return launch_k<7>(in, out, L, D, t, T, st);
        case 8: return launch_k<8>(in, out, L, D, t, T, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fhp
