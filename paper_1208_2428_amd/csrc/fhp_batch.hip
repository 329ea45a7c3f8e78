// fhp_batch.hip -- many independent lattices of uneven sizes in one
// persistent launch (and the C ABI of batches).
//
// Work decomposition.  Every lattice (member) is cut into bands of T rows
// (T even, T | H), as in the single-lattice blocked kernel.  A band needs one
// lane per 64-node word of a row, i.e. wd = W/64 lanes; bands with the same
// (wd, T) are packed side by side into the waves of one workgroup, each wave
// holding consecutive bands of a single member (so a wave can hold e.g. 32
// bands of one 128-wide lattice, and a 100-word band spans two waves).  All
// per-member values are then uniform across a wave and kept in scalar
// registers; per lane remain the word, the band and the hash base.  The
// horizontal carry exchange wraps inside each band's lanes.
//
// Work items are (pass, group) pairs in pass-major order: workgroup g takes
// item g first, later items come from a global counter.  A band's pass p
// reads its own rows and the K rows on each side, i.e. the neighbouring
// bands' results of pass p-1, and overwrites the buffer those bands read in
// pass p-1; so item (p, band b) waits until bands b-1, b, b+1 have completed
// p passes (agent-scope release/acquire on per-band counters).  Items are
// taken in order and every taken item is held by a running workgroup (the
// grid is never larger than what is resident at once), so the oldest
// unfinished item can always proceed.  The wait is bounded: on time-out the launch aborts and the
// host reports an error.  The last workgroup to leave advances every member's
// time and buffer index and resets the counters, so a launch can be replayed
// from a graph without host work in between.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <utility>
#include <vector>

#include "fhp_device.h"
#include "fhp_groups.h"
#include "fhp_internal.h"
#include "fhp_sweep.h"

namespace fhp {
namespace {

// Pointers into global memory (address space 1).
using GlobalU64 = __attribute__((address_space(1))) uint64_t;
using GlobalChar = __attribute__((address_space(1))) char;

// A member's seven planes are addressed through one buffer resource, whose
// byte offsets are 32-bit.
inline bool planes_fit_rsrc(uint32_t W, uint32_t H) {
    return 7ull * layout_for(W, H).plane_words * 8ull <= 0xffffffffull;
}

struct MemberDesc {
    uint64_t* buf[2];
    const uint64_t* S;   // obstacle plane or nullptr
    uint64_t ps;         // plane stride in words
    uint64_t t0;         // steps completed
    uint64_t key_chir, key_force;
    uint32_t thr_force;       // floor(f * 2^38) < 2^32
    uint32_t chi_and, chi_or; // chirality word = (hash & chi_and) | chi_or, per 32-bit half
    uint32_t H, wd, walls, cur;
    uint32_t passes;     // passes this member may still run (0xffffffff: no limit)
    uint32_t done_off;   // first band counter
    uint32_t nbands, T;
};

struct BatchHeader {
    uint32_t queue;     // next work item
    uint32_t exited;    // workgroups that left the launch
    uint32_t status;    // nonzero: a dependency wait timed out
    uint32_t n_groups, passes, n_members, n_done, K;
};

constexpr uint32_t kNoLimit = 0xffffffffu;
// Depth of batches and pools unless set (the deepest; the 512-lattice
// ensemble measured 14% faster at 5 than at 4).  Members are at least
// FHP_BATCH_MIN_HEIGHT = 8 >= K rows high, so a band's halo wraps a lattice
// at most once.
constexpr uint32_t kBatchDefaultDepth = FHP_BATCH_MAX_DEPTH;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint32_t load_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Scalar copy of a value that is uniform across the wave.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

template <int K, bool FORCE, bool MASK, int RULES>
__global__ void __launch_bounds__(512) k_batch(BatchHeader* __restrict__ hdr,
                                               MemberDesc* __restrict__ members,
                                               const GroupDesc* __restrict__ groups,
                                               const WaveDesc* __restrict__ waves,
                                               uint32_t* __restrict__ done) {
    extern __shared__ uint32_t xch[];  // 2 carry slots x 4 halves x nt entries, then one broadcast word
    const uint32_t nt = blockDim.x;
    const uint32_t lane = threadIdx.x;
    const uint32_t wave = uni(lane >> 6);
    uint32_t* bcast = xch + 8 * nt;
    const uint32_t n_groups = hdr->n_groups;
    const uint32_t passes = hdr->passes;
    const uint32_t n_items = n_groups * passes;
    uint32_t slot = 0;

    bool first = true;
    for (;;) {
        uint32_t item;
        if (first) {  // the first round of items is static: item = workgroup
            item = blockIdx.x;
            first = false;
        } else {
            if (n_items <= gridDim.x) break;
            if (lane == 0) bcast[0] = atomicAdd(&hdr->queue, 1u) + gridDim.x;
            __syncthreads();
            item = uni(bcast[0]);
            __syncthreads();
        }
        if (item >= n_items) break;
        const uint32_t p = item / n_groups;
        const GroupDesc G = groups[item - p * n_groups];
        const uint32_t wd = G.wd, T = G.T;
        const bool wave_on = wave < G.nwaves;
        const WaveDesc D = waves[G.first_wave + (wave_on ? wave : 0)];
        // this wave's member: every value read from it is wave-uniform
        const MemberDesc* M = members + uni(D.m);
        const uint32_t rel = uni(D.rel0) + (lane & 63);
        const uint32_t j = rel / wd;
        const uint32_t w = rel - j * wd;
        const bool valid = wave_on && j < uni(D.count);
        const uint32_t b = uni(D.band0) + (valid ? j : 0);
        const uint32_t m_passes = uni(M->passes);
        const bool active = valid && p < m_passes;
        if (!__syncthreads_or(active)) continue;

        const uint32_t nb = uni(M->nbands);
        const uint32_t done_off = uni(M->done_off);
        if (p > 0) {  // wait for the neighbouring bands' previous pass
            const uint32_t bm = b ? b - 1 : nb - 1, bq = (b + 1 == nb) ? 0 : b + 1;
            const uint32_t* dm = done + done_off;
            uint32_t spins = 0;
            int abort = 0;
            for (;;) {
                int ok = 1;
                if (active && w == 0)
                    ok = load_acquire(dm + bm) >= p && load_acquire(dm + b) >= p &&
                         load_acquire(dm + bq) >= p;
                if (__syncthreads_and(ok)) break;
                int stop = 0;
                if (lane == 0)
                    stop = (++spins > kSpinLimit) ||
                           __hip_atomic_load(&hdr->status, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) != 0;
                if (__syncthreads_or(stop)) {
                    abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (abort) {
                if (lane == 0) atomicOr(&hdr->status, 1u);
                break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }

        // ---- one pass (K steps) of this lane's band: the sweep of the
        // single-lattice blocked kernel, with rows counted relative to the
        // band (d = row - y0, the same for every lane of the item).
        const uint32_t H = uni(M->H);
        const uint32_t first = lane - w;  // the band's first lane
        const uint32_t wl = valid ? first + (w ? w - 1 : wd - 1) : lane;
        const uint32_t wr = valid ? first + ((w + 1 == wd) ? 0 : w + 1) : lane;
        const uint32_t cur = (uni(M->cur) + p) & 1;
        // Planes are read through buffer resources, one per state buffer (a
        // member's seven planes lie within 4 GiB, checked when it is added):
        // the row offset in a vector register, the plane offset in a scalar
        // one, no 64-bit address arithmetic; a member without obstacles gets
        // an empty range for S, whose loads return 0 without touching memory.
        // Output rows are stored the same way without forcing (the 512-lattice
        // ensemble ran 1.5% faster than with 64-bit global pointers); with
        // forcing through global pointers (the served stream ran 1.1% slower
        // with resource stores, 0.25% faster with resource loads).
        constexpr bool kRsrcStore = !FORCE;
        const uint64_t ps = uni(M->ps);
        const uint64_t in_addr = uni((uint64_t)M->buf[cur]);
        const uint64_t out_addr = uni((uint64_t)M->buf[cur ^ 1]);
        const uint64_t s_addr = MASK ? uni((uint64_t)M->S) : 0ull;
        const Planes<false> pin((const uint64_t*)in_addr, ps, 0);
        const Planes<false> pout((const uint64_t*)out_addr, ps, 0);
        const __amdgpu_buffer_rsrc_t rs = region_rsrc((const void*)s_addr, s_addr ? (uint32_t)(ps * 8) : 0u);
        // global (not generic) pointer: generic accesses would also count
        // against the LDS wait of every carry exchange
        GlobalU64* out = (GlobalU64*)out_addr;
        auto store_plane = [&](int c, uint32_t boff, uint64_t v) __attribute__((always_inline)) {
            if constexpr (kRsrcStore)
                pout.store(c, boff, v);
            else
                __builtin_nontemporal_store(v, (GlobalU64*)((GlobalChar*)(out + c * ps) + boff));
        };
        const bool walls = uni(M->walls) != 0;
        const uint64_t tp = uni(M->t0) + (uint64_t)p * K;
        uint32_t chi_and = uni(M->chi_and);  // kept in a vector register (see chir_word)
        asm("" : "+v"(chi_and));
        const uint32_t chi_or = uni(M->chi_or);
        const uint64_t thr = uni(M->thr_force);
        const bool top = b == 0, bot = b + 1 == nb;  // bands whose halos wrap
        const uint32_t y0 = b * T;
        // hash states of row y0 at time tp; row y0 + d at time tp + l - 1 adds
        // the uniform ((l - 1) 2^40 + d 2^20) gamma, and (H 2^20) gamma when
        // the row wraps
        const uint64_t R0 = row_term(tp, y0);
        const uint64_t zc0 = word_base(uni(M->key_chir), w) + R0;
        const uint64_t zf0 = word_base(uni(M->key_force), w) + R0;
        const uint64_t HG = row_term(0, H);
        const uint32_t base_off = y0 * wd + w;  // word offset of row y0 (planes < 2^29 words)
        const int n_iter = (int)T + 2 * K;

        // Word offset of row y0 + d, wrapped into [0, H).
        auto row_off = [&](int d) __attribute__((always_inline)) -> uint32_t {
            uint32_t off = base_off + (uint32_t)(d * (int)wd);
            if (d < 0) off += top ? H * wd : 0u;
            else if (d >= (int)T) off -= bot ? H * wd : 0u;
            return off;
        };
        auto load = [&](int d, Row& x) __attribute__((always_inline)) {
            const uint32_t boff = row_off(d) * 8u;
#pragma unroll
            for (int c = 0; c < 7; c++) x.p[c] = pin.load(c, boff);
            if (MASK) x.s = buf_load64(rs, boff, 0);
        };

        uint64_t a3[K + 1], a4[K + 1], bp[K + 1][7], bs[K + 1];
        uint32_t ac[K + 1], b2[K + 1], b5[K + 1], bq[K + 1];
        auto push = [&](auto lc, const Row& x) __attribute__((always_inline)) {
            constexpr int l = decltype(lc)::value;
            a3[l] = bp[l][3];
            a4[l] = bp[l][4];
            ac[l] = bq[l];
#pragma unroll
            for (int c = 0; c < 7; c++) bp[l][c] = x.p[c];
            bs[l] = x.s;
            b2[l] = x.c[1];
            b5[l] = x.c[2];
            bq[l] = x.c[3];
        };
        Row nxt;
        load(-K, nxt);
        constexpr bool kPairs = RULES != kRulesFHP3 && (K <= 4 || (!FORCE && !MASK));
        uint64_t held[7];  // the last even output row, stored with the next one (kPairs)

        auto body = [&](int i, auto full_c, auto par_c) __attribute__((always_inline)) {
            constexpr bool FULL = decltype(full_c)::value;
            constexpr int PAR = decltype(par_c)::value;
            const int d0 = i - K;  // loaded row, relative to y0
            Row X = nxt;
            load((i + 1 < n_iter) ? d0 + 1 : d0, nxt);
            uint64_t s = MASK ? X.s : 0ull;
            // wall rows 0 and H-1: rows y0 + d0 in {0, -1} of the first band
            // and {T - 1, T} of the last
            if (walls) {
                if (d0 == 0 || d0 == -1) s = top ? ~0ull : s;
                else if (d0 == (int)T - 1 || d0 == (int)T) s = bot ? ~0ull : s;
            }
            X.s = s;
            exchange<((PAR + K) & 1) != 0>(xch, slot, nt, lane, wl, wr, X);  // y0 even: parity of y
            bool have = true;
            static_for<1, K>([&](auto lc) __attribute__((always_inline)) {
                constexpr int l = decltype(lc)::value;
                if (!FULL) {
                    if (!have) return;
                    if (i < 2 * l) {
                        push(lc, X);
                        have = false;
                        return;
                    }
                }
                const int dl = d0 - l;  // row of this level, relative to y0
                constexpr bool odd = ((PAR + K + l) & 1) != 0;  // y0 even: parity of the row
                uint64_t n[7];
                stream_in<odd>(a3[l], a4[l], ac[l], bp[l], b2[l], b5[l], X, n);
                const uint64_t sw = bs[l];
                uint64_t dz = ((uint64_t)(l - 1) << 40) + ((uint64_t)(int64_t)dl << 20);
                dz = in_sgprs(dz * kGamma);
                uint64_t zc = zc0 + dz, zf = zf0 + dz;
                if (dl < 0) {
                    const uint64_t fix = top ? HG : 0ull;
                    zc += fix;
                    zf += fix;
                } else if (dl >= (int)T) {
                    const uint64_t fix = bot ? HG : 0ull;
                    zc -= fix;
                    zf -= fix;
                }
                const uint64_t chi = chir_word(mix64(zc), chi_and, chi_or);
                const uint64_t hf = FORCE ? mix64(zf) : 0ull;
                Row Y;
                update<RULES>(n, sw, chi, FORCE ? coin_bit(hf) : 0ull, FORCE ? coin_up(hf, thr) : 0u, Y.p);
                Y.s = sw;
                push(lc, X);
                if (l < K) {
                    exchange<odd>(xch, slot, nt, lane, wl, wr, Y);
                    X = Y;
                } else if (active) {
                    // Rows are stored in pairs (dl even, dl + 1; dl has the
                    // parity of i) where the registers allow: a row of wd
                    // words ends inside a 32-byte sector unless 4 | wd, and
                    // storing the two rows that share it together writes that
                    // sector once; stored a sweep iteration apart, a busy L2
                    // often wrote it back twice (17% more DRAM writes on the
                    // 512-lattice ensemble).  With forcing or obstacles at
                    // depth 5, and for FHP-III, the held row would spill.
                    if constexpr (!kPairs) {
                        const uint32_t boff = (base_off + (uint32_t)(dl * (int)wd)) * 8u;  // 0 <= dl < T
#pragma unroll
                        for (int c = 0; c < 7; c++)
                            store_plane(c, boff, Y.p[c]);
                    } else if constexpr (PAR == 0) {
#pragma unroll
                        for (int c = 0; c < 7; c++) held[c] = Y.p[c];
                    } else {
                        const uint32_t boff = (base_off + (uint32_t)(dl * (int)wd)) * 8u;  // 1 <= dl < T
                        const uint32_t hoff = boff - wd * 8u;                             // row dl - 1
#pragma unroll
                        for (int c = 0; c < 7; c++) {
                            store_plane(c, hoff, held[c]);
                            store_plane(c, boff, Y.p[c]);
                        }
                    }
                }
            });
        };
        using F = std::false_type;
        using Tt = std::true_type;
        using P0 = std::integral_constant<int, 0>;
        using P1 = std::integral_constant<int, 1>;
        int i = 0;
        for (; i < 2 * K; i += 2) {
            body(i, F{}, P0{});
            body(i + 1, F{}, P1{});
        }
        // Six rows per trip in the steady state, as in the single-lattice
        // kernel (no register moves for the three-iteration lifetimes), where
        // that fits in registers: at depth 5, and for FHP-III at depth 3, it
        // spills, and the 512-lattice ensemble ran 2.4% slower.
        constexpr bool kSix = K <= 4 && !(RULES == kRulesFHP3 && K >= 3);
        for (; kSix && i + 6 <= n_iter; i += 6) {
            body(i, Tt{}, P0{});
            body(i + 1, Tt{}, P1{});
            body(i + 2, Tt{}, P0{});
            body(i + 3, Tt{}, P1{});
            body(i + 4, Tt{}, P0{});
            body(i + 5, Tt{}, P1{});
        }
        for (; i < n_iter; i += 2) {
            body(i, Tt{}, P0{});
            body(i + 1, Tt{}, P1{});
        }

        // Publish this band's pass to later passes of the same launch (with a
        // single pass per launch the kernel boundary orders the passes).
        if (passes > 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (active && w == 0)
                __hip_atomic_fetch_add(done + done_off + b, 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // The last workgroup out advances the members and resets the counters.
    // With one pass per launch no workgroup reads what another wrote (the
    // member table is only read until a workgroup leaves, and the kernel
    // boundary publishes the rest), so the exit needs no agent-scope fence:
    // an L2 write-back per workgroup cost 13% of such a launch.
    __syncthreads();
    if (lane == 0) {
        if (passes > 1) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bcast[0] = atomicAdd(&hdr->exited, 1u);
    }
    __syncthreads();
    if (bcast[0] == gridDim.x - 1) {
        if (passes > 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (hdr->status == 0) {
            for (uint32_t k = lane; k < hdr->n_members; k += nt) {
                MemberDesc& M = members[k];
                const uint32_t eff = min(passes, M.passes);
                M.t0 += (uint64_t)eff * K;
                M.cur ^= eff & 1;
                if (M.passes != kNoLimit) M.passes -= eff;
            }
        }
        if (passes > 1)  // single-pass launches leave the counters at zero
            for (uint32_t k = lane; k < hdr->n_done; k += nt) done[k] = 0;
        __syncthreads();
        if (lane == 0) {
            hdr->queue = 0;
            hdr->exited = 0;
        }
    }
}

// Sets the pass count of the next launch (a kernel, so that it can be captured).
__global__ void k_batch_header(BatchHeader* hdr, uint32_t passes, uint32_t K) {
    hdr->passes = passes;
    hdr->K = K;
}

// Dynamic LDS of the batch kernel: two exchange slots of four 32-bit arrays
// of nt entries, then one broadcast word.
constexpr size_t batch_lds_bytes(uint32_t nt) { return 2 * 4 * (size_t)nt * sizeof(uint32_t) + sizeof(uint32_t); }

template <int K, bool FORCE, bool MASK, int RULES>
hipError_t launch_batch_t(BatchHeader* hdr, MemberDesc* members, const GroupDesc* groups,
                          const WaveDesc* waves, uint32_t* done, uint32_t grid, uint32_t nt,
                          hipStream_t st) {
    hipLaunchKernelGGL((k_batch<K, FORCE, MASK, RULES>), dim3(grid), dim3(nt), batch_lds_bytes(nt), st, hdr,
                       members, groups, waves, done);
    return hipGetLastError();
}

using BatchLaunch = hipError_t (*)(BatchHeader*, MemberDesc*, const GroupDesc*, const WaveDesc*,
                                   uint32_t*, uint32_t, uint32_t, hipStream_t);
using BatchKernel = const void*;

template <int K, bool FORCE, bool MASK, int RULES>
void pick_one(BatchLaunch* fn, BatchKernel* kern) {
    *fn = launch_batch_t<K, FORCE, MASK, RULES>;
    *kern = (const void*)k_batch<K, FORCE, MASK, RULES>;
}

// FHP-II has a kernel for every combination of forcing and obstacles; the
// other rule sets use the forcing variant (a zero rate draws no coin), and
// FHP-III runs at most kMaxDepthFHP3 steps per pass.
template <int K>
bool pick(bool force, bool mask, uint32_t rules, BatchLaunch* fn, BatchKernel* kern) {
    if (rules == kRulesFHP1) {
        if (mask) pick_one<K, true, true, kRulesFHP1>(fn, kern);
        else pick_one<K, true, false, kRulesFHP1>(fn, kern);
        return true;
    }
    if (rules == kRulesFHP3) {
        if constexpr (K <= kMaxDepthFHP3) {
            if (mask) pick_one<K, true, true, kRulesFHP3>(fn, kern);
            else pick_one<K, true, false, kRulesFHP3>(fn, kern);
            return true;
        }
        return false;
    }
    if (force && mask) pick_one<K, true, true, kRulesFHP2>(fn, kern);
    else if (force) pick_one<K, true, false, kRulesFHP2>(fn, kern);
    else if (mask) pick_one<K, false, true, kRulesFHP2>(fn, kern);
    else pick_one<K, false, false, kRulesFHP2>(fn, kern);
    return true;
}

bool pick_kernel(uint32_t K, bool force, bool mask, uint32_t rules, BatchLaunch* fn,
                 BatchKernel* kern) {
    switch (K) {
        case 1: return pick<1>(force, mask, rules, fn, kern);
        case 2: return pick<2>(force, mask, rules, fn, kern);
        case 3: return pick<3>(force, mask, rules, fn, kern);
        case 4: return pick<4>(force, mask, rules, fn, kern);
        case 5: return pick<5>(force, mask, rules, fn, kern);
        default: return false;
    }
}

// Steps per pass for a requested depth: FHP-III passes are at most
// kMaxDepthFHP3 deep.
uint32_t effective_depth(uint32_t depth, uint32_t rules) {
    return (rules == FHP_RULES_FHP3 && depth > kMaxDepthFHP3) ? kMaxDepthFHP3 : depth;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Band height for a member of height H: the largest even divisor of H that is
// at most `target` and at least K (so that halos reach only the neighbouring
// bands); the whole height if there is none.
uint32_t band_for(uint32_t H, uint32_t target, uint32_t K) {
    for (uint32_t T = (target < H ? target : H) & ~1u; T >= 2; T -= 2)
        if (H % T == 0 && T >= K) return T;
    return H;
}

// Default target band of a batch, from occupancy as for a single lattice:
// the largest even target up to 32 rows whose bands give every SIMD two
// waves, else one, else the target with the most waves; a member of wd words
// cut into b bands fills ceil(b * wd / 64) waves (narrow members share
// waves).  Measured on four 4096^2 channels at K = 5: 32-row bands 3.5e12,
// 8-row bands 5.3e12 node-updates/s.
uint32_t batch_default_band(const fhp_sim* sims, uint32_t n, uint32_t K) {
    const uint64_t simds = n ? sims[0].simds : 1024;
    auto waves = [&](uint32_t target) {
        uint64_t w = 0;
        for (uint32_t i = 0; i < n; i++) {
            const uint64_t bands = sims[i].L.H / band_for(sims[i].L.H, target, K);
            w += (bands * sims[i].L.wd + 63) / 64;
        }
        return w;
    };
    uint32_t lo = (K + 1) & ~1u;
    if (lo < 2) lo = 2;
    for (const uint64_t need : {2 * simds, simds})
        for (uint32_t T = 32; T >= lo; T -= 2)
            if (waves(T) >= need) return T;
    uint32_t best = 32;
    uint64_t most = waves(32);
    for (uint32_t T = 30; T >= lo; T -= 2) {
        const uint64_t w = waves(T);
        if (w > most) most = w, best = T;
    }
    return best;
}

}  // namespace
}  // namespace fhp

// ---------------------------------------------------------------------------
// Host side.  An Engine owns the device tables of one set of lattices and
// launches the batch kernel over them; batches (fixed members) and pools
// (members that come and go) both drive an Engine.

namespace fhp {
namespace {

struct Engine {
    hipStream_t st = nullptr;
    BatchHeader* hdr = nullptr;
    MemberDesc* members = nullptr;
    GroupDesc* groups = nullptr;
    WaveDesc* waves = nullptr;
    uint32_t* done = nullptr;
    uint32_t max_members = 0, max_segs = 0;
    // tiling
    uint32_t depth = kBatchDefaultDepth, band = 32, nt_req = 0, passes_per_launch = 1;
    uint32_t depth_req = kBatchDefaultDepth;  // depth asked for; depth = its effective value
    uint32_t rules = FHP_RULES_FHP2;          // rule set of every member
    int use_graph = 1;
    // current tables
    uint32_t nt = 64, n_groups = 0, n_done = 0, n_members = 0;
    bool force = false, mask = false;
    // pinned staging for the table uploads, reusable once `staged` completed
    uint8_t* stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t staged = nullptr;
    // graph of the last launch sequence
    hipGraphExec_t graph = nullptr;
    uint32_t g_K = 0, g_passes = 0, g_launches = 0, g_nt = 0, g_grid = 0;
    bool g_force = false, g_mask = false;
    uint32_t g_rules = 0;
};

// Device table space for up to `members` lattices and `segs` bands: header,
// members, groups (at most one per band), waves and per-band counters.
size_t engine_table_words(uint32_t members, uint32_t segs) {
    const size_t w = sizeof(uint64_t);
    return round_up(sizeof(BatchHeader), 256) / w + round_up((size_t)members * sizeof(MemberDesc), 256) / w +
           round_up((size_t)segs * sizeof(GroupDesc), 256) / w +
           round_up(max_waves(segs) * sizeof(WaveDesc), 256) / w + round_up((size_t)segs * 4, 256) / w;
}

int engine_init(Engine* e, uint64_t* tables, uint32_t members, uint32_t segs, hipStream_t st) {
    const size_t w = sizeof(uint64_t);
    uint64_t* p = tables;
    e->hdr = (BatchHeader*)p;
    p += round_up(sizeof(BatchHeader), 256) / w;
    e->members = (MemberDesc*)p;
    p += round_up((size_t)members * sizeof(MemberDesc), 256) / w;
    e->groups = (GroupDesc*)p;
    p += round_up((size_t)segs * sizeof(GroupDesc), 256) / w;
    e->waves = (WaveDesc*)p;
    p += round_up(max_waves(segs) * sizeof(WaveDesc), 256) / w;
    e->done = (uint32_t*)p;
    e->max_members = members;
    e->max_segs = segs;
    e->st = st;
    e->stage_bytes = sizeof(BatchHeader) + (size_t)members * sizeof(MemberDesc) +
                     (size_t)segs * sizeof(GroupDesc) + max_waves(segs) * sizeof(WaveDesc);
    if (fault_alloc()) return hip_fail(hipErrorOutOfMemory, "pinned (injected by FHP_FAULT)");
    FHP_HIP_TRY(hipHostMalloc((void**)&e->stage, e->stage_bytes, hipHostMallocDefault), "pinned");
    FHP_HIP_TRY(hipEventCreateWithFlags(&e->staged, hipEventDisableTiming), "event");
    FHP_HIP_TRY(launch_fill_u64((uint64_t*)e->done, (segs + 1) / 2, 0, st), "clear");
    return FHP_OK;
}

void engine_free(Engine* e) {
    if (e->graph) (void)hipGraphExecDestroy(e->graph);
    if (e->staged) (void)hipEventDestroy(e->staged);
    if (e->stage) (void)hipHostFree(e->stage);
    e->graph = nullptr;
    e->staged = nullptr;
    e->stage = nullptr;
}

MemberDesc member_desc(const fhp_sim* s, uint32_t passes, uint32_t T, uint32_t done_off) {
    MemberDesc M;
    memset(&M, 0, sizeof(M));
    M.buf[0] = s->buf[0];
    M.buf[1] = s->buf[1];
    M.S = s->has_mask ? s->S : nullptr;
    M.ps = s->L.ps;
    M.t0 = s->t;
    M.key_chir = s->D.key_chir;
    M.key_force = s->D.key_force;
    M.thr_force = (uint32_t)s->D.thr_force;
    M.chi_and = (s->D.chir_mode == FHP_CHIR_HASH) ? ~0u : 0u;
    M.chi_or = (s->D.chir_mode == FHP_CHIR_ONE) ? ~0u : 0u;
    M.H = s->L.H;
    M.wd = s->L.wd;
    M.walls = s->L.walls;
    M.cur = (uint32_t)s->cur;
    M.passes = passes;
    M.T = T;
    M.nbands = s->L.H / T;
    M.done_off = done_off;
    return M;
}

// Builds the member and group tables of sims[0..n) (pass limits `limit`, or
// no limit) and enqueues their upload on the engine's stream.
int engine_build(Engine* e, fhp_sim* const* sims, const uint32_t* limit, uint32_t n) {
    if (n > e->max_members) return fail(FHP_E_NOMEM, "%u lattices, room for %u", n, e->max_members);
    std::vector<MemberDesc> mem(n);
    std::vector<uint32_t> bandT(n), order(n);
    uint32_t done = 0, max_wd = 0;
    bool force = false, mask = false;
    for (uint32_t i = 0; i < n; i++) {
        const fhp_sim* s = sims[i];
        bandT[i] = band_for(s->L.H, e->band, e->depth);
        mem[i] = member_desc(s, limit ? limit[i] : kNoLimit, bandT[i], done);
        done += mem[i].nbands;
        order[i] = i;
        if (s->L.wd > max_wd) max_wd = s->L.wd;
        force |= s->D.thr_force != 0;
        mask |= s->has_mask != 0;
    }
    if (done > e->max_segs) return fail(FHP_E_NOMEM, "%u bands, room for %u", done, e->max_segs);
    // bands of equal (wd, T) share a workgroup: order the members by that
    // class, larger work first
    std::sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        const Lattice &a = sims[x]->L, &b = sims[y]->L;
        if (a.wd != b.wd) return a.wd > b.wd;
        if (bandT[x] != bandT[y]) return bandT[x] > bandT[y];
        if (a.H != b.H) return a.H > b.H;
        return x < y;
    });
    std::vector<MemberBands> mb;
    mb.reserve(n);
    for (uint32_t i : order) mb.push_back({i, sims[i]->L.wd, bandT[i], mem[i].nbands});
    uint32_t nt = e->nt_req ? e->nt_req : 64;
    const uint32_t need = (max_wd + 63) / 64 * 64;
    if (nt < need) nt = need;
    std::vector<GroupDesc> groups;
    std::vector<WaveDesc> waves;
    std::vector<uint32_t> lanes;
    pack_waves(mb, nt, groups, waves, lanes);
    order_groups(groups, lanes);
    if (waves.size() > max_waves(e->max_segs))
        return fail(FHP_E_NOMEM, "%zu waves, room for %llu", waves.size(),
                    (unsigned long long)max_waves(e->max_segs));
    BatchHeader h;
    memset(&h, 0, sizeof(h));
    h.n_groups = (uint32_t)groups.size();
    h.n_members = n;
    h.n_done = done;
    // stage into pinned memory (after the previous upload has been consumed)
    FHP_HIP_TRY(hipEventSynchronize(e->staged), "event");
    uint8_t* p = e->stage;
    const size_t bh = sizeof(h), bm = mem.size() * sizeof(MemberDesc),
                 bg = groups.size() * sizeof(GroupDesc), bw = waves.size() * sizeof(WaveDesc);
    memcpy(p, &h, bh);
    memcpy(p + bh, mem.data(), bm);
    memcpy(p + bh + bm, groups.data(), bg);
    memcpy(p + bh + bm + bg, waves.data(), bw);
    FHP_HIP_TRY(hipMemcpyAsync(e->hdr, p, bh, hipMemcpyHostToDevice, e->st), "upload");
    if (bm) FHP_HIP_TRY(hipMemcpyAsync(e->members, p + bh, bm, hipMemcpyHostToDevice, e->st), "upload");
    if (bg) FHP_HIP_TRY(hipMemcpyAsync(e->groups, p + bh + bm, bg, hipMemcpyHostToDevice, e->st), "upload");
    if (bw) FHP_HIP_TRY(hipMemcpyAsync(e->waves, p + bh + bm + bg, bw, hipMemcpyHostToDevice, e->st), "upload");
    FHP_HIP_TRY(hipEventRecord(e->staged, e->st), "event");
    if (done > e->n_done)  // counters beyond the previous tables may be stale
        FHP_HIP_TRY(launch_fill_u64((uint64_t*)e->done, (done + 1) / 2, 0, e->st), "clear");
    e->nt = nt;
    e->n_groups = h.n_groups;
    e->n_done = done;
    e->n_members = n;
    e->force = force;
    e->mask = mask;
    return FHP_OK;
}

// Persistent grid: every workgroup that fits on the device at once.
int engine_grid(uint32_t K, bool force, bool mask, uint32_t rules, uint32_t nt, uint32_t* grid) {
    BatchLaunch fn;
    BatchKernel kern;
    if (!pick_kernel(K, force, mask, rules, &fn, &kern))
        return fail(FHP_E_INVAL, "depth %u, rule set %u", K, rules);
    int per_cu = 0, dev = 0, cus = 0;
    FHP_HIP_TRY(hipGetDevice(&dev), "device");
    FHP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    FHP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)nt, batch_lds_bytes(nt)),
                "occupancy");
    *grid = (uint32_t)((per_cu < 1 ? 1 : per_cu) * cus);
    return FHP_OK;
}

int engine_kernel(Engine* e, uint32_t K, BatchLaunch* fn, uint32_t* grid) {
    BatchKernel kern;
    if (!pick_kernel(K, e->force, e->mask, e->rules, fn, &kern))
        return fail(FHP_E_INVAL, "depth %u, rule set %u", K, e->rules);
    return engine_grid(K, e->force, e->mask, e->rules, e->nt, grid);
}

int engine_enqueue(Engine* e, uint32_t K, uint32_t passes, uint32_t launches) {
    BatchLaunch fn;
    uint32_t grid;
    int rc = engine_kernel(e, K, &fn, &grid);
    if (rc) return rc;
    hipLaunchKernelGGL(k_batch_header, dim3(1), dim3(1), 0, e->st, e->hdr, passes, K);
    FHP_HIP_TRY(hipGetLastError(), "launch");
    for (uint32_t k = 0; k < launches; k++)
        FHP_HIP_TRY(fn(e->hdr, e->members, e->groups, e->waves, e->done, grid, e->nt, e->st),
                    "launch");
    return FHP_OK;
}

// `launches` launches of `passes` passes of depth K, replayed from a graph
// when enabled (the tables are read from device memory, so a graph stays valid
// while the number of groups and members changes).
int engine_run(Engine* e, uint32_t K, uint32_t passes, uint32_t launches) {
    if (!e->use_graph) return engine_enqueue(e, K, passes, launches);
    BatchLaunch fn;
    uint32_t grid;
    int rc = engine_kernel(e, K, &fn, &grid);
    if (rc) return rc;
    if (!e->graph || e->g_K != K || e->g_passes != passes || e->g_launches != launches ||
        e->g_nt != e->nt || e->g_grid != grid || e->g_force != e->force || e->g_mask != e->mask ||
        e->g_rules != e->rules) {
        if (e->graph) {
            (void)hipGraphExecDestroy(e->graph);
            e->graph = nullptr;
        }
        hipGraph_t g = nullptr;
        FHP_HIP_TRY(hipStreamBeginCapture(e->st, hipStreamCaptureModeThreadLocal), "capture");
        rc = engine_enqueue(e, K, passes, launches);
        hipError_t err = hipStreamEndCapture(e->st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (err != hipSuccess) return hip_fail(err, "end capture");
        err = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (err != hipSuccess) {
            e->graph = nullptr;
            return hip_fail(err, "instantiate");
        }
        e->g_K = K;
        e->g_passes = passes;
        e->g_launches = launches;
        e->g_nt = e->nt;
        e->g_grid = grid;
        e->g_force = e->force;
        e->g_mask = e->mask;
        e->g_rules = e->rules;
    }
    FHP_HIP_TRY(hipGraphLaunch(e->graph, e->st), "graph launch");
    return FHP_OK;
}

int engine_status(Engine* e) {
    FHP_HIP_TRY(hipStreamSynchronize(e->st), "sync");
    uint32_t status = 0;
    FHP_HIP_TRY(hipMemcpy(&status, &e->hdr->status, 4, hipMemcpyDeviceToHost), "copy");
    if (status) return fail(FHP_E_DEVICE, "batch launch aborted: a dependency wait timed out");
    return FHP_OK;
}

// Advances lattices whose tables are current by n steps: full passes through
// the engine, the remainder of n mod K as one more pass of that depth.
int engine_steps(Engine* e, uint64_t n) {
    const uint32_t K = e->depth;
    const uint64_t full = n / K;
    const uint32_t rest = (uint32_t)(n % K);
    if (full) {
        uint32_t per = e->passes_per_launch ? e->passes_per_launch : (uint32_t)full;
        if (per > full) per = (uint32_t)full;
        const uint32_t launches = (uint32_t)(full / per), tail = (uint32_t)(full % per);
        int rc = engine_run(e, K, per, launches);
        if (rc) return rc;
        if (tail) {
            rc = engine_enqueue(e, K, tail, 1);
            if (rc) return rc;
        }
    }
    if (rest) return engine_enqueue(e, rest, 1, 1);
    return FHP_OK;
}

// First-fit allocator of 256-byte blocks over the pool's lattice heap.
struct Heap {
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size) in words, sorted
    size_t alloc(size_t words) {
        for (size_t i = 0; i < free_list.size(); i++) {
            if (free_list[i].second >= words) {
                const size_t off = free_list[i].first;
                free_list[i].first += words;
                free_list[i].second -= words;
                if (!free_list[i].second) free_list.erase(free_list.begin() + i);
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t words) {
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
        it = free_list.insert(it, {off, words});
        if (it + 1 != free_list.end() && it->first + it->second == (it + 1)->first) {
            it->second += (it + 1)->second;
            free_list.erase(it + 1);
        }
        if (it != free_list.begin() && (it - 1)->first + (it - 1)->second == it->first) {
            (it - 1)->second += it->second;
            free_list.erase(it);
        }
    }
    size_t free_words() const {
        size_t s = 0;
        for (auto& f : free_list) s += f.second;
        return s;
    }
};

}  // namespace
}  // namespace fhp

using namespace fhp;

struct fhp_batch {
    uint32_t n;
    fhp_sim* sims;
    std::vector<fhp_sim*> ptrs;
    uint64_t* aux;
    Engine eng;
    bool tables_dirty;  // tiling changed: rebuild before the next step
    int changed;        // set by member handles when a member is changed alone
};

// One job of a pool.
struct PoolSlot {
    bool used = false;
    fhp_sim sim;
    size_t heap_off = 0, heap_words = 0;
    uint64_t remaining = 0;  // steps still to run
    hipEvent_t collected = nullptr;  // recorded after an asynchronous result copy
};

struct fhp_pool {
    Engine eng;
    uint64_t* heap_base;
    Heap heap;
    size_t heap_words;
    uint64_t* aux;
    std::vector<PoolSlot> slots;
    std::vector<uint32_t> finished;  // done slots not yet reported
    uint32_t max_bands, bands_used;
    int changed;         // membership or a member changed: rebuild the tables
    std::vector<uint32_t> table_slots;  // slots in the current tables
};

namespace {

struct BatchLayout {
    std::vector<size_t> member_off;  // word offsets of each member's planes
    size_t aux_off, tables_off, max_segs, total_bytes;
};

int batch_layout(const fhp_params* ps, uint32_t n, BatchLayout* bl) {
    if (!ps || n == 0) return fail(FHP_E_INVAL, "empty batch");
    size_t off = 0, segs = 0;
    bl->member_off.resize(n);
    for (uint32_t i = 0; i < n; i++) {
        int rc = validate(&ps[i]);
        if (rc) return fail(rc, "member %u: %s", i, fhp_last_error());
        if (ps[i].width / 64 > kMaxBlockedWords)
            return fail(FHP_E_INVAL, "member %u: width %u above %u", i, ps[i].width,
                        64 * kMaxBlockedWords);
        if (ps[i].height < FHP_BATCH_MIN_HEIGHT)
            return fail(FHP_E_INVAL, "member %u: height %u below %u", i, ps[i].height,
                        FHP_BATCH_MIN_HEIGHT);
        if (ps[i].rules != ps[0].rules)
            return fail(FHP_E_INVAL, "member %u: rule set %u, member 0 has %u; a batch runs one",
                        i, ps[i].rules, ps[0].rules);
        if (!planes_fit_rsrc(ps[i].width, ps[i].height))
            return fail(FHP_E_INVAL, "member %u: %u x %u, its seven planes exceed 4 GiB", i,
                        ps[i].width, ps[i].height);
        bl->member_off[i] = off;
        off += round_up(layout_for(ps[i].width, ps[i].height).aux_off, 32);  // planes and S
        segs += ps[i].height / 2;  // bands of at least 2 rows
    }
    bl->aux_off = off;
    off += kAuxWords;
    bl->tables_off = off;
    off += engine_table_words(n, (uint32_t)segs);
    bl->max_segs = segs;
    bl->total_bytes = off * sizeof(uint64_t);
    return FHP_OK;
}

int batch_rebuild(fhp_batch* b) {
    int rc = engine_build(&b->eng, b->ptrs.data(), nullptr, b->n);
    if (rc) return rc;
    b->tables_dirty = false;
    b->changed = 0;
    return FHP_OK;
}

// Pool member validation: the batch kernel's limits plus the pool's band room.
int pool_check(const fhp_params* p) {
    int rc = validate(p);
    if (rc) return rc;
    if (p->width / 64 > kMaxBlockedWords)
        return fail(FHP_E_INVAL, "width %u above %u", p->width, 64 * kMaxBlockedWords);
    if (p->height < FHP_BATCH_MIN_HEIGHT)
        return fail(FHP_E_INVAL, "height %u below %u", p->height, FHP_BATCH_MIN_HEIGHT);
    if (!planes_fit_rsrc(p->width, p->height))
        return fail(FHP_E_INVAL, "%u x %u: its seven planes exceed 4 GiB", p->width, p->height);
    return FHP_OK;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------ batches

int fhp_batch_workspace_bytes(const fhp_params* ps, uint32_t n, size_t* bytes) {
    if (!bytes) return fail(FHP_E_INVAL, "bytes is NULL");
    BatchLayout bl;
    int rc = batch_layout(ps, n, &bl);
    if (rc) return rc;
    *bytes = bl.total_bytes;
    return FHP_OK;
}

int fhp_batch_create(const fhp_params* ps, uint32_t n, void* dev_ws, size_t ws_bytes,
                     void* hip_stream, fhp_batch** out) {
    if (!out) return fail(FHP_E_INVAL, "out is NULL");
    *out = nullptr;
    BatchLayout bl;
    int rc = batch_layout(ps, n, &bl);
    if (rc) return rc;
    if (!dev_ws || ((uintptr_t)dev_ws & 255))
        return fail(FHP_E_INVAL, "workspace must be a non-NULL 256-byte aligned device pointer");
    if (ws_bytes < bl.total_bytes)
        return fail(FHP_E_NOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, bl.total_bytes);
    fhp_batch* b = new (std::nothrow) fhp_batch();
    if (!b) return fail(FHP_E_NOMEM, "host allocation failed");
    b->sims = (fhp_sim*)calloc(n, sizeof(fhp_sim));
    if (!b->sims) {
        delete b;
        return fail(FHP_E_NOMEM, "host allocation failed");
    }
    uint64_t* ws = (uint64_t*)dev_ws;
    hipStream_t st = (hipStream_t)hip_stream;
    b->n = n;
    b->aux = ws + bl.aux_off;
    rc = engine_init(&b->eng, ws + bl.tables_off, n, (uint32_t)bl.max_segs, st);
    b->eng.rules = ps[0].rules;
    b->eng.depth = effective_depth(b->eng.depth_req, b->eng.rules);
    for (uint32_t i = 0; i < n && !rc; i++) {
        const Layout lay = layout_for(ps[i].width, ps[i].height);
        rc = sim_setup(&b->sims[i], &ps[i], ws + bl.member_off[i], lay, b->aux, st);
        b->sims[i].owner = b;
        b->sims[i].changed = &b->changed;
        b->ptrs.push_back(&b->sims[i]);
    }
    if (!rc) {
        b->eng.band = batch_default_band(b->sims, n, b->eng.depth);
        rc = batch_rebuild(b);
    }
    if (rc) {
        engine_free(&b->eng);
        free(b->sims);
        delete b;
        return rc;
    }
    *out = b;
    return FHP_OK;
}

int fhp_batch_set_tiling(fhp_batch* b, uint32_t depth, uint32_t band, uint32_t group_threads,
                         uint32_t passes_per_launch) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    if (depth > FHP_BATCH_MAX_DEPTH) return fail(FHP_E_INVAL, "depth %u above %u", depth, FHP_BATCH_MAX_DEPTH);
    if (group_threads % 64 || group_threads > 512)
        return fail(FHP_E_INVAL, "group_threads %u: a multiple of 64 up to 512", group_threads);
    b->eng.depth_req = depth ? depth : kBatchDefaultDepth;
    b->eng.depth = effective_depth(b->eng.depth_req, b->eng.rules);
    b->eng.band = band ? band : batch_default_band(b->sims, b->n, b->eng.depth);
    b->eng.nt_req = group_threads;
    b->eng.passes_per_launch = passes_per_launch;
    return batch_rebuild(b);
}

int fhp_batch_set_graph(fhp_batch* b, int enable) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    b->eng.use_graph = enable != 0;
    return FHP_OK;
}

int fhp_batch_step(fhp_batch* b, uint64_t n) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    for (uint32_t i = 0; i < b->n; i++)
        if (b->sims[i].t + n >= kTimeLimit)
            return fail(FHP_E_STATE, "member %u: time would reach 2^24", i);
    if (b->tables_dirty || b->changed) {
        int rc = batch_rebuild(b);
        if (rc) return rc;
    }
    int rc = engine_steps(&b->eng, n);
    if (rc) return rc;
    // host mirror of the device-side bookkeeping
    const uint32_t K = b->eng.depth;
    const uint64_t passes = n / K + ((n % K) ? 1 : 0);
    for (uint32_t i = 0; i < b->n; i++) {
        b->sims[i].t += n;
        b->sims[i].cur ^= (int)(passes & 1);
    }
    return FHP_OK;
}

int fhp_batch_member(fhp_batch* b, uint32_t i, fhp_sim** view) {
    if (!b || !view) return fail(FHP_E_INVAL, "NULL argument");
    if (i >= b->n) return fail(FHP_E_INVAL, "member %u of %u", i, b->n);
    *view = &b->sims[i];
    return FHP_OK;
}

int fhp_batch_sync(fhp_batch* b) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    return engine_status(&b->eng);
}

void fhp_batch_destroy(fhp_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->eng.st);
    engine_free(&b->eng);
    free(b->sims);
    delete b;
}

// -------------------------------------------------------------------- pools

int fhp_pool_workspace_bytes(uint32_t max_slots, uint32_t max_bands, size_t lattice_bytes,
                             size_t* bytes) {
    if (!bytes || !max_slots || !max_bands) return fail(FHP_E_INVAL, "bad pool size");
    *bytes = (kAuxWords + engine_table_words(max_slots, max_bands)) * sizeof(uint64_t) +
             round_up(lattice_bytes, 256);
    return FHP_OK;
}

int fhp_pool_create(void* dev_arena, size_t arena_bytes, uint32_t max_slots, uint32_t max_bands,
                    void* hip_stream, fhp_pool** out) {
    if (!out) return fail(FHP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!dev_arena || ((uintptr_t)dev_arena & 255))
        return fail(FHP_E_INVAL, "arena must be a non-NULL 256-byte aligned device pointer");
    if (!max_slots || !max_bands) return fail(FHP_E_INVAL, "bad pool size");
    const size_t fixed = kAuxWords + engine_table_words(max_slots, max_bands);
    if (arena_bytes / sizeof(uint64_t) <= fixed)
        return fail(FHP_E_NOMEM, "arena of %zu bytes holds only the tables", arena_bytes);
    fhp_pool* pl = new (std::nothrow) fhp_pool();
    if (!pl) return fail(FHP_E_NOMEM, "host allocation failed");
    uint64_t* a = (uint64_t*)dev_arena;
    pl->aux = a;
    int rc = engine_init(&pl->eng, a + kAuxWords, max_slots, max_bands, (hipStream_t)hip_stream);
    if (rc) {
        engine_free(&pl->eng);
        delete pl;
        return rc;
    }
    pl->heap_base = a + fixed;
    pl->heap_words = (arena_bytes / sizeof(uint64_t) - fixed) / 32 * 32;
    pl->heap.free_list.push_back({0, pl->heap_words});
    pl->slots.resize(max_slots);
    pl->max_bands = max_bands;
    pl->bands_used = 0;
    *out = pl;
    return FHP_OK;
}

int fhp_pool_set_tiling(fhp_pool* pl, uint32_t depth, uint32_t band, uint32_t group_threads) {
    if (!pl) return fail(FHP_E_INVAL, "pool is NULL");
    if (depth > FHP_BATCH_MAX_DEPTH) return fail(FHP_E_INVAL, "depth %u above %u", depth, FHP_BATCH_MAX_DEPTH);
    if (group_threads % 64 || group_threads > 512)
        return fail(FHP_E_INVAL, "group_threads %u: a multiple of 64 up to 512", group_threads);
    for (auto& s : pl->slots)
        if (s.used) return fail(FHP_E_STATE, "tiling can change only while the pool is empty");
    pl->eng.depth_req = depth ? depth : kBatchDefaultDepth;
    pl->eng.depth = effective_depth(pl->eng.depth_req, pl->eng.rules);
    pl->eng.band = band ? band : 32;
    pl->eng.nt_req = group_threads;
    return FHP_OK;
}

int fhp_pool_set_rules(fhp_pool* pl, uint32_t rules) {
    if (!pl) return fail(FHP_E_INVAL, "pool is NULL");
    if (rules > FHP_RULES_FHP3) return fail(FHP_E_INVAL, "rule set %u unknown", rules);
    for (auto& s : pl->slots)
        if (s.used) return fail(FHP_E_STATE, "the rule set can change only while the pool is empty");
    pl->eng.rules = rules;
    pl->eng.depth = effective_depth(pl->eng.depth_req, rules);
    return FHP_OK;
}

int fhp_pool_admit(fhp_pool* pl, const fhp_params* p, uint64_t steps, uint32_t* slot) {
    if (!pl || !slot) return fail(FHP_E_INVAL, "NULL argument");
    int rc = pool_check(p);
    if (rc) return rc;
    if (p->rules != pl->eng.rules)
        return fail(FHP_E_INVAL, "rule set %u: this pool runs rule set %u (fhp_pool_set_rules)",
                    p->rules, pl->eng.rules);
    if (steps >= kTimeLimit) return fail(FHP_E_STATE, "%llu steps: time would reach 2^24",
                                         (unsigned long long)steps);
    uint32_t i = 0;
    while (i < pl->slots.size() && pl->slots[i].used) i++;
    if (i == pl->slots.size()) return fail(FHP_E_BUSY, "all %zu slots in use", pl->slots.size());
    const uint32_t T = band_for(p->height, pl->eng.band, pl->eng.depth);
    const uint32_t bands = p->height / T;
    if (pl->bands_used + bands > pl->max_bands)
        return fail(FHP_E_BUSY, "band table full (%u of %u)", pl->bands_used, pl->max_bands);
    const Layout lay = layout_for(p->width, p->height);
    const size_t words = round_up(lay.aux_off, 32);
    const size_t off = pl->heap.alloc(words);
    if (off == SIZE_MAX) return fail(FHP_E_BUSY, "arena full (%zu bytes free, %zu needed)",
                                     pl->heap.free_words() * 8, words * 8);
    PoolSlot& s = pl->slots[i];
    memset(&s.sim, 0, sizeof(s.sim));
    rc = sim_setup(&s.sim, p, pl->heap_base + off, lay, pl->aux, pl->eng.st, false);
    if (rc) {
        pl->heap.release(off, words);
        return rc;
    }
    s.sim.owner = pl;
    s.sim.changed = &pl->changed;
    s.used = true;
    s.heap_off = off;
    s.heap_words = words;
    s.remaining = steps;
    pl->bands_used += bands;
    pl->changed = 1;
    if (steps == 0) pl->finished.push_back(i);
    *slot = i;
    return FHP_OK;
}

int fhp_pool_tick(fhp_pool* pl, uint32_t passes) {
    if (!pl) return fail(FHP_E_INVAL, "pool is NULL");
    if (!passes) passes = 1;
    const uint32_t K = pl->eng.depth;
    // The tables list every job with full passes left and give each its total
    // count of full passes; the device counts them down, so the tables are
    // rebuilt only when jobs arrive or leave.
    if (pl->changed) {
        std::vector<fhp_sim*> act;
        std::vector<uint32_t> lim;
        pl->table_slots.clear();
        for (uint32_t i = 0; i < pl->slots.size(); i++) {
            PoolSlot& s = pl->slots[i];
            if (!s.used || s.remaining < K) continue;
            const uint64_t full = s.remaining / K;
            act.push_back(&s.sim);
            lim.push_back((uint32_t)(full < 0xfffffffeull ? full : 0xfffffffeull));
            pl->table_slots.push_back(i);
        }
        int rc = engine_build(&pl->eng, act.data(), lim.data(), (uint32_t)act.size());
        if (rc) return rc;
        pl->changed = 0;
    }
    std::vector<char> ran(pl->slots.size(), 0);
    bool any = false;
    for (uint32_t i : pl->table_slots) any |= pl->slots[i].remaining >= K;
    if (any) {
        int rc = engine_run(&pl->eng, K, 1, passes);  // one pass per launch
        if (rc) return rc;
        for (uint32_t i : pl->table_slots) {  // host mirror of the device bookkeeping
            PoolSlot& s = pl->slots[i];
            const uint64_t full = s.remaining / K;
            const uint64_t eff = full < passes ? full : passes;
            if (!eff) continue;
            s.sim.t += eff * K;
            s.sim.cur ^= (int)(eff & 1);
            s.remaining -= eff * K;
            ran[i] = 1;
        }
    }
    // Jobs left with fewer than K steps finish on the single-lattice kernels;
    // every job that reached its last step in this tick is reported once.
    for (uint32_t i = 0; i < pl->slots.size(); i++) {
        PoolSlot& s = pl->slots[i];
        if (!s.used) continue;
        if (s.remaining == 0) {
            if (ran[i]) pl->finished.push_back(i);
            continue;
        }
        if (s.remaining >= K) continue;
        const uint32_t r = (uint32_t)s.remaining;
        const uint32_t depth = s.sim.depth;
        s.sim.depth = r;
        int* ch = s.sim.changed;
        s.sim.changed = nullptr;
        int rc = fhp_step(&s.sim, r);
        s.sim.changed = ch;
        s.sim.depth = depth;
        if (rc) return rc;
        s.remaining = 0;
        pl->finished.push_back(i);
    }
    return FHP_OK;
}

int fhp_pool_done(fhp_pool* pl, uint32_t* slots, uint32_t cap, uint32_t* n_done) {
    if (!pl || !n_done || (cap && !slots)) return fail(FHP_E_INVAL, "NULL argument");
    const uint32_t n = (uint32_t)(pl->finished.size() < cap ? pl->finished.size() : cap);
    for (uint32_t k = 0; k < n; k++) slots[k] = pl->finished[k];
    pl->finished.erase(pl->finished.begin(), pl->finished.begin() + n);
    *n_done = n;
    return FHP_OK;
}

int fhp_pool_member(fhp_pool* pl, uint32_t slot, fhp_sim** view) {
    if (!pl || !view) return fail(FHP_E_INVAL, "NULL argument");
    if (slot >= pl->slots.size() || !pl->slots[slot].used)
        return fail(FHP_E_INVAL, "slot %u is not in use", slot);
    *view = &pl->slots[slot].sim;
    return FHP_OK;
}

int fhp_pool_result(fhp_pool* pl, uint32_t slot, uint32_t block, int32_t* host_dst, size_t bytes) {
    fhp_sim* s = nullptr;
    int rc = fhp_pool_member(pl, slot, &s);
    if (rc) return rc;
    return fhp_observe(s, FHP_OBS_BLOCKS, block, host_dst, bytes);
}

int fhp_pool_collect(fhp_pool* pl, uint32_t slot, uint32_t block, int32_t* host_dst,
                     size_t bytes) {
    fhp_sim* s = nullptr;
    int rc = fhp_pool_member(pl, slot, &s);
    if (rc) return rc;
    if (!host_dst) return fail(FHP_E_INVAL, "NULL destination");
    if (block == 0 || (block < 64 ? (64 % block) : (block % 64)))
        return fail(FHP_E_INVAL, "block %u must divide 64 or be a multiple of 64", block);
    const uint32_t bw = (s->L.W + block - 1) / block, bh = (s->L.H + block - 1) / block;
    const size_t need = (size_t)bw * bh * 3 * sizeof(int32_t);
    if (bytes < need) return fail(FHP_E_NOMEM, "destination of %zu bytes, %zu needed", bytes, need);
    if (need > s->lay.buf_words * sizeof(uint64_t))
        return fail(FHP_E_INVAL, "block %u too small for an asynchronous result", block);
    PoolSlot& ps = pl->slots[slot];
    if (!ps.collected) FHP_HIP_TRY(hipEventCreateWithFlags(&ps.collected, hipEventDisableTiming),
                                   "event");
    int32_t* stage = (int32_t*)s->buf[1 - s->cur];  // the idle buffer
    FHP_HIP_TRY(launch_observe_blocks(s->buf[s->cur], lattice_of(s), block, 0, bh, 0, bw, stage,
                                      s->st),
                "blocks");
    FHP_HIP_TRY(hipMemcpyAsync(host_dst, stage, need, hipMemcpyDeviceToHost, s->st), "copy");
    FHP_HIP_TRY(hipEventRecord(ps.collected, s->st), "event");
    return FHP_OK;
}

int fhp_pool_collected(fhp_pool* pl, uint32_t slot, int* ready) {
    if (!pl || !ready) return fail(FHP_E_INVAL, "NULL argument");
    if (slot >= pl->slots.size() || !pl->slots[slot].used)
        return fail(FHP_E_INVAL, "slot %u is not in use", slot);
    const PoolSlot& ps = pl->slots[slot];
    if (!ps.collected) return fail(FHP_E_STATE, "slot %u: no result was collected", slot);
    hipError_t e = hipEventQuery(ps.collected);
    if (e == hipErrorNotReady) {
        *ready = 0;
        return FHP_OK;
    }
    FHP_HIP_TRY(e, "event");
    *ready = 1;
    return FHP_OK;
}

int fhp_pool_release(fhp_pool* pl, uint32_t slot) {
    if (!pl) return fail(FHP_E_INVAL, "pool is NULL");
    if (slot >= pl->slots.size() || !pl->slots[slot].used)
        return fail(FHP_E_INVAL, "slot %u is not in use", slot);
    PoolSlot& s = pl->slots[slot];
    // No wait: work on this memory is already enqueued on the pool's stream,
    // and whatever reuses it is enqueued after it.
    pl->heap.release(s.heap_off, s.heap_words);
    pl->changed = 1;
    pl->bands_used -= s.sim.L.H / band_for(s.sim.L.H, pl->eng.band, pl->eng.depth);
    s.used = false;
    for (size_t k = 0; k < pl->finished.size(); k++)
        if (pl->finished[k] == slot) {
            pl->finished.erase(pl->finished.begin() + k);
            break;
        }
    return FHP_OK;
}

int fhp_pool_usage(const fhp_pool* pl, uint32_t* active, size_t* bytes_used, size_t* bytes_free) {
    if (!pl) return fail(FHP_E_INVAL, "pool is NULL");
    uint32_t n = 0;
    for (auto& s : pl->slots) n += s.used;
    if (active) *active = n;
    const size_t free_b = pl->heap.free_words() * 8;
    if (bytes_used) *bytes_used = pl->heap_words * 8 - free_b;
    if (bytes_free) *bytes_free = free_b;
    return FHP_OK;
}

int fhp_pool_sync(fhp_pool* pl) {
    if (!pl) return fail(FHP_E_INVAL, "pool is NULL");
    return engine_status(&pl->eng);
}

void fhp_pool_destroy(fhp_pool* pl) {
    if (!pl) return;
    (void)hipStreamSynchronize(pl->eng.st);
    for (auto& s : pl->slots)
        if (s.collected) (void)hipEventDestroy(s.collected);
    engine_free(&pl->eng);
    delete pl;
}

}  // extern "C"
