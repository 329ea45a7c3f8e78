// fhp_batch.hip -- many independent lattices of uneven sizes in one
// persistent launch (and the C ABI of batches).
//
// Work decomposition.  Every lattice (member) is cut into bands of T rows
// (T even, T | H), as in the single-lattice blocked kernel.  A band needs one
// thread per 64-node word of a row, i.e. wd = W/64 lanes; bands of lattices
// with the same (wd, T) are packed side by side into groups of one workgroup
// (floor(nt / wd) bands per group), so a wave can hold e.g. 32 bands of
// 128-wide lattices.  The horizontal carry exchange wraps inside each band's
// lane segment.
//
// Work items are (pass, group) pairs taken in pass-major order from a global
// counter by a persistent grid.  A band's pass p reads its own rows and the K
// rows on each side, i.e. the neighbouring bands' results of pass p-1, and
// overwrites the buffer those bands read in pass p-1; so item (p, band b)
// waits until bands b-1, b, b+1 have completed p passes (agent-scope
// release/acquire on per-band counters).  Items are taken in order and every
// taken item is held by a running workgroup, so the oldest unfinished item can
// always proceed.  The wait is bounded: on time-out the launch aborts and the
// host reports an error.  The last workgroup to leave advances every member's
// time and buffer index and resets the counters, so a launch can be replayed
// from a graph without host work in between.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fhp_device.h"
#include "fhp_internal.h"
#include "fhp_sweep.h"

namespace fhp {
namespace {

struct MemberDesc {
    uint64_t* buf[2];
    const uint64_t* S;   // obstacle plane or nullptr
    uint64_t ps;         // plane stride in words
    uint64_t t0;         // steps completed
    uint64_t key_chir, key_force, thr_force, chi_and, chi_or;
    uint32_t H, wd, walls, cur;
    uint32_t passes;     // passes this member may still run (0xffffffff: no limit)
    uint32_t done_off;   // first band counter
    uint32_t nbands, T;
};

struct GroupDesc {
    uint32_t first, nseg, wd, T;
};

struct BatchHeader {
    uint32_t queue;     // next work item
    uint32_t exited;    // workgroups that left the launch
    uint32_t status;    // nonzero: a dependency wait timed out
    uint32_t n_groups, passes, n_members, n_done, K;
};

constexpr uint32_t kNoLimit = 0xffffffffu;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint32_t load_acquire(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int K, bool FORCE, bool MASK>
__global__ void __launch_bounds__(512) k_batch(BatchHeader* __restrict__ hdr,
                                               MemberDesc* __restrict__ members,
                                               const GroupDesc* __restrict__ groups,
                                               const uint32_t* __restrict__ seg_member,
                                               const uint32_t* __restrict__ seg_band,
                                               uint32_t* __restrict__ done) {
    extern __shared__ uint32_t xch[];  // 2 carry slots x nt, then one broadcast word
    const uint32_t nt = blockDim.x;
    const uint32_t lane = threadIdx.x;
    uint32_t* bcast = xch + 2 * nt;
    const uint32_t n_groups = hdr->n_groups;
    const uint32_t passes = hdr->passes;
    const uint32_t n_items = n_groups * passes;
    uint32_t slot = 0;

    for (;;) {
        if (lane == 0) bcast[0] = atomicAdd(&hdr->queue, 1u);
        __syncthreads();
        const uint32_t item = bcast[0];
        __syncthreads();
        if (item >= n_items) break;
        const uint32_t p = item / n_groups;
        const GroupDesc G = groups[item - p * n_groups];
        const uint32_t seg = lane / G.wd;
        const uint32_t w = lane - seg * G.wd;
        const bool valid = seg < G.nseg;
        const uint32_t sidx = G.first + (valid ? seg : 0);
        const uint32_t m = seg_member[sidx];
        const uint32_t b = seg_band[sidx];
        const MemberDesc& M = members[m];
        const bool active = valid && p < M.passes;
        if (!__syncthreads_or(active)) continue;

        if (p > 0) {  // wait for the neighbouring bands' previous pass
            const uint32_t nb = M.nbands;
            const uint32_t bm = b ? b - 1 : nb - 1, bq = (b + 1 == nb) ? 0 : b + 1;
            const uint32_t* dm = done + M.done_off;
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
        // single-lattice blocked kernel with per-lane lattice parameters.
        const uint32_t H = M.H, wd = G.wd, T = G.T;
        const uint32_t base = seg * wd;
        const uint32_t wl = base + (w ? w - 1 : wd - 1);
        const uint32_t wr = base + ((w + 1 == wd) ? 0 : w + 1);
        const uint32_t cur = (M.cur + p) & 1;
        const uint64_t* in = M.buf[cur];
        uint64_t* out = M.buf[cur ^ 1];
        const uint64_t* S = M.S;
        const uint64_t ps = M.ps;
        const uint32_t walls = M.walls;
        const uint64_t tp = M.t0 + (uint64_t)p * K;
        const uint64_t chi_and = M.chi_and, chi_or = M.chi_or, thr = M.thr_force;
        const uint64_t base_chi = word_base(M.key_chir, w);
        const uint64_t base_frc = word_base(M.key_force, w);
        const int y0 = (int)(b * T);
        const int n_iter = (int)T + 2 * K;

        auto wrap_row = [&](int r) __attribute__((always_inline)) -> uint32_t {
            // r lies in [-K, H + K) and K <= H
            return (uint32_t)(r < 0 ? r + (int)H : (r >= (int)H ? r - (int)H : r));
        };
        auto load = [&](uint32_t y, Row& x) __attribute__((always_inline)) {
            const size_t off = (size_t)y * wd + w;
#pragma unroll
            for (int c = 0; c < 7; c++) x.p[c] = in[c * ps + off];
            if (MASK) x.s = S ? S[off] : 0ull;
        };

        uint64_t a3[K + 1], a4[K + 1], bp[K + 1][7], bs[K + 1];
        uint32_t ac[K + 1], bc[K + 1];
        auto push = [&](auto lc, const Row& x) __attribute__((always_inline)) {
            constexpr int l = decltype(lc)::value;
            a3[l] = bp[l][3];
            a4[l] = bp[l][4];
            ac[l] = bc[l];
#pragma unroll
            for (int c = 0; c < 7; c++) bp[l][c] = x.p[c];
            bs[l] = x.s;
            bc[l] = x.c;
        };
        Row nxt;
        load(wrap_row(y0 - K), nxt);

        auto body = [&](int i, auto full_c, auto par_c) __attribute__((always_inline)) {
            constexpr bool FULL = decltype(full_c)::value;
            constexpr int PAR = decltype(par_c)::value;
            const int r = y0 - K + i;
            const uint32_t y = wrap_row(r);
            Row X = nxt;
            load((i + 1 < n_iter) ? wrap_row(r + 1) : y, nxt);
            uint64_t s = MASK ? X.s : 0ull;
            if (walls && (y == 0 || y == H - 1)) s = ~0ull;
            X.s = s;
            exchange(xch, slot, nt, lane, wl, wr, X);
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
                const uint32_t rho = wrap_row(r - l);
                constexpr bool odd = ((PAR + K + l) & 1) != 0;  // y0 even: parity of rho
                uint64_t n[7];
                stream_in<odd>(a3[l], a4[l], ac[l], bp[l], bc[l], X, n);
                const uint64_t sw = bs[l];
                const uint64_t R = row_term(tp + (uint64_t)(l - 1), rho);
                const uint64_t chi = (mix64(base_chi + R) & chi_and) | chi_or;
                const uint64_t coin = FORCE ? coin_word(mix64(base_frc + R), thr) : 0ull;
                Row Y;
                update(n, sw, chi, coin, Y.p);
                Y.s = sw;
                push(lc, X);
                if (l < K) {
                    exchange(xch, slot, nt, lane, wl, wr, Y);
                    X = Y;
                } else if (active) {
                    const size_t off = (size_t)rho * wd + w;
#pragma unroll
                    for (int c = 0; c < 7; c++) out[c * ps + off] = Y.p[c];
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
                __hip_atomic_fetch_add(done + M.done_off + b, 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // The last workgroup out advances the members and resets the counters.
    __syncthreads();
    if (lane == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bcast[0] = atomicAdd(&hdr->exited, 1u);
    }
    __syncthreads();
    if (bcast[0] == gridDim.x - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (hdr->status == 0) {
            for (uint32_t k = lane; k < hdr->n_members; k += nt) {
                MemberDesc& M = members[k];
                const uint32_t eff = min(passes, M.passes);
                M.t0 += (uint64_t)eff * K;
                M.cur ^= eff & 1;
                if (M.passes != kNoLimit) M.passes -= eff;
            }
        }
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

template <int K, bool FORCE, bool MASK>
hipError_t launch_batch_t(BatchHeader* hdr, MemberDesc* members, const GroupDesc* groups,
                          const uint32_t* seg_member, const uint32_t* seg_band, uint32_t* done,
                          uint32_t grid, uint32_t nt, hipStream_t st) {
    hipLaunchKernelGGL((k_batch<K, FORCE, MASK>), dim3(grid), dim3(nt),
                       (2 * nt + 1) * sizeof(uint32_t), st, hdr, members, groups, seg_member,
                       seg_band, done);
    return hipGetLastError();
}

using BatchLaunch = hipError_t (*)(BatchHeader*, MemberDesc*, const GroupDesc*, const uint32_t*,
                                   const uint32_t*, uint32_t*, uint32_t, uint32_t, hipStream_t);
using BatchKernel = const void*;

template <int K>
void pick(bool force, bool mask, BatchLaunch* fn, BatchKernel* kern) {
    if (force && mask) {
        *fn = launch_batch_t<K, true, true>;
        *kern = (const void*)k_batch<K, true, true>;
    } else if (force) {
        *fn = launch_batch_t<K, true, false>;
        *kern = (const void*)k_batch<K, true, false>;
    } else if (mask) {
        *fn = launch_batch_t<K, false, true>;
        *kern = (const void*)k_batch<K, false, true>;
    } else {
        *fn = launch_batch_t<K, false, false>;
        *kern = (const void*)k_batch<K, false, false>;
    }
}

bool pick_kernel(uint32_t K, bool force, bool mask, BatchLaunch* fn, BatchKernel* kern) {
    switch (K) {
        case 1: pick<1>(force, mask, fn, kern); return true;
        case 2: pick<2>(force, mask, fn, kern); return true;
        case 3: pick<3>(force, mask, fn, kern); return true;
        case 4: pick<4>(force, mask, fn, kern); return true;
        default: return false;
    }
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

}  // namespace
}  // namespace fhp

using namespace fhp;

struct fhp_batch {
    uint32_t n;
    fhp_sim* sims;
    hipStream_t st;
    // device tables
    BatchHeader* hdr;
    MemberDesc* members;
    GroupDesc* groups;
    uint32_t* seg_member;
    uint32_t* seg_band;
    uint32_t* done;
    uint64_t* aux;
    size_t max_segs;
    // tiling
    uint32_t depth, band, nt, passes_per_launch;
    int use_graph;
    bool force, mask;
    bool tables_dirty;  // member table or grouping must be uploaded before the next launch
    int dirty_flag;     // set by member views when they are changed individually
    uint32_t n_groups, n_done;
    uint32_t grid;      // persistent workgroups of the current kernel
    // cached graph of one launch sequence
    hipGraphExec_t graph;
    uint32_t graph_K, graph_passes, graph_launches;
};

namespace {

struct BatchLayout {
    std::vector<size_t> member_off;  // word offsets of each member's planes
    size_t aux_off, hdr_off, members_off, groups_off, segm_off, segb_off, done_off;
    size_t max_segs, total_bytes;
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
        if (ps[i].height < 2 * FHP_MAX_DEPTH)
            return fail(FHP_E_INVAL, "member %u: height %u below %u", i, ps[i].height,
                        2 * FHP_MAX_DEPTH);
        bl->member_off[i] = off;
        off += layout_for(ps[i].width, ps[i].height).aux_off;  // planes and S, no aux
        off = round_up(off, 32);
        segs += ps[i].height / 2;  // bands of at least 2 rows
    }
    bl->aux_off = off;
    off += kAuxWords;
    const size_t w = sizeof(uint64_t);
    bl->hdr_off = off;
    off += round_up(sizeof(BatchHeader), 256) / w;
    bl->members_off = off;
    off += round_up((size_t)n * sizeof(MemberDesc), 256) / w;
    bl->groups_off = off;
    off += round_up(segs * sizeof(GroupDesc), 256) / w;
    bl->segm_off = off;
    off += round_up(segs * 4, 256) / w;
    bl->segb_off = off;
    off += round_up(segs * 4, 256) / w;
    bl->done_off = off;
    off += round_up(segs * 4, 256) / w;
    bl->max_segs = segs;
    bl->total_bytes = off * w;
    return FHP_OK;
}

// Rebuilds the member and group tables for the current tiling and uploads them.
int build_tables(fhp_batch* b) {
    FHP_HIP_TRY(hipStreamSynchronize(b->st), "sync");
    std::vector<MemberDesc> mem(b->n);
    struct Seg {
        uint32_t wd, T, m, band;
    };
    std::vector<Seg> segs;
    uint32_t done = 0, max_wd = 0;
    for (uint32_t i = 0; i < b->n; i++) {
        const fhp_sim* s = &b->sims[i];
        MemberDesc& M = mem[i];
        memset(&M, 0, sizeof(M));
        M.buf[0] = s->buf[0];
        M.buf[1] = s->buf[1];
        M.S = s->has_mask ? s->S : nullptr;
        M.ps = s->L.ps;
        M.t0 = s->t;
        M.key_chir = s->D.key_chir;
        M.key_force = s->D.key_force;
        M.thr_force = s->D.thr_force;
        M.chi_and = (s->D.chir_mode == FHP_CHIR_HASH) ? ~0ull : 0ull;
        M.chi_or = (s->D.chir_mode == FHP_CHIR_ONE) ? ~0ull : 0ull;
        M.H = s->L.H;
        M.wd = s->L.wd;
        M.walls = s->L.walls;
        M.cur = (uint32_t)s->cur;
        M.passes = kNoLimit;
        M.T = band_for(s->L.H, b->band, b->depth);
        M.nbands = s->L.H / M.T;
        M.done_off = done;
        done += M.nbands;
        for (uint32_t k = 0; k < M.nbands; k++) segs.push_back({M.wd, M.T, i, k});
        if (M.wd > max_wd) max_wd = M.wd;
    }
    uint32_t nt = b->nt ? b->nt : 64;
    const uint32_t need = (max_wd + 63) / 64 * 64;
    if (nt < need) nt = need;
    // group bands of equal (wd, T); larger work first
    std::stable_sort(segs.begin(), segs.end(), [](const Seg& x, const Seg& y) {
        if (x.wd != y.wd) return x.wd > y.wd;
        return x.T > y.T;
    });
    std::vector<GroupDesc> groups;
    std::vector<uint32_t> sm(segs.size()), sb(segs.size());
    for (size_t k = 0; k < segs.size();) {
        const uint32_t cap = nt / segs[k].wd;
        GroupDesc g;
        g.first = (uint32_t)k;
        g.wd = segs[k].wd;
        g.T = segs[k].T;
        g.nseg = 0;
        while (k < segs.size() && g.nseg < cap && segs[k].wd == g.wd && segs[k].T == g.T) {
            sm[k] = segs[k].m;
            sb[k] = segs[k].band;
            g.nseg++;
            k++;
        }
        groups.push_back(g);
    }
    std::stable_sort(groups.begin(), groups.end(), [](const GroupDesc& x, const GroupDesc& y) {
        return (uint64_t)x.nseg * x.wd * x.T > (uint64_t)y.nseg * y.wd * y.T;
    });
    BatchHeader h;
    memset(&h, 0, sizeof(h));
    h.n_groups = (uint32_t)groups.size();
    h.n_members = b->n;
    h.n_done = done;
    FHP_HIP_TRY(hipMemcpy(b->hdr, &h, sizeof(h), hipMemcpyHostToDevice), "upload");
    FHP_HIP_TRY(hipMemcpy(b->members, mem.data(), mem.size() * sizeof(MemberDesc),
                          hipMemcpyHostToDevice), "upload");
    FHP_HIP_TRY(hipMemcpy(b->groups, groups.data(), groups.size() * sizeof(GroupDesc),
                          hipMemcpyHostToDevice), "upload");
    FHP_HIP_TRY(hipMemcpy(b->seg_member, sm.data(), sm.size() * 4, hipMemcpyHostToDevice), "upload");
    FHP_HIP_TRY(hipMemcpy(b->seg_band, sb.data(), sb.size() * 4, hipMemcpyHostToDevice), "upload");
    FHP_HIP_TRY(launch_fill_u64((uint64_t*)b->done, (done + 1) / 2, 0, b->st), "clear");
    FHP_HIP_TRY(hipStreamSynchronize(b->st), "sync");
    b->nt = nt;
    b->n_groups = h.n_groups;
    b->n_done = done;
    b->force = b->mask = false;
    for (uint32_t i = 0; i < b->n; i++) {
        b->force |= b->sims[i].D.thr_force != 0;
        b->mask |= b->sims[i].has_mask != 0;
    }
    b->tables_dirty = false;
    b->dirty_flag = 0;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return FHP_OK;
}

int kernel_for(fhp_batch* b, uint32_t K, BatchLaunch* fn) {
    BatchKernel kern;
    if (!pick_kernel(K, b->force, b->mask, fn, &kern)) return fail(FHP_E_INVAL, "depth %u", K);
    int per_cu = 0, dev = 0, cus = 0;
    FHP_HIP_TRY(hipGetDevice(&dev), "device");
    FHP_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr");
    FHP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)b->nt,
                                                            (2 * b->nt + 1) * sizeof(uint32_t)),
                "occupancy");
    if (per_cu < 1) per_cu = 1;
    b->grid = (uint32_t)(per_cu * cus);
    return FHP_OK;
}

// Enqueues `launches` launches of `passes` passes of depth K.
int enqueue(fhp_batch* b, uint32_t K, uint32_t passes, uint32_t launches) {
    BatchLaunch fn;
    int rc = kernel_for(b, K, &fn);
    if (rc) return rc;
    hipLaunchKernelGGL(k_batch_header, dim3(1), dim3(1), 0, b->st, b->hdr, passes, K);
    FHP_HIP_TRY(hipGetLastError(), "launch");
    for (uint32_t k = 0; k < launches; k++)
        FHP_HIP_TRY(fn(b->hdr, b->members, b->groups, b->seg_member, b->seg_band, b->done,
                       b->grid, b->nt, b->st), "launch");
    return FHP_OK;
}

int launch_graphless(fhp_batch* b, uint32_t K, uint32_t passes, uint32_t launches) {
    return enqueue(b, K, passes, launches);
}

int launch_graph(fhp_batch* b, uint32_t K, uint32_t passes, uint32_t launches) {
    if (!b->graph || b->graph_K != K || b->graph_passes != passes || b->graph_launches != launches) {
        if (b->graph) {
            (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
        }
        hipGraph_t g = nullptr;
        FHP_HIP_TRY(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "capture");
        int rc = enqueue(b, K, passes, launches);
        hipError_t e = hipStreamEndCapture(b->st, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->graph = nullptr;
            return hip_fail(e, "instantiate");
        }
        b->graph_K = K;
        b->graph_passes = passes;
        b->graph_launches = launches;
    }
    FHP_HIP_TRY(hipGraphLaunch(b->graph, b->st), "graph launch");
    return FHP_OK;
}

}  // namespace

extern "C" {

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
    fhp_batch* b = (fhp_batch*)calloc(1, sizeof(fhp_batch));
    if (!b) return fail(FHP_E_NOMEM, "host allocation failed");
    b->sims = (fhp_sim*)calloc(n, sizeof(fhp_sim));
    if (!b->sims) {
        free(b);
        return fail(FHP_E_NOMEM, "host allocation failed");
    }
    uint64_t* ws = (uint64_t*)dev_ws;
    b->n = n;
    b->st = (hipStream_t)hip_stream;
    b->aux = ws + bl.aux_off;
    b->hdr = (BatchHeader*)(ws + bl.hdr_off);
    b->members = (MemberDesc*)(ws + bl.members_off);
    b->groups = (GroupDesc*)(ws + bl.groups_off);
    b->seg_member = (uint32_t*)(ws + bl.segm_off);
    b->seg_band = (uint32_t*)(ws + bl.segb_off);
    b->done = (uint32_t*)(ws + bl.done_off);
    b->max_segs = bl.max_segs;
    b->depth = FHP_MAX_DEPTH;
    b->band = 32;
    b->nt = 0;
    b->passes_per_launch = 1;
    b->use_graph = 1;
    for (uint32_t i = 0; i < n && !rc; i++) {
        const Layout lay = layout_for(ps[i].width, ps[i].height);
        rc = sim_setup(&b->sims[i], &ps[i], ws + bl.member_off[i], lay, b->aux, b->st);
        b->sims[i].owner = b;
        b->sims[i].changed = &b->dirty_flag;
    }
    if (!rc) rc = build_tables(b);
    if (rc) {
        free(b->sims);
        free(b);
        return rc;
    }
    *out = b;
    return FHP_OK;
}

int fhp_batch_set_tiling(fhp_batch* b, uint32_t depth, uint32_t band, uint32_t group_threads,
                         uint32_t passes_per_launch) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    if (depth > FHP_MAX_DEPTH) return fail(FHP_E_INVAL, "depth %u above %u", depth, FHP_MAX_DEPTH);
    if (group_threads % 64 || group_threads > 512)
        return fail(FHP_E_INVAL, "group_threads %u: a multiple of 64 up to 512", group_threads);
    b->depth = depth ? depth : FHP_MAX_DEPTH;
    b->band = band ? band : 32;
    b->nt = group_threads;
    b->passes_per_launch = passes_per_launch;  // 0: all passes of a call in one launch
    return build_tables(b);
}

int fhp_batch_set_graph(fhp_batch* b, int enable) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    b->use_graph = enable != 0;
    return FHP_OK;
}

int fhp_batch_step(fhp_batch* b, uint64_t n) {
    if (!b) return fail(FHP_E_INVAL, "batch is NULL");
    for (uint32_t i = 0; i < b->n; i++)
        if (b->sims[i].t + n >= kTimeLimit)
            return fail(FHP_E_STATE, "member %u: time would reach 2^24", i);
    if (b->tables_dirty || b->dirty_flag) {
        int rc = build_tables(b);
        if (rc) return rc;
    }
    const uint32_t K = b->depth;
    const uint64_t full = n / K;
    const uint32_t rest = (uint32_t)(n % K);
    if (full) {
        uint32_t per = b->passes_per_launch ? b->passes_per_launch : (uint32_t)full;
        if (per > full) per = (uint32_t)full;
        const uint32_t launches = (uint32_t)(full / per);
        const uint32_t tail = (uint32_t)(full % per);
        int rc = b->use_graph ? launch_graph(b, K, per, launches) : launch_graphless(b, K, per, launches);
        if (rc) return rc;
        if (tail) {
            rc = launch_graphless(b, K, tail, 1);
            if (rc) return rc;
        }
    }
    if (rest) {
        int rc = launch_graphless(b, rest, 1, 1);
        if (rc) return rc;
    }
    // host mirror of the device-side bookkeeping
    for (uint32_t i = 0; i < b->n; i++) {
        fhp_sim* s = &b->sims[i];
        const uint64_t passes = full + (rest ? 1 : 0);
        s->t += n;
        s->cur ^= (int)(passes & 1);
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
    FHP_HIP_TRY(hipStreamSynchronize(b->st), "sync");
    uint32_t status = 0;
    FHP_HIP_TRY(hipMemcpy(&status, &b->hdr->status, 4, hipMemcpyDeviceToHost), "copy");
    if (status) return fail(FHP_E_DEVICE, "batch launch aborted: a dependency wait timed out");
    return FHP_OK;
}

void fhp_batch_destroy(fhp_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->st);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    free(b->sims);
    free(b);
}

}  // extern "C"
