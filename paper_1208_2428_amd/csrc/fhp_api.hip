// fhp_api.hip -- the single-lattice part of the C ABI declared in include/fhp.h.
//
// Host-side bookkeeping only: parameter validation, the workspace layout,
// the time counter and the order of kernel launches.  Every step of the
// dynamics runs in the kernels of fhp_kernels.hip / fhp_stepk.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fhp_device.h"
#include "fhp_internal.h"

namespace fhp {

namespace {
thread_local char g_err[512] = "";

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bytes of the idle buffer, used as staging for host transfers.
size_t staging_bytes(const fhp_sim* s) { return s->lay.buf_words * sizeof(uint64_t); }

int refresh_has_mask(fhp_sim* s) {
    FHP_HIP_TRY(launch_fill_u64(s->aux, 1, 0, s->st), "clear aux");
    FHP_HIP_TRY(launch_or_reduce(s->S, (size_t)s->L.H * s->L.wd, s->aux, s->st), "mask reduce");
    uint64_t any = 0;
    FHP_HIP_TRY(hipMemcpyAsync(&any, s->aux, sizeof(any), hipMemcpyDeviceToHost, s->st), "copy");
    FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");
    s->has_mask = any != 0;
    return FHP_OK;
}

// Uploads W*H bytes in row chunks through the idle buffer and packs them.
int upload_bytes(fhp_sim* s, const uint8_t* host, int mask_only) {
    const uint32_t W = s->L.W, H = s->L.H;
    uint8_t* stage = (uint8_t*)s->buf[1 - s->cur];
    uint32_t rows = (uint32_t)(staging_bytes(s) / W);
    if (rows > H) rows = H;
    for (uint32_t r0 = 0; r0 < H; r0 += rows) {
        const uint32_t n = (r0 + rows <= H) ? rows : H - r0;
        FHP_HIP_TRY(hipMemcpyAsync(stage, host + (size_t)r0 * W, (size_t)n * W,
                                   hipMemcpyHostToDevice, s->st), "upload");
        FHP_HIP_TRY(launch_pack(stage, r0, n, s->L, s->buf[s->cur], s->S, mask_only, s->st),
                    "pack");
        FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");  // the stage is reused
    }
    return FHP_OK;
}
}  // namespace

namespace {
struct FaultPlan {
    bool launch = false, alloc = false;
    long long launch_after = 0;
    long long launches = 0;
};
FaultPlan& fault_plan() {
    static FaultPlan plan = [] {
        FaultPlan f;
        const char* v = getenv("FHP_FAULT");
        if (!v) return f;
        if (!strncmp(v, "launch", 6)) {
            f.launch = true;
            if (v[6] == '@') f.launch_after = atoll(v + 7);
        } else if (!strcmp(v, "alloc")) {
            f.alloc = true;
        }
        return f;
    }();
    return plan;
}
}  // namespace

bool fault_launch() {
    FaultPlan& f = fault_plan();
    return f.launch && f.launches++ >= f.launch_after;
}

bool fault_alloc() { return fault_plan().alloc; }

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(FHP_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int validate(const fhp_params* p) {
    if (!p) return fail(FHP_E_INVAL, "params is NULL");
    if (p->abi_version != FHP_ABI_VERSION)
        return fail(FHP_E_INVAL, "abi_version %u, library speaks %u", p->abi_version, FHP_ABI_VERSION);
    if (p->width == 0 || p->width % 64 || p->width >= (1u << 20))
        return fail(FHP_E_INVAL, "width %u must be a positive multiple of 64 below 2^20", p->width);
    if (p->height < 2 || p->height % 2 || p->height >= (1u << 20))
        return fail(FHP_E_INVAL, "height %u must be even, >= 2 and below 2^20", p->height);
    if ((uint64_t)p->width * p->height >= (1ull << 35))
        return fail(FHP_E_INVAL, "lattice of %llu nodes: a bit-plane must stay below 4 GiB",
                    (unsigned long long)p->width * p->height);
    if (p->walls > FHP_WALLS_CHANNEL) return fail(FHP_E_INVAL, "walls %u unknown", p->walls);
    if (p->chirality > FHP_CHIR_ONE) return fail(FHP_E_INVAL, "chirality %u unknown", p->chirality);
    if (p->rules > FHP_RULES_FHP3) return fail(FHP_E_INVAL, "rule set %u unknown", p->rules);
    if (!(p->fill >= 0.0 && p->fill <= 1.0)) return fail(FHP_E_INVAL, "fill must lie in [0, 1]");
    if (!(p->force_rate >= 0.0 && p->force_rate < 1.0 / 64.0))
        return fail(FHP_E_INVAL, "force_rate must lie in [0, 1/64)");
    return FHP_OK;
}

Layout layout_for(uint32_t W, uint32_t H) {
    Layout l;
    l.plane_words = round_up((size_t)H * (W / 64), 32);  // 256-byte multiple
    l.buf_words = 7 * l.plane_words;
    l.s_off = 2 * l.buf_words;
    l.aux_off = l.s_off + l.plane_words;
    l.total_bytes = (l.aux_off + kAuxWords) * sizeof(uint64_t);
    return l;
}

// Default band height of the blocked kernel, from occupancy: the largest even
// height up to 32 rows whose bands give every SIMD two waves (a band's
// workgroup holds ceil(wd / 64) waves); if that takes bands of 2 rows, the
// largest that gives every SIMD one wave (*one_wave set).  Shorter bands cost
// halo work (1 + (K - 1) / T level-rows per row, K halo rows loaded on each
// side), fewer waves leave SIMDs idle.  Measured at K = 5 (node-updates/s by
// band height): 16384^2 (four waves per band) 32 rows 9.9e12, 24-64 rows
// 7.7e12-9.4e12; 8192^2 (two) 4, 8, 16, 32 rows 5.10e12, 7.54e12, 5.37e12,
// 4.28e12; 4096^2 (one) 2, 4, 8, 32 rows 2.98e12, 3.61e12, 2.88e12, 1.20e12;
// 2048^2 (one, half used) 2, 4 rows 1.14e12, 0.93e12.  The rule picks 32, 8, 4
// and 2.
static uint32_t band_rule(uint32_t H, uint32_t wd, uint32_t simds, bool* one_wave) {
    const uint64_t waves = (wd + 63) / 64;
    auto largest = [&](uint64_t need) -> uint32_t {  // 0 when no height gives `need` waves
        for (uint32_t T = 32; T >= 2; T -= 2)
            if ((uint64_t)((H + T - 1) / T) * waves >= need) return T;
        return 0;
    };
    uint32_t T = largest(2ull * simds);
    *one_wave = T < 4;
    if (*one_wave) {
        const uint32_t T1 = largest(simds);
        T = T1 > 2 ? T1 : 2;
    }
    return H < T ? H : T;
}

uint32_t default_band(uint32_t H, uint32_t wd, uint32_t simds) {
    bool one_wave;
    return band_rule(H, wd, simds, &one_wave);
}

// Default depth from the default band: 3 on lattices too small to give every
// SIMD two waves, where a pass is bound by the latency of its level chain
// rather than by memory (25% less halo work per step than 5 at 4-row bands):
// 4096^2 channel flow at K = 2..5 measured 4.87e12, 4.95e12, 4.72e12 and
// 4.56e12 node-updates/s, 2048^2 at 2-row bands 1.45e12, 1.49e12, 1.40e12 and
// 1.29e12.  4 where the bands are 8 rows or shorter (8192^2 at 8-row bands
// 8.26e12 at K = 4, 8.04e12 at 5; 8192 x 4096 at 4-row bands 5.81e12 and
// 5.52e12), FHP_MAX_DEPTH otherwise: the deepest pass whose register queue
// fits without spilling, which moves 18% fewer bytes per step than depth 4
// for 3% more halo work (16384^2 at 32-row bands: 1.07e13 at 5, 0.99e13 at
// 4).  Rows wider than the blocked kernel takes run single steps.
uint32_t default_depth(uint32_t H, uint32_t wd, uint32_t simds) {
    if (wd > kMaxBlockedWords) return 1;
    bool one_wave;
    const uint32_t T = band_rule(H, wd, simds, &one_wave);
    if (one_wave) return 3;
    return T <= 8 ? 4 : FHP_MAX_DEPTH;
}

Dyn dyn_for(const fhp_params* p) {
    Dyn D;
    D.key_chir = hash64(p->seed, kTagChir);
    D.key_force = hash64(p->seed, kTagForce);
    D.thr_force = (uint64_t)floor(p->force_rate * 274877906944.0);  // f * 2^38
    D.chir_mode = p->chirality;
    D.rules = p->rules;
    return D;
}

uint32_t device_simds() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();  // not left for the next launch check to report
        cus = 256;                // the MI355X's compute units
    }
    return 4 * (uint32_t)cus;
}

Lattice lattice_of(const fhp_sim* s) {
    Lattice L = s->L;
    L.S = s->has_mask ? s->S : nullptr;
    return L;
}

int sim_setup(fhp_sim* s, const fhp_params* p, uint64_t* planes, const Layout& lay,
              uint64_t* aux, hipStream_t st, bool sync) {
    s->p = *p;
    s->p.solid = nullptr;
    s->lay = lay;
    s->buf[0] = planes;
    s->buf[1] = planes + lay.buf_words;
    s->S = planes + lay.s_off;
    s->aux = aux;
    s->cur = 0;
    s->t = 0;
    s->st = st;
    s->L.W = p->width;
    s->L.H = p->height;
    s->L.wd = p->width / 64;
    s->L.ps = lay.plane_words;
    s->L.walls = p->walls == FHP_WALLS_CHANNEL;
    s->D = dyn_for(p);
    s->simds = device_simds();
    s->depth = default_depth(s->L.H, s->L.wd, s->simds);
    s->band = 0;

    FHP_HIP_TRY(launch_fill_u64(s->S, lay.plane_words, 0, st), "clear solid plane");
    s->has_mask = 0;
    if (p->solid) {
        int r = upload_bytes(s, p->solid, 1);
        if (r) return r;
        r = refresh_has_mask(s);
        if (r) return r;
    }
    const uint64_t thr_fill = (uint64_t)floor(p->fill * 4294967296.0);  // fill * 2^32
    FHP_HIP_TRY(launch_init(s->buf[0], lattice_of(s), hash64(p->seed, kTagInit), thr_fill, st),
                "init");
    if (sync) FHP_HIP_TRY(hipStreamSynchronize(st), "sync");
    return FHP_OK;
}

}  // namespace fhp

using namespace fhp;

extern "C" {

const char* fhp_last_error(void) { return fhp::g_err; }

int fhp_workspace_bytes(const fhp_params* p, size_t* bytes) {
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return fail(FHP_E_INVAL, "bytes is NULL");
    *bytes = layout_for(p->width, p->height).total_bytes;
    return FHP_OK;
}

int fhp_create(const fhp_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, fhp_sim** out) {
    int rc = validate(p);
    if (rc) return rc;
    if (!out) return fail(FHP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!dev_ws || ((uintptr_t)dev_ws & 255))
        return fail(FHP_E_INVAL, "workspace must be a non-NULL 256-byte aligned device pointer");
    Layout lay = layout_for(p->width, p->height);
    if (ws_bytes < lay.total_bytes)
        return fail(FHP_E_NOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, lay.total_bytes);
    fhp_sim* s = (fhp_sim*)calloc(1, sizeof(fhp_sim));
    if (!s) return fail(FHP_E_NOMEM, "host allocation failed");
    uint64_t* ws = (uint64_t*)dev_ws;
    rc = sim_setup(s, p, ws, lay, ws + lay.aux_off, (hipStream_t)hip_stream);
    if (rc) {
        free(s);
        return rc;
    }
    *out = s;
    return FHP_OK;
}

int fhp_set_depth(fhp_sim* s, uint32_t k) {
    if (!s) return fail(FHP_E_INVAL, "sim is NULL");
    if (k > FHP_MAX_DEPTH) return fail(FHP_E_INVAL, "depth %u above %u", k, FHP_MAX_DEPTH);
    if (k > 1 && s->L.wd > kMaxBlockedWords)
        return fail(FHP_E_INVAL, "depth %u needs width <= %u", k, 64 * kMaxBlockedWords);
    s->depth = k ? k : default_depth(s->L.H, s->L.wd, s->simds);
    return FHP_OK;
}

int fhp_set_band(fhp_sim* s, uint32_t rows) {
    if (!s) return fail(FHP_E_INVAL, "sim is NULL");
    if (rows > s->L.H) return fail(FHP_E_INVAL, "band of %u rows exceeds height %u", rows, s->L.H);
    s->band = rows;
    return FHP_OK;
}

int fhp_get_band(const fhp_sim* s, uint32_t* rows) {
    if (!s || !rows) return fail(FHP_E_INVAL, "NULL argument");
    *rows = s->band ? s->band : default_band(s->L.H, s->L.wd, s->simds);
    return FHP_OK;
}

int fhp_get_depth(const fhp_sim* s, uint32_t* k) {
    if (!s || !k) return fail(FHP_E_INVAL, "NULL argument");
    *k = s->depth;
    return FHP_OK;
}

int fhp_step(fhp_sim* s, uint64_t n) {
    if (!s) return fail(FHP_E_INVAL, "sim is NULL");
    if (n >= kTimeLimit || s->t + n >= kTimeLimit)
        return fail(FHP_E_STATE, "time %llu + %llu would reach 2^24",
                    (unsigned long long)s->t, (unsigned long long)n);
    if (s->changed && n) *s->changed = 1;
    const Lattice L = lattice_of(s);
    uint32_t depth = s->depth;
    if (s->D.rules == FHP_RULES_FHP3 && depth > kMaxDepthFHP3) depth = kMaxDepthFHP3;
    const uint32_t T = s->band ? s->band : default_band(s->L.H, s->L.wd, s->simds);
    while (n > 0) {
        uint32_t k = (n >= depth) ? depth : (uint32_t)n;
        if (fault_launch()) return hip_fail(hipErrorLaunchFailure, "step (injected by FHP_FAULT)");
        if (k == 1)
            FHP_HIP_TRY(launch_step1(s->buf[s->cur], s->buf[1 - s->cur], L, s->D, s->t, s->st),
                        "step");
        else
            FHP_HIP_TRY(
                launch_stepk(k, s->buf[s->cur], s->buf[1 - s->cur], L, s->D, s->t, T, s->simds,
                             s->st),
                "step");
        s->cur ^= 1;
        s->t += k;
        n -= k;
    }
    return FHP_OK;
}

int fhp_observe(fhp_sim* s, int kind, uint32_t block, void* host_dst, size_t dst_bytes) {
    if (!s || !host_dst) return fail(FHP_E_INVAL, "NULL argument");
    const Lattice L = lattice_of(s);
    const uint64_t* planes = s->buf[s->cur];
    if (kind == FHP_OBS_GLOBAL || kind == FHP_OBS_DIGEST) {
        const size_t need = (kind == FHP_OBS_GLOBAL ? 11 : 1) * sizeof(uint64_t);
        if (dst_bytes < need)
            return fail(FHP_E_NOMEM, "destination of %zu bytes, %zu needed", dst_bytes, need);
        FHP_HIP_TRY(launch_fill_u64(s->aux, 11, 0, s->st), "clear aux");
        if (kind == FHP_OBS_GLOBAL)
            FHP_HIP_TRY(launch_observe_global(planes, L, s->aux, s->st), "observe");
        else
            FHP_HIP_TRY(launch_digest(planes, L, s->aux, s->st), "digest");
        FHP_HIP_TRY(hipMemcpyAsync(host_dst, s->aux, need, hipMemcpyDeviceToHost, s->st), "copy");
        FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");
        return FHP_OK;
    }
    if (kind == FHP_OBS_ROWS) {
        const size_t row_bytes = 3 * sizeof(int64_t);
        if (dst_bytes < row_bytes * L.H)
            return fail(FHP_E_NOMEM, "destination of %zu bytes, %zu needed", dst_bytes,
                        row_bytes * L.H);
        int64_t* stage = (int64_t*)s->buf[1 - s->cur];
        uint32_t rows = (uint32_t)(staging_bytes(s) / row_bytes);
        if (rows > L.H) rows = L.H;
        for (uint32_t r0 = 0; r0 < L.H; r0 += rows) {
            const uint32_t n = (r0 + rows <= L.H) ? rows : L.H - r0;
            FHP_HIP_TRY(launch_observe_rows(planes, L, r0, n, stage, s->st), "rows");
            FHP_HIP_TRY(hipMemcpyAsync((char*)host_dst + (size_t)r0 * row_bytes, stage,
                                       n * row_bytes, hipMemcpyDeviceToHost, s->st), "copy");
            FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");
        }
        return FHP_OK;
    }
    if (kind != FHP_OBS_BLOCKS) return fail(FHP_E_INVAL, "unknown observable %d", kind);
    if (block == 0 || (block < 64 ? (64 % block) : (block % 64)))
        return fail(FHP_E_INVAL, "block %u must divide 64 or be a multiple of 64", block);
    const uint32_t bw = (L.W + block - 1) / block, bh = (L.H + block - 1) / block;
    const size_t blk_bytes = 3 * sizeof(int32_t), row_bytes = (size_t)bw * blk_bytes;
    if (dst_bytes < row_bytes * bh)
        return fail(FHP_E_NOMEM, "destination of %zu bytes, %zu needed", dst_bytes, row_bytes * bh);
    int32_t* stage = (int32_t*)s->buf[1 - s->cur];
    // The stage holds at least 7 planes of 32 words, i.e. 149 blocks: whole
    // block rows when one fits, else pieces of one block row.
    const size_t cap = staging_bytes(s) / blk_bytes;
    const uint32_t rows = (uint32_t)((cap / bw < bh) ? cap / bw : bh);
    const uint32_t cols = rows ? bw : (uint32_t)cap;
    for (uint32_t r0 = 0; r0 < bh; r0 += rows ? rows : 1) {
        const uint32_t n = rows ? ((r0 + rows <= bh) ? rows : bh - r0) : 1;
        for (uint32_t c0 = 0; c0 < bw; c0 += cols) {
            const uint32_t m = (c0 + cols <= bw) ? cols : bw - c0;
            FHP_HIP_TRY(launch_observe_blocks(planes, L, block, r0, n, c0, m, stage, s->st), "blocks");
            FHP_HIP_TRY(hipMemcpyAsync((char*)host_dst + ((size_t)r0 * bw + c0) * blk_bytes, stage,
                                       (size_t)n * m * blk_bytes, hipMemcpyDeviceToHost, s->st),
                        "copy");
            FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");
        }
    }
    return FHP_OK;
}

int fhp_get_state(fhp_sim* s, uint8_t* host_dst, size_t bytes) {
    if (!s || !host_dst) return fail(FHP_E_INVAL, "NULL argument");
    const uint32_t W = s->L.W, H = s->L.H;
    if (bytes < (size_t)W * H)
        return fail(FHP_E_NOMEM, "destination of %zu bytes, %zu needed", bytes, (size_t)W * H);
    const Lattice L = lattice_of(s);
    uint8_t* stage = (uint8_t*)s->buf[1 - s->cur];
    uint32_t rows = (uint32_t)(staging_bytes(s) / W);
    if (rows > H) rows = H;
    for (uint32_t r0 = 0; r0 < H; r0 += rows) {
        const uint32_t n = (r0 + rows <= H) ? rows : H - r0;
        FHP_HIP_TRY(launch_unpack(s->buf[s->cur], L, r0, n, stage, s->st), "unpack");
        FHP_HIP_TRY(hipMemcpyAsync(host_dst + (size_t)r0 * W, stage, (size_t)n * W,
                                   hipMemcpyDeviceToHost, s->st), "download");
        FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");
    }
    return FHP_OK;
}

int fhp_set_state(fhp_sim* s, const uint8_t* host_src, size_t bytes, uint64_t t) {
    if (!s || !host_src) return fail(FHP_E_INVAL, "NULL argument");
    if (bytes != (size_t)s->L.W * s->L.H)
        return fail(FHP_E_INVAL, "state of %zu bytes, %zu expected", bytes, (size_t)s->L.W * s->L.H);
    if (t >= kTimeLimit) return fail(FHP_E_STATE, "time %llu at or above 2^24", (unsigned long long)t);
    if (s->changed) *s->changed = 1;
    int rc = upload_bytes(s, host_src, 0);
    if (rc) return rc;
    rc = refresh_has_mask(s);
    if (rc) return rc;
    s->t = t;
    return FHP_OK;
}

int fhp_time(const fhp_sim* s, uint64_t* t) {
    if (!s || !t) return fail(FHP_E_INVAL, "NULL argument");
    *t = s->t;
    return FHP_OK;
}

int fhp_sync(fhp_sim* s) {
    if (!s) return fail(FHP_E_INVAL, "sim is NULL");
    FHP_HIP_TRY(hipStreamSynchronize(s->st), "sync");
    FHP_HIP_TRY(hipGetLastError(), "device");
    return FHP_OK;
}

void fhp_destroy(fhp_sim* s) {
    if (!s || s->owner) return;  // batch members are released with their batch
    (void)hipStreamSynchronize(s->st);
    free(s);
}

}  // extern "C"
