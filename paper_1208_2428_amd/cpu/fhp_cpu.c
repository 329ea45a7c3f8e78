/*
 * fhp_cpu.c -- host bit-plane FHP stepper: OpenMP over rows, SIMD along rows.
 *
 * The FHP time step of arXiv:1208.2428, Sec. 2, for a CPU: every node holds
 * seven channels (six velocities c_0..c_5 and a rest particle) and a boundary
 * flag; a step moves every particle to the neighbour it points at, then
 * scatters particles at fluid nodes (mass and momentum conserved), reflects
 * them at boundary nodes, and lets a constant horizontal force exchange an
 * W-moving for an E-moving particle now and then.  The paper's CPU codes
 * (Sec. 3.1) keep a byte per node and vectorise the motion over bytes; here a
 * node is one bit of each of seven 64-bit words (bit-planes), so one vector
 * instruction handles 512 (AVX-512) or 256 (AVX2) nodes of one channel, and
 * the collision is a boolean function of the seven planes.
 *
 * Readings of what the paper leaves open (identical to the GPU library's, so
 * the states agree bit for bit):
 *   - odd rows are shifted by +1/2; c_i points at (i-2)*60 degrees: c_2 = E,
 *     c_3 = NE, c_4 = NW, c_5 = W, c_0 = SW, c_1 = SE;
 *   - collisions FHP-II: a head-on pair alone turns by +60 degrees (chirality
 *     1) or -60 degrees (chirality 0), the rest particle a spectator; the
 *     triples {0,2,4} and {1,3,5} swap when there is no rest particle; one
 *     particle with a rest particle becomes the two particles at +-60 degrees
 *     from it, and back;
 *   - step = stream, then collide (fluid) or bounce back c_i -> c_{i+3} (solid,
 *     rest particle kept), then force: on a fluid node with the coin up and
 *     channel 5 set, channel 2 clear, the two are exchanged;
 *   - random numbers: H(key, n) = SplitMix64 output n+1 from state key
 *     (Steele, Lea & Flood 2014); key_tag = H(seed, tag), INIT 1, CHIR 2,
 *     FORCE 3; the chirality of node x of row y at step t is bit x mod 64 of
 *     H(key_chir, t*2^40 + y*2^20 + floor(x/64)); the coin of that word is
 *     h = H(key_force, same counter), up iff h mod 2^32 < floor(f*2^38), and
 *     lands on node h >> 58 of the word;
 *   - initial state: fluid node bit c set iff
 *     H(key_init, c*2^40 + y*2^20 + x) >> 32 < floor(fill*2^32).
 *
 * Pull streaming on bit-planes: the particle that arrives at (x, y) with
 * velocity c_i left the node at (x, y) - c_i.  A shift "from x-1" (towards
 * larger x, taking the top bit of the word to the left) is written shl1, a
 * shift "from x+1" shr1:
 *   c_2 from row y with shl1, c_5 from row y with shr1, c_6 (rest) stays;
 *   c_3 from row y-1, shl1 when y is even; c_4 from row y-1, shr1 when y is odd;
 *   c_0 from row y+1, shr1 when y is odd; c_1 from row y+1, shl1 when y is even.
 * Rows and words wrap (the lattice is a torus; walls are solid rows).
 */
#include <math.h>
#include <omp.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fhp_cpu.h"

#define GAMMA 0x9E3779B97F4A7C15ull
#define TIME_LIMIT (1ull << 24)
#define VW 8 /* words per vector */

typedef uint64_t vec __attribute__((vector_size(8 * VW)));

struct fhpcpu_sim {
    uint32_t W, H, wd;  /* nodes per row, rows, words per row */
    size_t plane;       /* words per plane */
    uint64_t *buf[2];   /* 7 planes each */
    uint64_t *solid;    /* obstacles (wall rows are added when read) */
    int cur, walls;
    uint64_t t, key_init, key_chir, key_force, thr_force;
};

static _Thread_local char last_error[256];

const char *fhpcpu_last_error(void) { return last_error; }

static int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(last_error, sizeof last_error, fmt, ap);
    va_end(ap);
    return code;
}

/* ------------------------------------------------------------- SplitMix64 */

static inline uint64_t finalise(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t hash(uint64_t key, uint64_t n) { return finalise(key + (n + 1) * GAMMA); }

static inline vec vfinalise(vec z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------- the node update */

/* One step for VW words of one row, after streaming: a[0..5] moving, a[6]
 * rest, s solid, chi chirality words, coin (at most one bit per word, already
 * gated by the rate).  FHP-II by explicit patterns of the six moving
 * channels: q[j] = channels j and j+1 both empty. */
static inline __attribute__((always_inline)) void update(const vec a[7], vec s, vec chi, vec coin,
                                                         vec o[7]) {
    vec e[6], q[6];
    for (int j = 0; j < 6; j++) e[j] = ~a[j];
    for (int j = 0; j < 6; j++) q[j] = e[j] & e[(j + 1) % 6];
    const vec r = a[6], nr = ~a[6];
    /* head-on pair {i, i+3} and nothing else moving (rest either way) */
    vec hp[3];
    for (int i = 0; i < 3; i++) hp[i] = a[i] & a[i + 3] & q[(i + 1) % 6] & q[(i + 4) % 6];
    /* the symmetric triples, without rest particle */
    const vec t0 = a[0] & a[2] & a[4] & e[1] & e[3] & e[5] & nr;
    const vec t1 = a[1] & a[3] & a[5] & e[0] & e[2] & e[4] & nr;
    /* one particle i with rest; the pair {i-1, i+1} without rest */
    vec one[6], two[6];
    for (int i = 0; i < 6; i++) {
        one[i] = a[i] & q[(i + 1) % 6] & q[(i + 3) % 6] & e[(i + 5) % 6] & r;
        two[i] = a[(i + 5) % 6] & a[(i + 1) % 6] & e[i] & q[(i + 2) % 6] & e[(i + 4) % 6] & nr;
    }
    vec any = hp[0] | hp[1] | hp[2] | t0 | t1;
    vec any_one = one[0] | one[1] | one[2] | one[3] | one[4] | one[5];
    vec any_two = two[0] | two[1] | two[2] | two[3] | two[4] | two[5];
    any |= any_one | any_two;
    const vec fluid = ~s;
    for (int j = 0; j < 6; j++) {
        /* what the rules put into channel j */
        vec g = (hp[(j + 5) % 3] & chi) | (hp[(j + 1) % 3] & ~chi);
        g |= (j & 1) ? t0 : t1;
        g |= one[(j + 1) % 6] | one[(j + 5) % 6] | two[j];
        const vec coll = (a[j] & ~any) | g;
        o[j] = (fluid & coll) | (s & a[(j + 3) % 6]);
    }
    o[6] = r ^ (fluid & (any_one | any_two));
    /* forcing: 5 -> 2 on fluid nodes where the coin is up */
    const vec m = coin & fluid & o[5] & ~o[2];
    o[5] ^= m;
    o[2] ^= m;
}

/* Shifts of a row by one node with wrap-around: shl1 takes the bit from
 * x - 1, shr1 from x + 1. */
static inline void shl1_row(const uint64_t *src, uint64_t *dst, uint32_t wd) {
    dst[0] = (src[0] << 1) | (src[wd - 1] >> 63);
    for (uint32_t w = 1; w < wd; w++) dst[w] = (src[w] << 1) | (src[w - 1] >> 63);
}
static inline void shr1_row(const uint64_t *src, uint64_t *dst, uint32_t wd) {
    for (uint32_t w = 0; w + 1 < wd; w++) dst[w] = (src[w] >> 1) | (src[w + 1] << 63);
    dst[wd - 1] = (src[wd - 1] >> 1) | (src[0] << 63);
}

struct row_args {
    const uint64_t *in;   /* 7 planes */
    uint64_t *out;
    const uint64_t *solid;
    size_t plane;
    uint32_t wd, H, walls;
    uint64_t kc, kf;      /* per-row hash states: key + (counter(t, y, 0) + 1) * gamma */
    uint64_t thr, force;
    uint64_t *tmp;        /* 8 padded rows of this thread */
    uint32_t wdp, y;
};

/* The update of row y, written once and compiled for several instruction
 * sets (see the dispatch below). */
static inline __attribute__((always_inline)) void row_impl(const struct row_args *A) {
    const uint32_t wd = A->wd, wdp = A->wdp, H = A->H, y = A->y;
    const uint32_t ym = y ? y - 1 : H - 1, yp = (y + 1 == H) ? 0 : y + 1;
    const size_t ps = A->plane;
    const uint64_t *in = A->in;
    uint64_t *src[8];
    for (int c = 0; c < 8; c++) src[c] = A->tmp + (size_t)c * wdp;
    const int odd = y & 1;
#define ROW(c, yy) (in + (size_t)(c) * ps + (size_t)(yy) * wd)
    shl1_row(ROW(2, y), src[2], wd);
    shr1_row(ROW(5, y), src[5], wd);
    memcpy(src[6], ROW(6, y), wd * 8);
    if (odd) {
        memcpy(src[3], ROW(3, ym), wd * 8);
        shr1_row(ROW(4, ym), src[4], wd);
        shr1_row(ROW(0, yp), src[0], wd);
        memcpy(src[1], ROW(1, yp), wd * 8);
    } else {
        shl1_row(ROW(3, ym), src[3], wd);
        memcpy(src[4], ROW(4, ym), wd * 8);
        memcpy(src[0], ROW(0, yp), wd * 8);
        shl1_row(ROW(1, yp), src[1], wd);
    }
#undef ROW
    const int wall = A->walls && (y == 0 || y + 1 == H);
    if (wall)
        memset(src[7], 0xff, wd * 8);
    else
        memcpy(src[7], A->solid + (size_t)y * wd, wd * 8);
    for (int c = 0; c < 8; c++)  /* padding lanes: empty nodes */
        for (uint32_t w = wd; w < wdp; w++) src[c][w] = 0;

    vec lane;
    for (int k = 0; k < VW; k++) lane[k] = (uint64_t)k * GAMMA;
    for (uint32_t w0 = 0; w0 < wdp; w0 += VW) {
        vec a[7], o[7], s;
        for (int c = 0; c < 7; c++) memcpy(&a[c], src[c] + w0, sizeof(vec));
        memcpy(&s, src[7] + w0, sizeof(vec));
        const uint64_t step = (uint64_t)w0 * GAMMA;
        const vec chi = vfinalise(A->kc + step + lane);
        vec coin = {0};
        if (A->force) {
            const vec hf = vfinalise(A->kf + step + lane);
            const vec up = (vec)((hf & 0xffffffffull) < A->thr);
            coin = up & ((vec){1, 1, 1, 1, 1, 1, 1, 1} << (hf >> 58));
        }
        update(a, s, chi, coin, o);
        for (int c = 0; c < 7; c++) memcpy(src[c] + w0, &o[c], sizeof(vec));
    }
    for (int c = 0; c < 7; c++) memcpy(A->out + (size_t)c * ps + (size_t)y * wd, src[c], wd * 8);
}

__attribute__((target("avx512f,avx512dq,avx512bw,avx512vl"))) static void row_avx512(
    const struct row_args *A) {
    row_impl(A);
}
__attribute__((target("avx2"))) static void row_avx2(const struct row_args *A) { row_impl(A); }
static void row_generic(const struct row_args *A) { row_impl(A); }

typedef void (*row_fn)(const struct row_args *);

static row_fn pick_row(const char **name) {
    __builtin_cpu_init();
    if (__builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512dq") &&
        __builtin_cpu_supports("avx512bw") && __builtin_cpu_supports("avx512vl")) {
        if (name) *name = "avx512";
        return row_avx512;
    }
    if (__builtin_cpu_supports("avx2")) {
        if (name) *name = "avx2";
        return row_avx2;
    }
    if (name) *name = "generic";
    return row_generic;
}

const char *fhpcpu_isa(void) {
    const char *n = "generic";
    (void)pick_row(&n);
    return n;
}

/* ------------------------------------------------------------ the handle */

static uint64_t threshold(double f) { return (uint64_t)floor(f * 274877906944.0); /* 2^38 */ }

int fhpcpu_create(uint32_t W, uint32_t H, uint64_t seed, double fill, double force_rate, int walls,
                  const uint8_t *solid, fhpcpu_sim **out) {
    if (!out) return fail(FHPCPU_E_INVAL, "out is NULL");
    *out = NULL;
    if (W < 64 || W % 64 || H < 2 || H % 2 || W >= (1u << 20) || H >= (1u << 20))
        return fail(FHPCPU_E_INVAL, "lattice %ux%u: W must be a multiple of 64, H even, both in [2, 2^20)",
                    W, H);
    if (!(fill >= 0.0 && fill <= 1.0)) return fail(FHPCPU_E_INVAL, "fill %g outside [0, 1]", fill);
    if (!(force_rate >= 0.0 && force_rate < 1.0 / 64)) return fail(FHPCPU_E_INVAL, "force rate %g outside [0, 1/64)", force_rate);
    fhpcpu_sim *s = calloc(1, sizeof *s);
    if (!s) return fail(FHPCPU_E_NOMEM, "out of host memory");
    s->W = W;
    s->H = H;
    s->wd = W / 64;
    s->plane = (size_t)s->wd * H;
    s->walls = walls != 0;
    s->key_init = hash(seed, 1);
    s->key_chir = hash(seed, 2);
    s->key_force = hash(seed, 3);
    s->thr_force = threshold(force_rate);
    for (int b = 0; b < 2; b++) s->buf[b] = aligned_alloc(64, (7 * s->plane * 8 + 63) / 64 * 64);
    s->solid = aligned_alloc(64, (s->plane * 8 + 63) / 64 * 64);
    if (!s->buf[0] || !s->buf[1] || !s->solid) {
        fhpcpu_destroy(s);
        return fail(FHPCPU_E_NOMEM, "out of host memory");
    }
    memset(s->solid, 0, s->plane * 8);
    if (solid)
        for (uint32_t y = 0; y < H; y++)
            for (uint32_t x = 0; x < W; x++)
                if (solid[(size_t)y * W + x]) s->solid[(size_t)y * s->wd + x / 64] |= 1ull << (x % 64);
    /* initial state: per node and channel, fluid nodes only */
    const uint64_t thr = (uint64_t)floor(fill * 4294967296.0); /* 2^32 */
    uint64_t *P = s->buf[0];
#pragma omp parallel for schedule(static)
    for (uint32_t y = 0; y < H; y++) {
        const int wall = s->walls && (y == 0 || y + 1 == H);
        for (uint32_t w = 0; w < s->wd; w++) {
            const uint64_t sw = wall ? ~0ull : s->solid[(size_t)y * s->wd + w];
            for (int c = 0; c < 7; c++) {
                uint64_t word = 0;
                for (int b = 0; b < 64; b++) {
                    const uint64_t x = (uint64_t)w * 64 + b;
                    const uint64_t h = hash(s->key_init, ((uint64_t)c << 40) + ((uint64_t)y << 20) + x);
                    if ((h >> 32) < thr) word |= 1ull << b;
                }
                P[(size_t)c * s->plane + (size_t)y * s->wd + w] = word & ~sw;
            }
        }
    }
    *out = s;
    return FHPCPU_OK;
}

int fhpcpu_step(fhpcpu_sim *s, uint64_t n, int threads) {
    if (!s) return fail(FHPCPU_E_INVAL, "sim is NULL");
    if (s->t + n >= TIME_LIMIT) return fail(FHPCPU_E_STATE, "time would reach 2^24");
    const row_fn fn = pick_row(NULL);
    const uint32_t wdp = (s->wd + VW - 1) / VW * VW;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
    for (uint64_t k = 0; k < n; k++) {
        const uint64_t t = s->t;
        const uint64_t *in = s->buf[s->cur];
        uint64_t *outp = s->buf[s->cur ^ 1];
#pragma omp parallel num_threads(nt)
        {
            uint64_t *tmp = aligned_alloc(64, (size_t)8 * wdp * 8);
            struct row_args A = {in, outp, s->solid, s->plane, s->wd, s->H, (uint32_t)s->walls, 0, 0,
                                 s->thr_force, s->thr_force != 0, tmp, wdp, 0};
#pragma omp for schedule(static)
            for (uint32_t y = 0; y < s->H; y++) {
                const uint64_t ctr = (t << 40) + ((uint64_t)y << 20);
                A.y = y;
                A.kc = s->key_chir + (ctr + 1) * GAMMA;
                A.kf = s->key_force + (ctr + 1) * GAMMA;
                fn(&A);
            }
            free(tmp);
        }
        s->cur ^= 1;
        s->t++;
    }
    return FHPCPU_OK;
}

int fhpcpu_get_state(const fhpcpu_sim *s, uint8_t *dst, size_t bytes) {
    if (!s || !dst) return fail(FHPCPU_E_INVAL, "NULL argument");
    if (bytes != (size_t)s->W * s->H) return fail(FHPCPU_E_INVAL, "%zu bytes, %zu expected", bytes,
                                                  (size_t)s->W * s->H);
    const uint64_t *P = s->buf[s->cur];
#pragma omp parallel for schedule(static)
    for (uint32_t y = 0; y < s->H; y++) {
        const int wall = s->walls && (y == 0 || y + 1 == s->H);
        for (uint32_t x = 0; x < s->W; x++) {
            const size_t i = (size_t)y * s->wd + x / 64;
            const int b = x % 64;
            uint8_t v = 0;
            for (int c = 0; c < 7; c++) v |= (uint8_t)(((P[(size_t)c * s->plane + i] >> b) & 1) << c);
            if (wall || ((s->solid[i] >> b) & 1)) v |= 0x80;
            dst[(size_t)y * s->W + x] = v;
        }
    }
    return FHPCPU_OK;
}

int fhpcpu_set_state(fhpcpu_sim *s, const uint8_t *src, size_t bytes, uint64_t t) {
    if (!s || !src) return fail(FHPCPU_E_INVAL, "NULL argument");
    if (bytes != (size_t)s->W * s->H) return fail(FHPCPU_E_INVAL, "%zu bytes, %zu expected", bytes,
                                                  (size_t)s->W * s->H);
    if (t >= TIME_LIMIT) return fail(FHPCPU_E_STATE, "time at or above 2^24");
    uint64_t *P = s->buf[s->cur];
#pragma omp parallel for schedule(static)
    for (uint32_t y = 0; y < s->H; y++)
        for (uint32_t w = 0; w < s->wd; w++) {
            uint64_t words[8] = {0};
            for (int b = 0; b < 64; b++) {
                const uint8_t v = src[(size_t)y * s->W + (size_t)w * 64 + b];
                for (int c = 0; c < 8; c++) words[c] |= (uint64_t)((v >> c) & 1) << b;
            }
            const size_t i = (size_t)y * s->wd + w;
            for (int c = 0; c < 7; c++) P[(size_t)c * s->plane + i] = words[c];
            s->solid[i] = words[7];
        }
    s->t = t;
    return FHPCPU_OK;
}

int fhpcpu_time(const fhpcpu_sim *s, uint64_t *t) {
    if (!s || !t) return fail(FHPCPU_E_INVAL, "NULL argument");
    *t = s->t;
    return FHPCPU_OK;
}

int fhpcpu_digest(const fhpcpu_sim *s, uint64_t *out) {
    if (!s || !out) return fail(FHPCPU_E_INVAL, "NULL argument");
    const uint64_t *P = s->buf[s->cur];
    uint64_t sum = 0;
#pragma omp parallel for schedule(static) reduction(+ : sum)
    for (uint32_t y = 0; y < s->H; y++) {
        const int wall = s->walls && (y == 0 || y + 1 == s->H);
        for (uint32_t w = 0; w < s->wd; w++) {
            const size_t i = (size_t)y * s->wd + w;
            const uint64_t ctr = ((uint64_t)y << 20) + w;
            for (int c = 0; c < 7; c++) sum += hash(P[(size_t)c * s->plane + i], ((uint64_t)c << 40) + ctr);
            sum += hash(wall ? ~0ull : s->solid[i], (7ull << 40) + ctr);
        }
    }
    *out = sum;
    return FHPCPU_OK;
}

void fhpcpu_destroy(fhpcpu_sim *s) {
    if (!s) return;
    free(s->buf[0]);
    free(s->buf[1]);
    free(s->solid);
    free(s);
}
