/*
 * fhp_oracle.c -- CPU oracle for the FHP lattice-gas time step.
 *
 * TEST INFRASTRUCTURE ONLY (see fhp_oracle.h).  Plain C, one node at a time,
 * one byte per node, two arrays, collision by table look-up.  Nothing here is
 * blocked, fused or reordered: each function follows the definition it cites.
 *
 * Geometry (the paper maps the triangular lattice onto a rectangular array by
 * shifting every second row by half a lattice constant, Sec. 2, Fig. 3; the
 * direction of the shift and the numbering of the velocities are not given):
 *   - odd rows are shifted by +1/2: node (x, y) sits at (x + (y mod 2)/2,
 *     y*sqrt(3)/2);
 *   - c_i points at angle (i - 2) * 60 degrees, so c_2 = E and c_5 = W are the
 *     horizontal pair that the forcing rule swaps (Sec. 2, last paragraph),
 *     c_3 = NE, c_4 = NW, c_0 = SW, c_1 = SE and c_{i+3} = -c_i.
 */
#include "fhp_oracle.h"

#include <math.h>
#include <stddef.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Counter-based hash: SplitMix64 (Steele, Lea & Flood 2014).              */

#define SM64_GAMMA 0x9E3779B97F4A7C15ull

static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The generator advances its state by gamma and returns mix(state); output
 * number n+1 from state `key` is therefore mix(key + (n+1)*gamma). */
uint64_t fhpo_hash(uint64_t key, uint64_t n)
{
    return sm64_mix(key + (n + 1) * SM64_GAMMA);
}

static uint64_t key_for(uint64_t seed, uint64_t tag) { return fhpo_hash(seed, tag); }

/* Counter of a (t, y, column) triple: t*2^40 + y*2^20 + col. */
static uint64_t counter(uint64_t t, uint64_t y, uint64_t col)
{
    return (t << 40) + (y << 20) + col;
}

/* ---------------------------------------------------------------------- */
/* Neighbours on the row-shifted rectangular array.                        */

/* Offset (dx, dy) from node (x, y) to its neighbour in direction c_i; dx
 * depends on the parity of y because odd rows are shifted by +1/2. */
static const int DX[6][2] = {
    /* c0 SW */ {-1, 0},
    /* c1 SE */ {0, 1},
    /* c2 E  */ {1, 1},
    /* c3 NE */ {0, 1},
    /* c4 NW */ {-1, 0},
    /* c5 W  */ {-1, -1},
};
static const int DY[6] = {-1, -1, 0, 1, 1, 0};

static uint32_t wrap(int64_t v, uint32_t n)
{
    int64_t r = v % (int64_t)n;
    return (uint32_t)(r < 0 ? r + n : r);
}

/* Index of the neighbour of (x, y) in direction c_i, on the W x H torus. */
static size_t neighbour(int i, uint32_t x, uint32_t y, uint32_t W, uint32_t H)
{
    uint32_t nx = wrap((int64_t)x + DX[i][y & 1], W);
    uint32_t ny = wrap((int64_t)y + DY[i], H);
    return (size_t)ny * W + nx;
}

/* ---------------------------------------------------------------------- */
/* Collision table.                                                         */

/* The paper's collision rules are in a figure that is not available
 * (Sec. 2, Fig. 2); the text requires only conservation of mass and momentum
 * and a rest channel.  The rule set used is FHP-II (seven channels):
 *   R1 a head-on pair {i, i+3} and no other moving particle turns to
 *      {i+1, i+4} when chi = 1 or to {i-1, i+2} when chi = 0; the rest
 *      particle, if any, is a spectator;
 *   R2 the symmetric triple {0, 2, 4} and {1, 3, 5} swap when there is no
 *      rest particle;
 *   R3 one moving particle i plus a rest particle becomes the pair
 *      {i-1, i+1} without rest particle, and back;
 *   every other state is unchanged.
 * Indices are mod 6.  Bit i of a state is channel i; bit 6 is the rest
 * particle. */
static int bit(int i) { return 1 << (((i % 6) + 6) % 6); }

void fhpo_collision_table(int chi, uint8_t out[128])
{
    for (int s = 0; s < 128; s++) {
        int moving = s & 63;
        int rest = (s >> 6) & 1;
        int res = s;
        for (int i = 0; i < 3; i++) { /* R1 */
            if (moving == (bit(i) | bit(i + 3))) {
                int turned = chi ? (bit(i + 1) | bit(i + 4)) : (bit(i - 1) | bit(i + 2));
                res = turned | (rest << 6);
            }
        }
        if (!rest) { /* R2 */
            int even = bit(0) | bit(2) | bit(4);
            int odd = bit(1) | bit(3) | bit(5);
            if (moving == even) res = odd;
            if (moving == odd) res = even;
        }
        for (int i = 0; i < 6; i++) { /* R3 */
            int pair = bit(i - 1) | bit(i + 1);
            if (rest && moving == bit(i)) res = pair;
            if (!rest && moving == pair) res = bit(i) | (1 << 6);
        }
        out[s] = (uint8_t)res;
    }
}

/* FHP-I (Frisch, Hasslacher & Pomeau 1986): six moving channels only.  A
 * head-on pair alone turns by +60 degrees (chi = 1) or -60 degrees (chi = 0);
 * the symmetric triples {0,2,4} and {1,3,5} exchange.  The rest bit is a
 * spectator: it never changes and never blocks a collision. */
static void fhp1_table(int chi, uint8_t out[128])
{
    for (int s = 0; s < 128; s++) {
        int moving = s & 63;
        int rest = s & 64;
        int res = s;
        for (int i = 0; i < 3; i++) {
            if (moving == (bit(i) | bit(i + 3)))
                res = (chi ? (bit(i + 1) | bit(i + 4)) : (bit(i - 1) | bit(i + 2))) | rest;
        }
        int even = bit(0) | bit(2) | bit(4);
        int odd = bit(1) | bit(3) | bit(5);
        if (moving == even) res = odd | rest;
        if (moving == odd) res = even | rest;
        out[s] = (uint8_t)res;
    }
}

static int mass_of(int s)
{
    int m = 0;
    for (int c = 0; c < 7; c++) m += (s >> c) & 1;
    return m;
}

/* FHP-III, collision-saturated: every state that shares its mass and
 * momentum with another state changes.  Reading used here:
 *   - states of mass <= 3: FHP-II where FHP-II changes the state; FHP-II
 *     leaves unchanged, of the states that can change, exactly the six
 *     three-member classes {A_j, B_j, C_j} (j = 0..5) with
 *       A_j = {j, j+1, j+4}   (head-on pair j+1, j+4 and spectator j),
 *       B_j = {j, j+2, j+5}   (the pair turned by +60 degrees),
 *       C_j = {j+1, j+5} + rest,
 *     which cycle A -> B -> C -> A for chi = 1 and the other way for chi = 0;
 *   - states of mass >= 4 follow by particle-hole duality:
 *     T(s) = ~T(~s) on the seven particle bits. */
static void fhp3_table(int chi, uint8_t out[128])
{
    uint8_t low[128];
    fhpo_collision_table(chi, low);
    for (int j = 0; j < 6; j++) {
        int A = bit(j) | bit(j + 1) | bit(j + 4);
        int B = bit(j) | bit(j + 2) | bit(j + 5);
        int C = bit(j + 1) | bit(j + 5) | 64;
        low[A] = (uint8_t)(chi ? B : C);
        low[B] = (uint8_t)(chi ? C : A);
        low[C] = (uint8_t)(chi ? A : B);
    }
    for (int s = 0; s < 128; s++)
        out[s] = mass_of(s) <= 3 ? low[s] : (uint8_t)(~low[~s & 127] & 127);
}

int fhpo_rule_table(int rules, int chi, uint8_t out[128])
{
    if (!out || (chi != 0 && chi != 1)) return -1;
    switch (rules) {
        case FHPO_RULES_FHP2: fhpo_collision_table(chi, out); return 0;
        case FHPO_RULES_FHP1: fhp1_table(chi, out); return 0;
        case FHPO_RULES_FHP3: fhp3_table(chi, out); return 0;
        default: return -1;
    }
}

/* ---------------------------------------------------------------------- */
/* Initial state.                                                           */

int fhpo_init(uint32_t W, uint32_t H, uint64_t seed, double fill,
              const uint8_t *mask, int walls, uint8_t *state)
{
    if (!state || W == 0 || H == 0 || !(fill >= 0.0 && fill <= 1.0)) return -1;
    uint64_t key_init = key_for(seed, FHPO_TAG_INIT);
    uint64_t thr = (uint64_t)floor(fill * 4294967296.0); /* floor(fill * 2^32) */
    for (uint32_t y = 0; y < H; y++) {
        for (uint32_t x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            int solid = (mask && mask[i]) || (walls && (y == 0 || y == H - 1));
            uint8_t s = 0;
            if (solid) {
                s = 0x80;
            } else {
                for (uint64_t c = 0; c < 7; c++) {
                    uint64_t h = fhpo_hash(key_init, (c << 40) + ((uint64_t)y << 20) + x);
                    if ((h >> 32) < thr) s |= (uint8_t)(1u << c);
                }
            }
            state[i] = s;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* One time step.                                                           */

/* Chirality of node (x, y) at step t: bit (x mod 64) of
 * H(key_chir, t*2^40 + y*2^20 + floor(x/64)). */
static int chirality(uint64_t key_chir, int mode, uint64_t t, uint32_t x, uint32_t y)
{
    if (mode == FHPO_CHIR_ZERO) return 0;
    if (mode == FHPO_CHIR_ONE) return 1;
    uint64_t h = fhpo_hash(key_chir, counter(t, y, x / 64));
    return (int)((h >> (x % 64)) & 1);
}

/* Forcing coin of node (x, y) at step t.  With
 * h = H(key_force, t*2^40 + y*2^20 + floor(x/64)) the coin is up iff
 * (h mod 2^32) < floor(f * 2^38) and (h >> 58) == x mod 64: at most one node
 * per 64-node group per step, each node with probability floor(f*2^38)/2^38. */
static int coin(uint64_t key_force, uint64_t thr, uint64_t t, uint32_t x, uint32_t y)
{
    if (thr == 0) return 0;
    uint64_t h = fhpo_hash(key_force, counter(t, y, x / 64));
    return (h & 0xffffffffull) < thr && (h >> 58) == (uint64_t)(x % 64);
}

int64_t fhpo_step(const uint8_t *in, uint8_t *out, uint32_t W, uint32_t H,
                  uint64_t t, uint64_t seed, double force_rate, int chir_mode,
                  int nthreads)
{
    return fhpo_step_rules(in, out, W, H, t, seed, force_rate, chir_mode, FHPO_RULES_FHP2,
                           nthreads);
}

int64_t fhpo_step_rules(const uint8_t *in, uint8_t *out, uint32_t W, uint32_t H,
                        uint64_t t, uint64_t seed, double force_rate, int chir_mode,
                        int rules, int nthreads)
{
    if (!in || !out || in == out || W == 0 || H == 0 || (H & 1)) return -1;
    if (!(force_rate >= 0.0 && force_rate < 1.0 / 64.0)) return -1;
    if (chir_mode < FHPO_CHIR_HASH || chir_mode > FHPO_CHIR_ONE) return -1;

    uint8_t table[2][128];
    if (fhpo_rule_table(rules, 0, table[0]) || fhpo_rule_table(rules, 1, table[1])) return -1;
    uint64_t key_chir = key_for(seed, FHPO_TAG_CHIR);
    uint64_t key_force = key_for(seed, FHPO_TAG_FORCE);
    uint64_t thr = (uint64_t)floor(force_rate * 274877906944.0); /* floor(f * 2^38) */
    int64_t swaps = 0;
    if (nthreads <= 0) nthreads = 1;

#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(+ : swaps)
    for (int64_t yy = 0; yy < (int64_t)H; yy++) {
        uint32_t y = (uint32_t)yy;
        for (uint32_t x = 0; x < W; x++) {
            size_t here = (size_t)y * W + x;
            /* Motion: the particle arriving with velocity c_i comes from the
             * neighbour in direction c_{i+3} = -c_i; the rest particle stays. */
            int n = 0;
            for (int i = 0; i < 6; i++) {
                uint8_t src = in[neighbour((i + 3) % 6, x, y, W, H)];
                n |= ((src >> i) & 1) << i;
            }
            n |= in[here] & 0x40;
            int solid = (in[here] >> 7) & 1;

            int s;
            if (solid) {
                /* Bounce-back: every moving particle reverses, c_i -> c_{i+3};
                 * the rest particle stays. */
                s = n & 0x40;
                for (int i = 0; i < 6; i++) s |= ((n >> ((i + 3) % 6)) & 1) << i;
            } else {
                s = table[chirality(key_chir, chir_mode, t, x, y)][n];
                /* Forcing: pattern (..1..0..) -> (..0..1..) on bits 5 and 2. */
                if (coin(key_force, thr, t, x, y) && ((s >> 5) & 1) && !((s >> 2) & 1)) {
                    s = (s & ~0x20) | 0x04;
                    swaps += 1;
                }
            }
            out[here] = (uint8_t)(s | (solid << 7));
        }
    }
    return swaps;
}

int fhpo_run(uint8_t *state, uint8_t *tmp, uint32_t W, uint32_t H, uint64_t t0,
             uint64_t n, uint64_t seed, double force_rate, int chir_mode,
             int nthreads, int64_t *swaps)
{
    return fhpo_run_rules(state, tmp, W, H, t0, n, seed, force_rate, chir_mode,
                          FHPO_RULES_FHP2, nthreads, swaps);
}

int fhpo_run_rules(uint8_t *state, uint8_t *tmp, uint32_t W, uint32_t H, uint64_t t0,
                   uint64_t n, uint64_t seed, double force_rate, int chir_mode,
                   int rules, int nthreads, int64_t *swaps)
{
    int64_t total = 0;
    size_t bytes = (size_t)W * H;
    for (uint64_t k = 0; k < n; k++) {
        int64_t r = fhpo_step_rules(state, tmp, W, H, t0 + k, seed, force_rate, chir_mode, rules,
                                    nthreads);
        if (r < 0) return -1;
        total += r;
        memcpy(state, tmp, bytes);
    }
    if (swaps) *swaps = total;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Observables.                                                             */

/* Momentum of channel i in units (1/2, sqrt(3)/2): c_i = (cos, sin) of
 * (i - 2) * 60 degrees. */
static const int PX[7] = {-1, 1, 2, 1, -1, -2, 0};
static const int PY[7] = {-1, -1, 0, 1, 1, 0, 0};

void fhpo_observe_global(const uint8_t *state, uint32_t W, uint32_t H, int64_t out[11])
{
    memset(out, 0, 11 * sizeof(int64_t));
    for (size_t i = 0; i < (size_t)W * H; i++) {
        for (int c = 0; c < 7; c++) {
            if ((state[i] >> c) & 1) {
                out[0] += 1;
                out[1] += PX[c];
                out[2] += PY[c];
                out[3 + c] += 1;
            }
        }
        out[10] += (state[i] >> 7) & 1;
    }
}

void fhpo_observe_rows(const uint8_t *state, uint32_t W, uint32_t H, int64_t *out)
{
    memset(out, 0, (size_t)H * 3 * sizeof(int64_t));
    for (uint32_t y = 0; y < H; y++) {
        int64_t *o = out + (size_t)y * 3;
        for (uint32_t x = 0; x < W; x++) {
            uint8_t s = state[(size_t)y * W + x];
            for (int c = 0; c < 7; c++) {
                if ((s >> c) & 1) {
                    o[0] += 1;
                    o[1] += PX[c];
                    o[2] += PY[c];
                }
            }
        }
    }
}

int fhpo_observe_blocks(const uint8_t *state, uint32_t W, uint32_t H, uint32_t b, int32_t *out)
{
    if (!state || !out || b == 0) return -1;
    uint32_t bw = (W + b - 1) / b, bh = (H + b - 1) / b;
    memset(out, 0, (size_t)bw * bh * 3 * sizeof(int32_t));
    for (uint32_t y = 0; y < H; y++) {
        for (uint32_t x = 0; x < W; x++) {
            int32_t *o = out + ((size_t)(y / b) * bw + x / b) * 3;
            uint8_t s = state[(size_t)y * W + x];
            for (int c = 0; c < 7; c++) {
                if ((s >> c) & 1) {
                    o[0] += 1;
                    o[1] += PX[c];
                    o[2] += PY[c];
                }
            }
        }
    }
    return 0;
}

uint64_t fhpo_digest(const uint8_t *state, uint32_t W, uint32_t H)
{
    uint64_t d = 0;
    uint32_t words = (W + 63) / 64;
    for (uint64_t c = 0; c < 8; c++) {
        for (uint32_t y = 0; y < H; y++) {
            for (uint32_t w = 0; w < words; w++) {
                uint64_t word = 0;
                for (uint32_t b = 0; b < 64 && 64 * w + b < W; b++) {
                    uint64_t v = (state[(size_t)y * W + 64 * w + b] >> c) & 1;
                    word |= v << b;
                }
                d += fhpo_hash(word, counter(c, y, w));
            }
        }
    }
    return d;
}
