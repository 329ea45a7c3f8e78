/*
 * fhp_oracle.h -- CPU oracle for the FHP lattice-gas time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously correct
 * definition of the FHP dynamics that the GPU library is checked against.  It
 * is built and called only by the test suite, the smoke check and the CPU
 * baseline leg of the benchmark.  The GPU library never includes, links or
 * calls it, and it shares no code, header or table with the GPU library.
 *
 * Model (Szkoda, Koza & Tykierko, "Accelerating cellular automata simulations
 * using AVX and CUDA", arXiv:1208.2428):
 *   - one byte per node (Sec. 2, Fig. 1): bits 0-5 = particle moving with
 *     velocity c_i, bit 6 = rest particle, bit 7 = boundary (solid) node;
 *   - a step is motion followed by scattering (Sec. 2, itemised list);
 *   - scattering uses a 256-entry look-up table (Sec. 2) and includes the
 *     bounce-back from boundary nodes (Sec. 2, citing Chopard & Droz);
 *   - the triangular lattice is stored as a rectangular array with every
 *     second row shifted by half a lattice constant (Sec. 2, Fig. 3);
 *   - periodic in x (Sec. 2, Fig. 4); the horizontal forcing flips a
 *     W-moving particle to E-moving with some probability (Sec. 2, last
 *     paragraph).
 * Where the paper is silent (collision rule set, numbering, random chirality,
 * forcing coin, initial state) the readings below are used; each is repeated
 * at the function that implements it.
 *
 * Node (x, y) is byte state[y*W + x], 0 <= x < W, 0 <= y < H.  The lattice is
 * a torus in both directions; H must be even so that row parity is consistent.
 *
 * Parity pins: every function here is pinned by a CPU test against geometry,
 * conservation laws, closed forms, the textbook SplitMix64 sequence or brute
 * force (tests/test_oracle_*.py).  None is "parity unpinned".
 */
#ifndef FHP_ORACLE_H
#define FHP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Chirality modes.  HASH is the model; ZERO/ONE fix the chirality bit for tests. */
#define FHPO_CHIR_HASH 0
#define FHPO_CHIR_ZERO 1
#define FHPO_CHIR_ONE 2

/* Hash tags used to derive the per-purpose keys key_tag = H(seed, tag). */
#define FHPO_TAG_INIT 1
#define FHPO_TAG_CHIR 2
#define FHPO_TAG_FORCE 3

/* H(key, n): output number n+1 of SplitMix64 started from state `key`
 * (Steele, Lea & Flood, OOPSLA 2014), i.e. mix(key + (n+1)*gamma) mod 2^64. */
uint64_t fhpo_hash(uint64_t key, uint64_t n);

/* Rule sets.  The paper's rule figure is missing (Sec. 2); FHP-II is the
 * reading of its model, FHP-I and the collision-saturated FHP-III are the
 * variants of the same lattice gas (Frisch et al. 1987). */
#define FHPO_RULES_FHP2 0
#define FHPO_RULES_FHP1 1
#define FHPO_RULES_FHP3 2

/* Collision table T_chi for fluid nodes: out[s] for s = 0..127 (7 particle
 * bits, FHP-II rule set).  chi must be 0 or 1. */
void fhpo_collision_table(int chi, uint8_t out[128]);

/* Collision table of rule set `rules` (FHPO_RULES_*).  Returns 0, or -1 for an
 * unknown rule set or chi not in {0, 1}. */
int fhpo_rule_table(int rules, int chi, uint8_t out[128]);

/* Initial state: fluid node bit c (c = 0..6) is set iff
 * (H(key_init, c*2^40 + y*2^20 + x) >> 32) < floor(fill * 2^32).  Solid nodes
 * (mask nonzero, or rows 0 and H-1 when walls != 0) get only bit 7.
 * mask may be NULL (no obstacles).  Returns 0, or -1 on bad arguments. */
int fhpo_init(uint32_t W, uint32_t H, uint64_t seed, double fill,
              const uint8_t *mask, int walls, uint8_t *state);

/* One time step t -> t+1 (t = steps already completed): motion (pull from the
 * six neighbours), then collision (fluid) or bounce-back (solid), then forcing.
 * `in` and `out` are distinct W*H arrays.  force_rate f must lie in [0, 1/64).
 * nthreads <= 0 means one thread.  Returns the number of forcing swaps applied,
 * or -1 on bad arguments. */
int64_t fhpo_step(const uint8_t *in, uint8_t *out, uint32_t W, uint32_t H,
                  uint64_t t, uint64_t seed, double force_rate, int chir_mode,
                  int nthreads);

/* fhpo_step with the collision of rule set `rules` (fhpo_step uses FHP-II). */
int64_t fhpo_step_rules(const uint8_t *in, uint8_t *out, uint32_t W, uint32_t H,
                        uint64_t t, uint64_t seed, double force_rate, int chir_mode,
                        int rules, int nthreads);

/* Runs n steps starting at time t0 with two arrays; the final state is left in
 * `state`.  `tmp` is a caller-provided W*H scratch array.  swaps (nullable)
 * receives the total forcing swaps.  Returns 0 or -1. */
int fhpo_run(uint8_t *state, uint8_t *tmp, uint32_t W, uint32_t H, uint64_t t0,
             uint64_t n, uint64_t seed, double force_rate, int chir_mode,
             int nthreads, int64_t *swaps);

/* fhpo_run with the collision of rule set `rules`. */
int fhpo_run_rules(uint8_t *state, uint8_t *tmp, uint32_t W, uint32_t H, uint64_t t0,
                   uint64_t n, uint64_t seed, double force_rate, int chir_mode,
                   int rules, int nthreads, int64_t *swaps);

/* Global observables, summed over all nodes (solid ones included):
 * out[0] = mass, out[1] = p_x, out[2] = p_y (momentum in units of (1/2,
 * sqrt(3)/2) lattice constants), out[3..9] = particle count per channel 0..6,
 * out[10] = number of solid nodes. */
void fhpo_observe_global(const uint8_t *state, uint32_t W, uint32_t H,
                         int64_t out[11]);

/* Row sums: out is int64[H][3] holding (rho, p_x, p_y) of each row. */
void fhpo_observe_rows(const uint8_t *state, uint32_t W, uint32_t H, int64_t *out);

/* Block sums over b x b blocks in index space: out is
 * int32[ceil(H/b)][ceil(W/b)][3] holding (rho, p_x, p_y). */
int fhpo_observe_blocks(const uint8_t *state, uint32_t W, uint32_t H,
                        uint32_t b, int32_t *out);

/* State digest: sum over planes c = 0..7, rows y and 64-node words w of
 * H(word_c(y, w), c*2^40 + y*2^20 + w) mod 2^64, where word_c(y, w) holds bit c
 * of nodes x = 64w .. 64w+63 of row y (bit b <-> x = 64w + b; nodes beyond W
 * contribute 0 bits). */
uint64_t fhpo_digest(const uint8_t *state, uint32_t W, uint32_t H);

#ifdef __cplusplus
}
#endif
#endif
