/*
 * fhp.h -- C ABI of the MI355X (gfx950) FHP lattice-gas library.
 *
 * The library advances the FHP cellular automaton of Szkoda, Koza & Tykierko,
 * "Accelerating cellular automata simulations using AVX and CUDA"
 * (arXiv:1208.2428):
 *   - Sec. 2: seven boolean channels per node of a triangular lattice (six
 *     velocities c_0..c_5 and a rest particle) plus a boundary flag, one byte
 *     per node (Fig. 1); a time step is motion to the six nearest neighbours
 *     followed by scattering that conserves mass and momentum; boundary nodes
 *     reflect particles; the triangular lattice is stored as a rectangular
 *     array with every second row shifted by half a lattice constant (Fig. 3);
 *     walls on top and bottom, periodic in x (Fig. 4); a constant horizontal
 *     force realised by exchanging bits 2 and 5 with some probability;
 *   - Sec. 4: throughput is counted in lattice-site updates per second.
 *
 * Readings of points the paper leaves open (they define the results bit for
 * bit, and the CPU oracle used by the tests implements the same readings
 * independently):
 *   - numbering: odd rows are shifted by +1/2; c_i points at (i-2)*60 degrees
 *     (c_2 = E, c_3 = NE, c_4 = NW, c_5 = W, c_0 = SW, c_1 = SE);
 *   - collisions: FHP-II (head-on pairs turn by +-60 degrees according to a
 *     chirality bit, rest particle as spectator; the symmetric triples swap
 *     without rest particle; one particle plus rest <-> the two particles at
 *     +-60 degrees from it);
 *   - the step is: stream (pull from the neighbours), then collide (fluid) or
 *     bounce back c_i -> c_{i+3} (solid, rest particle kept), then forcing;
 *   - H(key, n) = SplitMix64 output n+1 from state key (Steele, Lea & Flood
 *     2014); key_tag = H(seed, tag) with tags INIT=1, CHIR=2, FORCE=3;
 *   - chirality of node (x, y) at step t (t = steps already done) is bit
 *     x mod 64 of H(key_chir, t*2^40 + y*2^20 + floor(x/64));
 *   - forcing coin: with h = H(key_force, t*2^40 + y*2^20 + floor(x/64)) the
 *     coin is up iff (h mod 2^32) < floor(f*2^38) and h>>58 == x mod 64; on a
 *     fluid node whose post-collision state has bit 5 set and bit 2 clear,
 *     bits 5 and 2 are exchanged;
 *   - initial state: fluid node bit c (0..6) is set iff
 *     (H(key_init, c*2^40 + y*2^20 + x) >> 32) < floor(fill*2^32); solid nodes
 *     start empty.
 * The lattice is a torus in both directions; FHP_WALLS_CHANNEL makes rows 0 and
 * H-1 solid.
 *
 * Device layout: seven bit-planes of uint64 words per buffer (bit b of word w
 * of row y is node x = 64w + b), two buffers (ping-pong), one solid plane.
 * Interchange layout (get/set state): the paper's byte per node, row-major
 * [y][x], bits 0-5 moving, bit 6 rest, bit 7 solid.
 *
 * Ownership: the caller owns every host buffer and the device workspace; the
 * library keeps only the pointers it was given and never frees them.  Calls
 * return FHP_OK (0) or a negative FHP_E_* code; fhp_last_error() returns a
 * message for the calling thread's last failure.  A handle is not thread-safe.
 * Work is enqueued on the handle's HIP stream; asynchronous device faults are
 * reported as FHP_E_DEVICE by the next call that synchronises.
 *
 * Testing the error paths: the environment variable FHP_FAULT, read once per
 * process, injects host-side failures that never reach the device --
 * "launch@N": every fhp_step launch after the first N fails (FHP_E_DEVICE; the
 * passes before it are kept and the time counter matches them); "alloc": the
 * pinned staging buffer of fhp_batch_create and fhp_pool_create is not
 * allocated (FHP_E_DEVICE, nothing is left allocated).
 */
#ifndef FHP_H
#define FHP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FHP_ABI_VERSION 1u
#define FHP_MAX_DEPTH 5u       /* largest temporal-block depth k of one HBM pass */
#define FHP_BATCH_MAX_DEPTH 5u  /* the same for batches and pools */
#define FHP_BATCH_MIN_HEIGHT 8u /* shortest lattice a batch or pool takes */

enum {
    FHP_OK = 0,
    FHP_E_INVAL = -1,  /* bad argument, size or layout */
    FHP_E_NOMEM = -2,  /* workspace or destination too small */
    FHP_E_DEVICE = -3, /* HIP runtime or kernel error */
    FHP_E_STATE = -4,  /* time counter would exceed 2^24 steps */
    FHP_E_BUSY = -5    /* no room (pool admission) */
};

enum { FHP_WALLS_NONE = 0, FHP_WALLS_CHANNEL = 1 };
enum { FHP_CHIR_HASH = 0, FHP_CHIR_ZERO = 1, FHP_CHIR_ONE = 2 };

/* Collision rule sets.  FHP_RULES_FHP2 is the model above.  FHP_RULES_FHP1:
 * head-on pairs turn by +-60 degrees by the chirality bit and the symmetric
 * triples swap, whatever the rest bit, which never changes.  FHP_RULES_FHP3
 * (collision-saturated): FHP-II on states of at most three particles, plus the
 * cycle A_j -> B_j -> C_j -> A_j (chirality 1; reversed for 0) with
 * A_j = {j, j+1, j+4}, B_j = {j, j+2, j+5}, C_j = {j+1, j+5} + rest, and on
 * states of four or more particles T(s) = ~T(~s) (particle-hole duality):
 * every state that shares mass and momentum with another one changes. */
enum { FHP_RULES_FHP2 = 0, FHP_RULES_FHP1 = 1, FHP_RULES_FHP3 = 2 };

/* Observable kinds for fhp_observe. */
enum {
    /* int64[11]: mass, p_x, p_y (momentum in units (1/2, sqrt(3)/2)),
     * particle count of channels 0..6, number of solid nodes; summed over all
     * nodes, solid ones included. */
    FHP_OBS_GLOBAL = 0,
    /* int32[ceil(H/b)][ceil(W/b)][3]: (rho, p_x, p_y) summed over b x b blocks
     * in index space; b must divide 64 or be a multiple of 64. */
    FHP_OBS_BLOCKS = 1,
    /* uint64[1]: sum over planes c = 0..7 (7 = solid), rows y and words w of
     * H(word, c*2^40 + y*2^20 + w) mod 2^64. */
    FHP_OBS_DIGEST = 2,
    /* int64[H][3]: (rho, p_x, p_y) summed over each row, e.g. for the velocity
     * profile across a channel (the flows of Sec. 2 and Sec. 4). */
    FHP_OBS_ROWS = 3
};

typedef struct fhp_params {
    uint32_t abi_version; /* FHP_ABI_VERSION */
    uint32_t width;       /* W: multiple of 64, < 2^20 */
    uint32_t height;      /* H: even, >= 2, < 2^20; W*H < 2^35 */
    uint32_t walls;       /* FHP_WALLS_* */
    uint32_t chirality;   /* FHP_CHIR_*; ZERO and ONE are test modes */
    uint32_t rules;       /* FHP_RULES_*; 0 = FHP-II */
    uint64_t seed;
    double fill;          /* per-channel occupancy of fluid nodes at t = 0, in [0, 1] */
    double force_rate;    /* forcing coin rate f per node and step, in [0, 1/64) */
    const uint8_t *solid; /* optional host mask, W*H bytes row-major, nonzero = solid;
                             copied at create; NULL = no obstacles */
} fhp_params;

typedef struct fhp_sim fhp_sim;

/* Message describing the calling thread's most recent error ("" if none). */
const char *fhp_last_error(void);

/* Device workspace needed by fhp_create for these parameters. */
int fhp_workspace_bytes(const fhp_params *p, size_t *bytes);

/* Creates a simulation at t = 0 with the initial state defined above.
 * dev_ws: device memory of at least fhp_workspace_bytes, 256-byte aligned, owned
 * by the caller and kept alive until fhp_destroy.  hip_stream: a hipStream_t
 * (NULL = default stream) on which all work of this handle is enqueued.
 * Synchronises the stream before returning. */
int fhp_create(const fhp_params *p, void *dev_ws, size_t ws_bytes, void *hip_stream,
               fhp_sim **out);

/* Temporal-block depth k (1..FHP_MAX_DEPTH): fhp_step runs k steps per pass over
 * HBM (the last pass of a call may be shorter).  0 selects the library's default
 * for this lattice: 3 where the lattice is too small to give every SIMD of the
 * device two waves (as for 4096 x 4096 on 256 compute units), 4 where the
 * default band (fhp_get_band) is 8 rows or fewer, FHP_MAX_DEPTH otherwise.
 * k > 1 needs width <= 32768.
 * FHP_RULES_FHP3 lattices run passes of at most 3 steps whatever k.  Results
 * do not depend on k. */
int fhp_set_depth(fhp_sim *s, uint32_t k);
int fhp_get_depth(const fhp_sim *s, uint32_t *k);

/* Rows per workgroup band of the blocked kernel (0 = library default: the
 * largest even height up to 32 whose bands give every SIMD of the device two
 * waves, or one where two would take bands of 2 rows).  Each band also reads
 * K halo rows above and below it.  Results do not depend on it.  FHP_E_INVAL
 * above the lattice height. */
int fhp_set_band(fhp_sim *s, uint32_t rows);
/* The band height fhp_step uses: the one set, or the default it resolves to. */
int fhp_get_band(const fhp_sim *s, uint32_t *rows);

/* Advances n steps (Sec. 2: motion then scattering, each step).  Asynchronous:
 * enqueued on the handle's stream.  FHP_E_STATE if t + n would reach 2^24. */
int fhp_step(fhp_sim *s, uint64_t n);

/* Computes an observable of the current state into host_dst (dst_bytes long)
 * and synchronises.  block is used by FHP_OBS_BLOCKS only. */
int fhp_observe(fhp_sim *s, int kind, uint32_t block, void *host_dst, size_t dst_bytes);

/* Copies the current state to host_dst in the byte-per-node layout (W*H bytes,
 * bit 7 = solid).  Synchronises. */
int fhp_get_state(fhp_sim *s, uint8_t *host_dst, size_t bytes);

/* Replaces the state by host_src (W*H bytes, byte-per-node layout) and sets the
 * time counter to t.  Bit 7 becomes the obstacle mask; with FHP_WALLS_CHANNEL
 * rows 0 and H-1 stay solid whatever bit 7 says.  Particles on solid nodes are
 * allowed.  Synchronises. */
int fhp_set_state(fhp_sim *s, const uint8_t *host_src, size_t bytes, uint64_t t);

/* Steps completed so far. */
int fhp_time(const fhp_sim *s, uint64_t *t);

/* Waits for the handle's work; reports asynchronous device errors. */
int fhp_sync(fhp_sim *s);

/* Releases the handle (host memory only; the workspace stays the caller's).
 * Does nothing for a batch member (released with its batch). */
void fhp_destroy(fhp_sim *s);

/* ---------------------------------------------------------------------------
 * Batches: n independent lattices (any mix of sizes, seeds and parameters)
 * advanced together by one persistent kernel.  Lattices are cut into bands of
 * rows; bands of lattices with the same row width are packed side by side into
 * one workgroup, and a persistent grid takes (pass, band group) work items from
 * a device counter.  With more than one pass per launch, a band waits for its
 * two neighbouring bands' previous pass (per-band counters on the device).
 * Each member's results are identical to those of a standalone simulation with
 * the same parameters (Sec. 2 model; the same readings as above).
 * Members need width <= 32768, height >= FHP_BATCH_MIN_HEIGHT and seven
 * planes of at most 4 GiB (width x height below about 4.9e9 nodes; larger
 * lattices run as single simulations), and all members share one rule set
 * (FHP_RULES_FHP3 batches run passes of at most 3 steps).
 * ------------------------------------------------------------------------- */
typedef struct fhp_batch fhp_batch;

/* Device workspace for a batch of the n lattices ps[0..n-1]. */
int fhp_batch_workspace_bytes(const fhp_params *ps, uint32_t n, size_t *bytes);

/* Creates the batch at t = 0 (every member in its initial state), in dev_ws
 * (caller-owned, 256-byte aligned, kept alive until fhp_batch_destroy).  All
 * work goes to hip_stream; graph replay needs a stream other than the NULL
 * stream.  Synchronises. */
int fhp_batch_create(const fhp_params *ps, uint32_t n, void *dev_ws, size_t ws_bytes,
                     void *hip_stream, fhp_batch **out);

/* Tiling of the batch kernel: depth K (0 = FHP_BATCH_MAX_DEPTH), target band height
 * (0 = from occupancy: the largest even target up to 32 whose bands give every
 * SIMD two waves, else one, else the one with most waves; per member the
 * largest even divisor of H not above it and >= K),
 * threads per workgroup (0 = smallest multiple of 64 holding the widest row),
 * passes per launch (1 = one launch per pass; 0 = all passes of an
 * fhp_batch_step call in one launch, ordered by per-band dependencies).
 * Results do not depend on the tiling.  Synchronises. */
int fhp_batch_set_tiling(fhp_batch *b, uint32_t depth, uint32_t band, uint32_t group_threads,
                         uint32_t passes_per_launch);

/* Graph replay of the launch sequence of fhp_batch_step (1 = on, the default). */
int fhp_batch_set_graph(fhp_batch *b, int enable);

/* Advances every member by n steps.  Asynchronous; FHP_E_STATE if a member's
 * time would reach 2^24. */
int fhp_batch_step(fhp_batch *b, uint64_t n);

/* Handle of member i, usable with fhp_observe, fhp_get_state, fhp_set_state,
 * fhp_time, fhp_step and fhp_sync; owned by the batch. */
int fhp_batch_member(fhp_batch *b, uint32_t i, fhp_sim **view);

/* Waits for the batch's work; FHP_E_DEVICE if a launch aborted. */
int fhp_batch_sync(fhp_batch *b);

/* Releases the batch and its member handles (not the workspace). */
void fhp_batch_destroy(fhp_batch *b);

/* ---------------------------------------------------------------------------
 * Pools: continuous batching of simulation jobs that arrive and leave.  A pool
 * owns a caller-provided device arena (the HBM budget); a job is admitted when
 * a slot, arena memory and band-table room are free, stays resident until it
 * is released, and advances with every tick together with all other resident
 * jobs (one batch-kernel launch per pass over all of them, each job clipped to
 * its remaining steps; the last steps that do not fill a pass run on the
 * single-lattice kernels).  A job's result does not depend on the other jobs
 * or on when it was admitted.  Members need width <= 32768, height >= 8 and
 * seven planes of at most 4 GiB.
 * ------------------------------------------------------------------------- */
typedef struct fhp_pool fhp_pool;

/* Arena size for max_slots jobs, max_bands bands of rows in total (a job of
 * height H uses about H/32 bands) and lattice_bytes of lattice storage (a
 * W x H job takes about 1.875*W*H bytes: two 7-plane buffers and an obstacle
 * plane). */
int fhp_pool_workspace_bytes(uint32_t max_slots, uint32_t max_bands, size_t lattice_bytes,
                             size_t *bytes);

/* Creates an empty pool in dev_arena (caller-owned, 256-byte aligned, kept
 * alive until fhp_pool_destroy).  Work goes to hip_stream (not the NULL stream
 * if ticks are to be graph-replayed). */
int fhp_pool_create(void *dev_arena, size_t arena_bytes, uint32_t max_slots, uint32_t max_bands,
                    void *hip_stream, fhp_pool **out);

/* Depth (0 = FHP_BATCH_MAX_DEPTH), target band height (0 = 32) and workgroup size
 * (0 = smallest that holds the widest row) of the pool's launches; only while
 * the pool is empty. */
int fhp_pool_set_tiling(fhp_pool *pl, uint32_t depth, uint32_t band, uint32_t group_threads);

/* Rule set (FHP_RULES_*) of every job of the pool, FHP-II until set; only
 * while the pool is empty.  fhp_pool_admit rejects jobs of another rule set
 * with FHP_E_INVAL. */
int fhp_pool_set_rules(fhp_pool *pl, uint32_t rules);

/* Admits a job: creates the lattice of *p at t = 0 in the arena and schedules
 * `steps` steps.  FHP_E_BUSY when no slot, memory or band room is free (the
 * caller keeps the job queued).  Asynchronous unless p->solid is given. */
int fhp_pool_admit(fhp_pool *pl, const fhp_params *p, uint64_t steps, uint32_t *slot);

/* Runs up to `passes` passes (depth K each) of every resident job that has
 * steps left, and finishes jobs whose remaining steps are fewer than K.
 * Asynchronous. */
int fhp_pool_tick(fhp_pool *pl, uint32_t passes);

/* Returns (and forgets) up to cap slots whose jobs have had all their steps
 * enqueued since the last call. */
int fhp_pool_done(fhp_pool *pl, uint32_t *slots, uint32_t cap, uint32_t *n_done);

/* Block sums (FHP_OBS_BLOCKS layout) of a job's current state; synchronises. */
int fhp_pool_result(fhp_pool *pl, uint32_t slot, uint32_t block, int32_t *host_dst, size_t bytes);

/* Asynchronous form of fhp_pool_result: enqueues the block sums of the job's
 * state and their copy into host_dst (pinned host memory for a truly
 * asynchronous copy; kept alive until fhp_pool_collected reports it ready). */
int fhp_pool_collect(fhp_pool *pl, uint32_t slot, uint32_t block, int32_t *host_dst,
                     size_t bytes);

/* *ready = 1 once the last fhp_pool_collect of `slot` has completed. */
int fhp_pool_collected(fhp_pool *pl, uint32_t slot, int *ready);

/* Handle of the job in `slot` (observables, state access), owned by the pool. */
int fhp_pool_member(fhp_pool *pl, uint32_t slot, fhp_sim **view);

/* Frees the slot and its arena memory.  Work already enqueued on the job runs
 * before anything that later reuses the memory (stream order). */
int fhp_pool_release(fhp_pool *pl, uint32_t slot);

/* Resident jobs and arena bytes in use / free. */
int fhp_pool_usage(const fhp_pool *pl, uint32_t *active, size_t *bytes_used, size_t *bytes_free);

/* Waits for the pool's work; FHP_E_DEVICE if a launch aborted. */
int fhp_pool_sync(fhp_pool *pl);

/* Releases the pool (not the arena). */
void fhp_pool_destroy(fhp_pool *pl);

/* ---------------------------------------------------------------------------
 * Allocation-free stepping, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.
 * ------------------------------------------------------------------------- */

/* Largest state (seven bit-planes) fhp_step_noalloc takes: 64 MiB, i.e.
 * W*H <= 76,695,844 nodes (8192 x 8192 fits).  The library keeps a device
 * array of this size on every GPU it runs on until the process ends. */
#define FHP_NOALLOC_MAX_STATE_BYTES (64u << 20)

/* Advances a lattice whose state at time t is in dev_in by n steps and writes
 * the state at time t + n to dev_out, with the kernels of fhp_step and the
 * same results bit for bit.  Enqueued on hip_stream (NULL = default stream);
 * allocates nothing, neither on the host nor on the device: runs of more than
 * one pass keep the state between passes in a library-owned device array.
 *   p:         the lattice's parameters (seed, force_rate, walls, chirality,
 *              rules; fill is unused); p->solid must be NULL;
 *   dev_in:    device, 256-byte aligned, 7 planes of H * (W/64) uint64 words
 *              each, packed (plane c at word c*H*(W/64), row y of a plane at
 *              word y*(W/64), bit b of word w is node x = 64w + b); read only;
 *   dev_out:   device, 256-byte aligned, the same layout; must not overlap
 *              dev_in (n = 0 copies dev_in);
 *   dev_solid: device, H * (W/64) uint64 words, bit set = obstacle node, or
 *              NULL for none; FHP_WALLS_CHANNEL adds rows 0 and H-1;
 *   t:         steps already done (the hash counters use it);
 *   depth:     steps per pass as for fhp_set_depth (0 = default).
 * All buffers stay the caller's and must stay alive until the work has run.
 * Errors: FHP_E_INVAL for bad parameters or pointers, FHP_E_NOMEM for a state
 * above FHP_NOALLOC_MAX_STATE_BYTES, FHP_E_STATE if t + n would reach 2^24,
 * FHP_E_DEVICE for a HIP error; nothing is enqueued on an error.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other threads) race; enqueue them on one stream.
 * The array keeps the last call's contents, and no call reads what it has not
 * written itself.  The first call on each GPU looks up the array's address:
 * make it outside graph capture. */
int fhp_step_noalloc(const fhp_params *p, const uint64_t *dev_in, uint64_t *dev_out,
                     const uint64_t *dev_solid, uint64_t t, uint64_t n, uint32_t depth,
                     void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
