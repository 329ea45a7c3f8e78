/*
 * fhp_cpu.h -- C ABI of the host bit-plane FHP stepper (libfhpcpu.so).
 *
 * A multi-core SIMD implementation of the same FHP time step as the GPU
 * library (fhp.h), for the host CPU: the counterpart of the paper's
 * vectorised and threaded CPU codes (arXiv:1208.2428, Sec. 3.1 and the
 * SSE/AVX/pthreads rows of Table 1 in Sec. 4), built on bit-planes instead of
 * a byte per node.  It computes exactly the dynamics fhp.h defines, with the
 * same readings (numbering, FHP-II rules, stream -> collide or bounce back ->
 * force, SplitMix64 chirality and forcing coin, initial state), so its states
 * are bit-identical to the GPU library's and the CPU oracle's.
 *
 * Layout: seven bit-planes of uint64 words (bit b of word w of row y is node
 * x = 64w + b) plus a solid plane, two buffers.  Rows are split over threads
 * (OpenMP); along a row the per-word update runs on SIMD lanes (AVX-512 or
 * AVX2, chosen at load time from what the CPU supports, else plain 64-bit
 * code).  Rule set: FHP-II only.
 *
 * Calls return 0 (FHPCPU_OK) or a negative error code; fhpcpu_last_error()
 * gives a message for the calling thread's last failure.  A handle is not
 * thread-safe (it uses threads internally).  The caller owns every buffer it
 * passes; the library copies what it keeps.
 */
#ifndef FHP_CPU_H
#define FHP_CPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FHPCPU_OK = 0, FHPCPU_E_INVAL = -1, FHPCPU_E_NOMEM = -2, FHPCPU_E_STATE = -4 };

typedef struct fhpcpu_sim fhpcpu_sim;

/* Message of the calling thread's last failure ("" if none). */
const char *fhpcpu_last_error(void);

/* Creates a W x H lattice (Sec. 2: seven channels per node, boundary flag;
 * W a multiple of 64, H even, both >= 2 and below 2^20).  fill in [0, 1] is
 * the per-channel occupancy of fluid nodes at t = 0; force_rate in [0, 1/64)
 * the forcing rate per node and step; walls != 0 makes rows 0 and H-1 solid;
 * solid (nullable) is a W*H row-major host mask, nonzero = obstacle, copied. */
int fhpcpu_create(uint32_t width, uint32_t height, uint64_t seed, double fill,
                  double force_rate, int walls, const uint8_t *solid, fhpcpu_sim **out);

/* Advances n steps on `threads` threads (<= 0: the OpenMP default).
 * FHPCPU_E_STATE if the time would reach 2^24. */
int fhpcpu_step(fhpcpu_sim *s, uint64_t n, int threads);

/* State in the paper's byte-per-node layout (Fig. 1): W*H bytes, row-major,
 * bits 0-5 moving, bit 6 rest, bit 7 solid. */
int fhpcpu_get_state(const fhpcpu_sim *s, uint8_t *dst, size_t bytes);

/* Replaces the state (byte layout; bit 7 becomes the obstacle mask, wall rows
 * stay solid) and sets the time to t. */
int fhpcpu_set_state(fhpcpu_sim *s, const uint8_t *src, size_t bytes, uint64_t t);

/* Steps done so far. */
int fhpcpu_time(const fhpcpu_sim *s, uint64_t *t);

/* State digest: the sum over planes c = 0..7 (7 = solid), rows y and words w
 * of H(plane word, c*2^40 + y*2^20 + w) mod 2^64, the same value the GPU
 * library's FHP_OBS_DIGEST returns. */
int fhpcpu_digest(const fhpcpu_sim *s, uint64_t *out);

/* Instruction set of the update loop in use: "avx512", "avx2" or "generic". */
const char *fhpcpu_isa(void);

void fhpcpu_destroy(fhpcpu_sim *s);

#ifdef __cplusplus
}
#endif
#endif
