/* fhp_calib.h -- streaming reference kernels: the memory ceiling of a pass.
 *
 * Not part of the FHP dynamics.  A pass of the blocked step kernel reads the
 * seven bit-planes of a lattice (and its obstacle plane) band by band, row by
 * row, one 64-bit word per thread through buffer resources, and writes seven
 * planes.  fhp_calib_pass performs exactly those memory accesses with no
 * arithmetic, so its bandwidth is the most a pass of that shape can reach on
 * the device; fhp_calib_flat streams a flat buffer with 16-byte accesses per
 * thread, the device's plain streaming bandwidth.  bench.py reports the step
 * kernel's bandwidth against both, beside the 8 TB/s HBM specification.
 *
 * Same conventions as fhp.h: every call returns FHP_OK or a negative FHP_E_*
 * code with a message from fhp_last_error(); pointers are device pointers the
 * caller owns; calls are asynchronous on the given HIP stream (NULL = the
 * default stream).
 */
#ifndef FHP_CALIB_H
#define FHP_CALIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FHP_CALIB_COPY = 0,  /* read every input word, write it to the output      */
    FHP_CALIB_READ = 1,  /* read every input word; one word per thread written */
    FHP_CALIB_WRITE = 2  /* write every output word (a constant), read nothing */
};

/* The access pattern of one blocked pass.
 *   in, out:   seven planes each, plane c at base + c * plane_stride words,
 *              word (y, w) of a plane at y * wd + w; 7 * plane_stride * 8 bytes
 *              must stay below 4 GiB;
 *   mask:      one more plane read with the input planes (NULL = none);
 *   wd:        words per row, 1 .. 512 (one thread per word, a workgroup per band);
 *   H:         rows (>= 1); band: rows per workgroup (>= 1);
 *   halo:      rows loaded above and below every band as well (0 .. 8), wrapping
 *              at the lattice edges, as a pass of that depth loads them.
 * COPY writes band rows of the seven input planes to the same place in out;
 * READ writes one XOR of everything a thread read to out[band * wd + w], so out
 * must hold at least ceil(H / band) * wd words; WRITE reads nothing.
 * Errors: FHP_E_INVAL for sizes outside these limits or NULL buffers the mode
 * needs; FHP_E_DEVICE if the launch fails. */
int fhp_calib_pass(int mode, const uint64_t* in, uint64_t* out, const uint64_t* mask, uint32_t wd,
                   uint32_t H, uint64_t plane_stride, uint32_t band, uint32_t halo, void* hip_stream);

/* Plain streaming of `bytes` bytes (a positive multiple of 16; src and dst
 * 16-byte aligned, not overlapping): COPY src -> dst, READ src (one 16-byte
 * XOR per thread written to dst, which must then hold blocks * 256 * 16 bytes,
 * blocks as returned through *blocks_used), WRITE dst.  `blocks` workgroups of
 * 256 threads stride over the buffer (0 = 8 per compute unit).
 * Errors: FHP_E_INVAL, FHP_E_DEVICE as above. */
int fhp_calib_flat(int mode, const void* src, void* dst, size_t bytes, uint32_t blocks,
                   uint32_t* blocks_used, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FHP_CALIB_H */
