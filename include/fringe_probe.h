/*
 * fringe_probe.h -- roof probes of libfringe.so: two plain kernels that
 * measure what the device achieves on its two roofs, so that the search's
 * figures can be read against measured as well as published peaks.  They
 * are not part of the search.
 *
 * Conventions as in fringe.h (0 or a negative FRINGE_E_* code, detail in
 * fringe_last_error()).  Both calls only enqueue work on hip_stream (NULL =
 * the default stream); the caller times them (e.g. with HIP events on the
 * same stream) and owns every buffer.
 */
#ifndef FRINGE_PROBE_H
#define FRINGE_PROBE_H

#include <stdint.h>

#include "fringe.h"

#ifdef __cplusplus
extern "C" {
#endif

/* FP32 FMA loop: n_blocks workgroups of 256 lanes, each lane running 16
 * independent chains of `iters` fused multiply-adds (non-packed FP32
 * instructions, like the search kernels), then storing one float to
 * d_out[block * 256 + lane] (so d_out holds n_blocks * 256 floats).
 * *flops receives the floating-point operations of one launch:
 * 2 * 16 * iters * 256 * n_blocks.  Errors: FRINGE_E_INVALID for a null
 * pointer, n_blocks outside [1, 2^31 - 1] or iters < 1; FRINGE_E_HIP for a
 * failed launch. */
int fringe_probe_fma(int64_t n_blocks, int32_t iters, float* d_out, double* flops,
                     void* hip_stream);

/* Device-to-device copy of `bytes` bytes (a multiple of 16; both pointers
 * 16-byte aligned, buffers not overlapping) by a grid-stride kernel of
 * 16-byte loads and stores: `bytes` read and `bytes` written in HBM.
 * Errors: FRINGE_E_INVALID for null pointers, bytes < 16, bytes not a
 * multiple of 16 or misaligned pointers; FRINGE_E_HIP for a failed launch. */
int fringe_probe_copy(const void* d_src, void* d_dst, int64_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FRINGE_PROBE_H */
