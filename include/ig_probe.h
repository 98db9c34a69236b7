/*
 * ig_probe.h -- attainable-peak probes of libig's device (measurement only).
 *
 * The subset-test contractions of the method (Eq. 3, Eq. 2 and Eq. 4 evaluated
 * as dense products, see ig.h) run on the fp4 matrix cores; the candidate
 * de-duplication stages stream HBM.  These calls measure what the device
 * actually delivers for each, so that the kernels' rates can be stated as
 * fractions of a measured peak as well as of the vendor's figure.  They compute
 * nothing of the method and never touch a model.
 *
 * Conventions as in ig.h: device pointers are named d_*, every call returns an
 * ig_status (ig_last_error() holds the text), work is ordered on `stream` and
 * the call waits for it before returning.
 */
#ifndef IG_PROBE_H
#define IG_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include "ig.h"

#ifdef __cplusplus
extern "C" {
#endif

/* fp4 matrix-core rate: every SIMD of the device issues `iters` x 4 independent
 * v_mfma_scale_f32_32x32x64_f8f6f4 (fp4 e2m1 operands, fp32 accumulators) per
 * wave, 8 waves per SIMD.  *ops_per_s = 2 * 32 * 32 * 64 operations per
 * instruction / the launch's duration; *ms (may be NULL) = that duration.
 * iters in 1 .. 2^24 (IG_E_INVAL otherwise).  Uses a few KB of scratch. */
ig_status ig_probe_mfma_fp4(uint32_t iters, void *stream, double *ops_per_s, float *ms);

/* HBM copy rate: `bytes` (a positive multiple of 16) from d_src to d_dst with
 * 16-byte loads and stores; *bytes_per_s = 2 * bytes (read + write) / the
 * launch's duration, *ms (may be NULL) = that duration.  Both buffers belong to
 * the caller, are 16-byte aligned and do not overlap (IG_E_INVAL otherwise). */
ig_status ig_probe_hbm_copy(const void *d_src, void *d_dst, size_t bytes, void *stream, double *bytes_per_s,
                            float *ms);

#ifdef __cplusplus
}
#endif
#endif /* IG_PROBE_H */
