/*
 * gpp_microbench.h -- empirical machine ceilings used to read the GPP
 * kernels' roofline (the measured-ceiling idea of the Empirical Roofline
 * Toolkit the paper cites in Sec. I).  Not part of the GPP computation.
 *
 * Both enqueue one kernel on `stream` (hipStream_t, NULL = default) and
 * return without synchronising; the caller times them with events.
 * Return 0 on success, 1 on invalid arguments, 2 on a HIP launch error.
 */
#ifndef GPP_MICROBENCH_H
#define GPP_MICROBENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* fp64 FMA issue rate: `blocks` workgroups of 256 lanes, each lane running
 * 16 independent FMA chains for `iters` rounds.  out: device double
 * [blocks * 256] (written, keeps the work live).  *flops (host, may be
 * NULL) receives the fp64 operation count (an FMA counts 2). */
int gpp_mb_fp64_fma(double *out, int blocks, int iters, void *stream, double *flops);

/* Streaming copy of `bytes` (multiple of 16) from src to dst (device,
 * 16-byte aligned, non-overlapping) with `blocks` workgroups of 256 lanes:
 * reads and writes exactly `bytes` each, the reference for scaling
 * FETCH_SIZE / WRITE_SIZE hardware counters. */
int gpp_mb_copy(const void *src, void *dst, int64_t bytes, int blocks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GPP_MICROBENCH_H */
