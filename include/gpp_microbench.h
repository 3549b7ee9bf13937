/*
 * gpp_microbench.h -- empirical machine ceilings used to read the GPP
 * kernels' roofline (the measured-ceiling idea of the Empirical Roofline
 * Toolkit the paper cites in Sec. I).  Not part of the GPP computation.
 *
 * Each enqueues one kernel on `stream` (hipStream_t, NULL = default) and
 * returns without synchronising; the caller times it with events.
 * Return 0 on success, 1 on invalid arguments, 2 on a HIP launch error,
 * 5 when the current device is not a gfx950 (or there is none); on 1 and 5
 * nothing is enqueued.
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

/* Read bandwidth of the level that holds the working set: `blocks`
 * workgroups of 256 lanes each read a window of `window_bytes` (multiple of
 * 16) `reps` times.  shared = 0: workgroup b reads bytes
 * [b*window_bytes, (b+1)*window_bytes) of buf, so buf holds
 * blocks*window_bytes; shared != 0: every workgroup reads the first
 * window, from its own rotated start, so buf holds window_bytes.  Bytes
 * read = blocks * window_bytes * reps.  out: device double [blocks * 256]
 * (written, keeps the loads live).  A small per-workgroup window measures
 * the vector L1, a shared window of a few MB the L2, one of tens of MB the
 * MALL (Infinity Cache), and large per-workgroup windows HBM. */
int gpp_mb_read(const void *buf, int64_t window_bytes, int shared, int blocks, int reps,
                double *out, void *stream);

/* LDS access patterns of 16-byte elements, for the bank-conflict and
 * LDS-cycle counters (SQ_LDS_BANK_CONFLICT, SQ_LDS_IDX_ACTIVE): `blocks`
 * workgroups of 64 lanes, each on its own LDS array of 8 rows x 64
 * elements (e = (64 r + j, 1.0) at row r, entry j), `reps` rounds.  Lane l
 * is (tj, tk) = (l / 8, l % 8).  Per round:
 *   pattern 0: 8 writes, lane l writes entry l of every row;
 *   pattern 1: 8 reads of row tj, entries 8 tk + ((c + tk + tj) mod 8),
 *              c = 0..7 (each lane 8 consecutive entries, rotated);
 *   pattern 2: 8 reads of row tj, entries tk + 8 ((c + tj) mod 8) (each
 *              octet of lanes 128 contiguous bytes, rows staggered);
 *   pattern 3: 8 reads of row tj, entries 8 tk + c (not rotated).
 * Pattern 0 writes (64 (8 i + r) + l, 1.0) in round i; afterwards lane l
 * reads entry 63 - l of row l % 8.  out: device double [blocks * 64], lane
 * l's value: for the reads the sum over all rounds of re + im of what it
 * read, for the writes the real part read back,
 * 64 (8 (reps - 1) + l % 8) + 63 - l.  Returns as the functions above
 * (1 also for a pattern outside 0..3). */
int gpp_mb_lds(int pattern, int blocks, int reps, double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GPP_MICROBENCH_H */
