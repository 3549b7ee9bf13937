/*
 * gpp_ladder.h -- the paper's optimisation steps replayed on MI355X.
 *
 * Sec. III of the paper takes the GPP kernel through eight steps on a V100
 * (v0 baseline, v1 reciprocals for divides, v2 two-way branch, v3 squared
 * compares instead of abs(), v4 band loop serial inside each thread, v5
 * frequency loop outside the kernel, v6 cache blocking, v7 band-contiguous
 * layout of the band-indexed arrays, v8 register cap for occupancy; Table I
 * gives the times).  These entry points run the same forward reduction as
 * gpp_sigma_fwd (include/gpp.h: same arguments, same outputs, same
 * conventions) through a kernel that embodies one step of that ladder, built
 * for gfx950, so the steps can be timed against each other and against the
 * production kernel on one GPU.  They are measurement variants, not a second
 * product path: gpp_sigma_fwd is the tuned implementation.
 *
 * Steps (gpp_ladder_name gives the same text):
 *   0  v0  one thread per (band, G', G) with G fastest (the collapsed
 *          three-loop nest) in a grid-stride loop; IEEE complex divides;
 *          predicates on |x - om| and |om / (x - om)| via square roots;
 *          three-way branch
 *   1  v1  as 0, complex divides by one reciprocal (+2 Newton steps) of
 *          |denominator|^2
 *   2  v2  as 1, two-way branch (outputs preset to zero)
 *   3  v3  as 2, squared compares (the exact cross-multiplied predicate of
 *          gpp.h; from here on branch decisions are bit-identical to it)
 *   4  v4  one thread per (G', G), bands serial inside the thread, all
 *          frequencies in registers
 *   5  v5  as 4, one launch per frequency (frequency loop outside)
 *   6  v6  as 5, the aqsntemp rows of 16 bands staged in LDS and shared by
 *          the four waves of a workgroup (four G' columns, same 64 G rows)
 *   7  v7  as 6, aqsmtemp read from a band-contiguous [ngpown][number_bands]
 *          copy made by a transpose kernel inside the call
 *   8  v8  as 7, register cap of 80 VGPRs (6 waves per SIMD instead of
 *          the 5 its natural allocation gives; a few registers spill)
 *   9  m1  as 4, with the Coulomb-hole sum factored as in the production
 *          kernel (om/(x - om) = r (x om - |om|^2): two running sums per
 *          frequency, e and vcoul applied once per (G', G)), one reciprocal
 *          per term
 *  10  m2  as m1, with the denominators of 3 bands x nfreq frequencies
 *          inverted together (one reciprocal per batch) and the branch mask
 *          applied by clearing the high word
 *  11  the production forward (gpp_sigma_fwd)
 *
 * The abs() predicates of steps 0-2 take moduli by square roots and compare
 * them multiplied out (A: |x - om| > 0.5 and |om| < 500 |x - om|; B:
 * |om| > 1e-6 |x - om|), so an exact pole needs no quotient.  They describe
 * the same regions as the exact predicate, but at an exact boundary
 * (|x - om|^2 == 0.25, or |om|^2 == 250000 |x - om|^2) rounding can put a
 * term on the other side.  Steps 0-10 support nfreq 1..4.
 */
#ifndef GPP_LADDER_H
#define GPP_LADDER_H

#include "gpp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GPP_LADDER_STEPS 12
#define GPP_LADDER_MAX_NFREQ 4

/* Number of steps (GPP_LADDER_STEPS). */
int32_t gpp_ladder_steps(void);

/* Static name of a step ("v0 collapse-3, IEEE divides, abs, 3-way", ...),
 * or NULL outside [0, GPP_LADDER_STEPS). */
const char *gpp_ladder_name(int32_t step);

/* Device workspace bytes gpp_ladder_fwd needs for this step and these
 * sizes, or 0 when the dims or the step are invalid. */
size_t gpp_ladder_workspace(int32_t step, const gpp_dims *dims);

/* The forward reduction of gpp_sigma_fwd computed by ladder step `step`.
 * Arguments, layouts, ownership and error behaviour as gpp_sigma_fwd; in
 * addition GPP_ERR_INVALID for a step outside [0, GPP_LADDER_STEPS) or, for
 * steps 0-10, nfreq > GPP_LADDER_MAX_NFREQ.  The workspace (16-byte aligned)
 * must hold gpp_ladder_workspace(step, dims) bytes. */
gpp_status gpp_ladder_fwd(int32_t step, const gpp_dims *dims, const gpp_inputs *inputs,
                          double *achtemp, double *asxtemp, void *workspace,
                          size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GPP_LADDER_H */
