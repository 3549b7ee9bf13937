/*
 * gpp_oracle_ld.c -- long-double brute force for tiny GPP problems.
 *
 * TEST INFRASTRUCTURE ONLY (used to pin the fp64 oracle; never by the
 * product path).  It is written independently of gpp_oracle.c and takes
 * the plasmon-pole terms in their delw form instead of the simplified one:
 *
 *   wdiff = x - om,   delw = om / wdiff,   Omega2 = om^2 e
 *   A:  sch = delw e,         ssx = Omega2 / (x^2 - om^2)
 *   B:  sch = 0,              ssx = -Omega2 delw / (4 om^2 (delw + 1/2))
 *   C:  sch = ssx = 0
 *
 * Values and sums are in x87 80-bit long double with C99 complex
 * arithmetic.  The branch decision is the fp64 specification (the same
 * rounded quantities both the oracle and the GPU compare), evaluated here
 * with its own code; see Sec. III v2 (3-way branch) and v3 (squared
 * compares) of the paper.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>

typedef long double complex lcplx;

static int ld_branch(double x, double om_re, double om_im)
{
    const double limittwo = 0.25, limitone = 250000.0, tol_zero = 1e-12;
    double dr = x - om_re;
    double wi2 = om_im * om_im;
    double wdiffr = fma(dr, dr, wi2);
    double wtr = fma(om_re, om_re, wi2);
    int a = (wdiffr > limittwo) && (wtr < limitone * wdiffr);
    if (a) return 0;
    if (wtr > tol_zero * wdiffr) return 1;
    return 2;
}

/*
 * oracle_ld_sigma_fwd: brute-force achtemp/asxtemp over all (w, n, p, g),
 * same argument conventions as oracle_sigma_fwd (dims = {number_bands,
 * nvband, ncouls, ngpown, nfreq}); outputs rounded to fp64.  Tiny sizes only.
 */
int oracle_ld_sigma_fwd(const int64_t *dims, const double *aqsm,
                        const double *aqsn, const double *ieps,
                        const double *wt, const double *vcoul,
                        const double *wx, double *ach, double *asx)
{
    int64_t nb = dims[0], nv = dims[1], ng = dims[2], np = dims[3],
            nw = dims[4];
    if (nb < 0 || nv < 0 || ng < 0 || np < 0 || nw < 0 || nv > nb || np > ng)
        return 1;
    for (int64_t w = 0; w < nw; ++w) {
        lcplx sum_ch = 0.0L, sum_sx = 0.0L;
        for (int64_t n = 0; n < nb; ++n) {
            long double x = wx[w * nb + n];
            for (int64_t p = 0; p < np; ++p) {
                lcplx m = (long double)aqsm[2 * (n * ng + p)] +
                          I * (long double)aqsm[2 * (n * ng + p) + 1];
                for (int64_t g = 0; g < ng; ++g) {
                    int64_t pg = p * ng + g, ngi = n * ng + g;
                    lcplx an = (long double)aqsn[2 * ngi] +
                               I * (long double)aqsn[2 * ngi + 1];
                    lcplx om = (long double)wt[2 * pg] +
                               I * (long double)wt[2 * pg + 1];
                    lcplx e = (long double)ieps[2 * pg] +
                              I * (long double)ieps[2 * pg + 1];
                    long double v = vcoul[g];
                    lcplx matngmatmgp = an * conjl(m);
                    int br = ld_branch(wx[w * nb + n], wt[2 * pg], wt[2 * pg + 1]);
                    lcplx sch = 0.0L, ssx = 0.0L;
                    if (br != 2) {
                        lcplx wdiff = x - om;
                        lcplx delw = om / wdiff;
                        lcplx omega2 = om * om * e;
                        if (br == 0) {
                            sch = delw * e;
                            ssx = omega2 / (x * x - om * om);
                        } else {
                            ssx = -omega2 * delw / (4.0L * om * om * (delw + 0.5L));
                        }
                    }
                    sum_ch += 0.5L * v * matngmatmgp * sch;
                    if (n < nv) sum_sx += v * matngmatmgp * ssx;
                }
            }
        }
        ach[2 * w] = (double)creall(sum_ch);
        ach[2 * w + 1] = (double)cimagl(sum_ch);
        asx[2 * w] = (double)creall(sum_sx);
        asx[2 * w + 1] = (double)cimagl(sum_sx);
    }
    return 0;
}
