// gpp_bwd.hip -- adjoint of the GPP reduction on gfx950 (fp64, no MFMA).
//
// Loss L = sum_w Re(conj(ga[w]) achtemp[w] + conj(gs[w]) asxtemp[w]); the
// gradient of a complex input z is dL/dRe z + i dL/dIm z (no derivative
// through the branch).  Nothing is stored by the forward: every term's
// wdiff, reciprocal and branch are recomputed here.
//
// Per (n, p, g), with u_w = conj(1/(x_w - om)) for branch-A terms (else 0)
// and the exchange quantities of occupied bands (ssx = e sigma,
// d ssx/d om = e delta):
//   K  = sum_w ga_w/2 u_w            L  = sum_w x_w ga_w/2 u_w^2
//   KS = sum_w gs_w conj(sigma_w)    LS = sum_w gs_w conj(delta_w)
//   Z  = conj(om) K + KS             W  = L + LS
// the gradients are
//   dI_eps[p][g]    = vcoul[g]         sum_n conj(M) Z
//   dwtilde[p][g]   = vcoul[g] conj(e) sum_n conj(M) W
//   daqsntemp[n][g] = sum_p vcoul[g] conj(e) aqsmtemp[n][p] Z
//   daqsmtemp[n][p] = sum_g vcoul[g] e aqsntemp[n][g] conj(Z)
// with M = aqsntemp[n][g] conj(aqsmtemp[n][p]).
//
// Kernels.  bwd_pairs (lane = g, wave-uniform p, bands serial) writes
// dwtilde and dI_eps.  K and L are linear in ga/2, so over unoccupied bands
// (with at most four frequencies) the lane never forms them: it keeps four
// sums per frequency over the bands, weighted by conj(M),
//   A2_w = sum_n conj(M) r,           B1_w = sum_n conj(M) x r,
//   B2_w = sum_n conj(M) x r^2,       B3_w = sum_n conj(M) x (x - Re om) r^2
// (r the reciprocal of |x - om|^2 on branch-A terms, which add nothing
// otherwise) and applies ga/2 once at the end: with u = (x - om) r and, on
// branch A, |x - om|^2 r = 1,
//   sum_n conj(M) K = sum_w ga_w/2 (B1_w - om A2_w),
//   sum_n conj(M) L = sum_w ga_w/2 (B1_w - 2 (Im om)^2 B2_w - 2i Im om B3_w).
// Occupied bands, a ragged tail and more frequencies form K and L per band.
// bwd_bands (lane = g; a workgroup of four waves owns kBandTile bands and
// 256 consecutive rows, 64 per wave, and walks a range of G' columns)
// forms vcoul conj(e) Z per term, adds aqsmtemp[n][p] times it into
// daqsntemp (registers), and takes aqsntemp[n][g] conj(vcoul conj(e) Z) =
// vcoul e aqsntemp conj(Z) as the term of daqsmtemp[n][p]: those terms go
// through a per-wave LDS slab (8 lanes per row, then a DPP sum over the 8),
// are added over the workgroup's four waves and written as one partial per
// 256-row block; reduce_am sums the partials in a fixed order and zero-fills
// columns >= ngpown.  No atomics: results are bitwise reproducible.
#include "gpp_device.h"
#include "gpp_internal.h"

namespace gpp {

constexpr int kBwdWaves = 4;
constexpr int kBwdThreads = kBwdWaves * kWave;
constexpr int kRowsPerBlock = kBwdWaves * kWave;  // g rows per workgroup (both kernels)
// Bands per batch-inverted group of the per-band forms: 3, or 1 with more
// than four frequencies, so that a group never holds more than 12
// denominators (the range for which batch_reciprocal's (Im om)^2 >= 2^-60
// lane test keeps every prefix product normal).
constexpr int bwd_group(int nw) { return nw <= 4 ? 3 : 1; }
// The pairs kernel's band-sum form: frequencies it takes, and bands per
// batch-inverted group there (at most 12 / 4 = 3).
constexpr int kPairsSumsMaxNW = 4;
#ifndef GPP_BWD_PAIRS_GROUP
#define GPP_BWD_PAIRS_GROUP 2
#endif
constexpr int kPairsGroup = GPP_BWD_PAIRS_GROUP;
static_assert(kPairsGroup * kPairsSumsMaxNW <= 12, "pairs groups hold at most 12 denominators");
constexpr int kOctet = 8;                          // lanes that share one row sum
// Minimum waves per SIMD the compiler must allow (register cap): pairs with
// at most three frequencies (128 VGPRs; more frequencies take 3 waves, as
// their band sums need more registers), and the bands kernel without and
// with the daqsmtemp sums.  Bands per bands-kernel workgroup: four, so
// that the daqsmtemp slab of two columns fills the 8 rows an octet of
// lanes reduces.  Measured on MI355X at the adjoint workload's sizes
// against three bands at 5 and 4 waves: the kernel with daqsmtemp 4.5 %
// faster at nfreq 3 (7.39 against 7.74 ms; at 4 waves, with four bands,
// it spilled and ran 28 % slower), without daqsmtemp 3 % faster at nfreq 3
// and 2-2.5x faster at nfreq 4 and 8, where three bands at 5 waves spilled;
// the whole adjoint 1 % and 5 % faster at nfreq 3 and 4, 1-2 % slower at
// nfreq 5 and 8.
#ifndef GPP_BWD_PAIRS_WAVES
#define GPP_BWD_PAIRS_WAVES 4
#endif
constexpr int pairs_waves(int nw) { return nw <= 3 ? GPP_BWD_PAIRS_WAVES : 3; }
#ifndef GPP_BWD_BANDS_WAVES
#define GPP_BWD_BANDS_WAVES 4
#endif
#ifndef GPP_BWD_BANDS_AM_WAVES
#define GPP_BWD_BANDS_AM_WAVES 3
#endif
#ifndef GPP_BWD_BAND_TILE
#define GPP_BWD_BAND_TILE 4
#endif
constexpr int kBandTile = GPP_BWD_BAND_TILE;       // bands per bands-kernel workgroup
// Bands-kernel p-range split (see bwd_geometry): resident bands waves of the
// MI355X (256 CUs x 4 SIMDs x GPP_BWD_BANDS_WAVES), rounds of them to aim
// at, and the shortest segment.
#ifndef GPP_BWD_BANDS_ROUNDS
#define GPP_BWD_BANDS_ROUNDS 16
#endif
constexpr long kBandsWaveSlots = 256L * 4 * GPP_BWD_BANDS_WAVES;
constexpr int kBandsRounds = GPP_BWD_BANDS_ROUNDS;
constexpr int kMinSegCols = 64;
// Bands per batch-inverted group of the bands kernel: the largest divisor
// of the band tile whose group holds at most 12 denominators.
constexpr int bands_group(int nw)
{
    for (int g = kBandTile; g > 1; --g)
        if (kBandTile % g == 0 && g * nw <= 12) return g;
    return 1;
}
// daqsmtemp sums of the bands kernel: the slab holds the terms of two G'
// columns (kBandTile rows each); every kAmCols columns (even) the four
// waves' row sums are added and written.
constexpr int kSlabRows = 2 * kBandTile;
constexpr int kAmCols = 16;
constexpr int kAmRows = kBandTile * kAmCols;
static_assert(kSlabRows <= kOctet && kAmCols % 2 == 0, "slab layout");

// Upstream gradient scaled for the kernels: gh[w] = ga[w]/2 and
// xgh[w][n] = wx[w][n] ga[w]/2, written once by bwd_prepare.
__global__ void bwd_prepare(int nb, int nw, const double *__restrict__ wx,
                            const double2 *__restrict__ ga, double2 *__restrict__ gh,
                            double2 *__restrict__ xgh)
{
    // 64-bit: nfreq x number_bands passes 2^31 from 2^28 bands on
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) gh[i] = make_double2(0.5 * ga[i].x, 0.5 * ga[i].y);
    if (i < (long)nw * nb) {
        const int w = (int)(i / nb);
        const double x = wx[i];
        xgh[i] = make_double2(0.5 * x * ga[w].x, 0.5 * x * ga[w].y);
    }
}

// Lane exchange inside a row of 16 lanes (DPP), both halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    // every source lane of the controls used here exists, so no lane keeps
    // an old value (bound_ctrl only matters for lanes outside the row)
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over each aligned group of 8 lanes; every lane of the group gets it.
__device__ __forceinline__ double octet_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);  // row_half_mirror: lane i <-> 7 - i within 8
    return v;
}

// Order this wave's LDS writes before its later LDS reads (and the reverse)
// when lanes exchange data through LDS without a workgroup barrier.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exchange term of an occupied band: ssx = e sigma, d ssx/d om = e delta,
// with d = x - om, s = x + om and D = d s = x^2 - om^2:
//   A:  sigma = om^2 / D,       delta = 2 om x^2 / D^2
//   B:  sigma = -om / (2 s),    delta = -x / (2 s^2)
// evaluated without a divide as in the forward: 1/D = conj(D) r rs and
// 1/s = conj(s) rs with r = 1/|d|^2, rs = 1/|s|^2, where conj(D) =
// (fma(Re d, Re s, (Im om)^2), 2 Re om Im om) and om conj(s) =
// (fma(Re om, Re s, (Im om)^2), Im om x).
__device__ inline void sx_sigma_delta(double x, double a, double b, double wi2, double wtr,
                                      double thr, cplx &sigma, cplx &delta)
{
    const double dr = x - a, sp = x + a;
    const double wd = fma(dr, dr, wi2);
    if (wd > thr) {  // A
        const double ws = fma(sp, sp, wi2);
        const double q = rcp_nr2(wd) * rcp_nr2(ws);
        const double ab2 = 2.0 * a * b;
        const cplx cd = cmake(fma(dr, sp, wi2), ab2);  // conj(D)
        const cplx om2 = cmake(fma(a, a, -wi2), ab2);  // om^2
        sigma = cscale(q, cmul(om2, cd));
        const cplx cd2 = cmul(cd, cd);
        delta = cscale(2.0 * x * x * q * q, cmul(cmake(a, b), cd2));
    } else if (branch_b_holds(wtr, wd)) {  // B
        const double ws = fma(sp, sp, wi2);
        const double h = -0.5 * rcp_nr2(ws);
        sigma = cmake(fma(a, sp, wi2) * h, (b * x) * h);
        // conj(s)^2 = (sp^2 - b^2, -2 sp b)
        const double hh = h * rcp_nr2(ws) * x;
        delta = cmake(fma(sp, sp, -wi2) * hh, -2.0 * sp * b * hh);
    } else {
        sigma = delta = cmake(0.0, 0.0);
    }
}

// K (and, with WANT_L, L) of BU bands starting at band n for one lane:
// batch-inverted reciprocals over the BU*NW terms, masked to branch A.
template <int NW, int BU, bool WANT_L>
__device__ __forceinline__ void ch_bands_kl(int n, int nb, const double *__restrict__ wx,
                                            const double2 *__restrict__ gh,
                                            const double2 *__restrict__ xgh, double a, double b,
                                            double wi2, double thr, bool wide, cplx (&K)[BU],
                                            cplx (&L)[BU])
{
    constexpr int Kt = BU * NW;
    double xs[Kt], dc[Kt], drs[Kt], r[Kt];
    bool isA[Kt];
#pragma unroll
    for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int w = 0; w < NW; ++w) xs[u * NW + w] = wx[(size_t)w * nb + n + u];
#pragma unroll
    for (int k = 0; k < Kt; ++k) {
        drs[k] = xs[k] - a;
        const double wd = fma(drs[k], drs[k], wi2);
        isA[k] = wd > thr;
        dc[k] = wd;  // unclamped: see batch_reciprocal
    }
    batch_reciprocal<Kt>(dc, r, wide);
#pragma unroll
    for (int u = 0; u < BU; ++u) {
        K[u] = L[u] = cmake(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int k = u * NW + w;
            const double re = mask_keep(isA[k], r[k]);
            const cplx uu = cmake(drs[k] * re, -b * re);  // conj(1/(x - om))
            cmac(K[u], cload(gh + w), uu);
            if (WANT_L) cmac(L[u], cload(xgh + (size_t)w * nb + n + u), cmul(uu, uu));
        }
    }
}

// KS, LS of one occupied band n for one lane.
template <int NW>
__device__ __forceinline__ void sx_band_kl(int n, int nb, const double *__restrict__ wx,
                                           const double2 *__restrict__ gs, double a, double b,
                                           double wi2, double wtr, double thr, cplx &KS, cplx &LS)
{
    KS = LS = cmake(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        cplx sigma, delta;
        sx_sigma_delta(wx[(size_t)w * nb + n], a, b, wi2, wtr, thr, sigma, delta);
        const cplx g = cload(gs + w);
        cmac(KS, g, cmake(sigma.re, -sigma.im));
        cmac(LS, g, cmake(delta.re, -delta.im));
    }
}

struct PairState {
    double a, b, wi2, wtr, thr;
    double b2, wi2x2;  // 2 Im om and 2 (Im om)^2
    bool wide;  // (Im om)^2 >= kMinUnclampedWi2: batch inversion allowed
    cplx om, e, ve;  // ve = vcoul[g] e (0 for rows beyond ncouls)
};

__device__ __forceinline__ PairState load_pair(const double2 *wt, const double2 *ieps,
                                               const double *vcoul, int p, int ng, int gc,
                                               bool valid)
{
    PairState s;
    s.om = cload(wt + (size_t)p * ng + gc);
    s.e = cload(ieps + (size_t)p * ng + gc);
    s.a = s.om.re;
    s.b = s.om.im;
    s.wi2 = s.b * s.b;
    s.b2 = 2.0 * s.b;
    s.wi2x2 = 2.0 * s.wi2;
    s.wtr = fma(s.a, s.a, s.wi2);
    s.thr = branch_a_threshold(s.wtr);
    s.wide = s.wi2 >= kMinUnclampedWi2;
    s.ve = cscale(valid ? vcoul[gc] : 0.0, s.e);
    return s;
}

// One branch-A term of the pairs kernel's band sums: A2 += cM r,
// B1 += cM x r, B2 += cM x r^2, B3 += cM x dr r^2 (dr = x - Re om), with
// the compare d > thr as the execution mask (a term off branch A adds
// nothing, whatever its reciprocal).
__device__ __forceinline__ void pairs_term(double d, double thr, double r, double x, double dr,
                                           cplx cm, cplx &A2, cplx &B1, cplx &B2, cplx &B3)
{
#if GPP_EXEC_MASK == 2
    unsigned long long saved;
    double xr, xr2, xdr2;
    asm("s_mov_b64 %[sv], exec\n\t"
        "v_cmpx_gt_f64_e32 vcc, %[d], %[thr]\n\t"
        "v_mul_f64 %[xr], %[r], %[x]\n\t"
        "v_fma_f64 %[a2r], %[r], %[cr], %[a2r]\n\t"
        "v_fma_f64 %[a2i], %[r], %[ci], %[a2i]\n\t"
        "v_mul_f64 %[xr2], %[xr], %[r]\n\t"
        "v_fma_f64 %[b1r], %[xr], %[cr], %[b1r]\n\t"
        "v_fma_f64 %[b1i], %[xr], %[ci], %[b1i]\n\t"
        "v_mul_f64 %[xdr2], %[xr2], %[dr]\n\t"
        "v_fma_f64 %[b2r], %[xr2], %[cr], %[b2r]\n\t"
        "v_fma_f64 %[b2i], %[xr2], %[ci], %[b2i]\n\t"
        "v_fma_f64 %[b3r], %[xdr2], %[cr], %[b3r]\n\t"
        "v_fma_f64 %[b3i], %[xdr2], %[ci], %[b3i]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [sv] "=&s"(saved), [xr] "=&v"(xr), [xr2] "=&v"(xr2), [xdr2] "=&v"(xdr2),
          [a2r] "+v"(A2.re), [a2i] "+v"(A2.im), [b1r] "+v"(B1.re), [b1i] "+v"(B1.im),
          [b2r] "+v"(B2.re), [b2i] "+v"(B2.im), [b3r] "+v"(B3.re), [b3i] "+v"(B3.im)
        : [d] "v"(d), [thr] "v"(thr), [r] "v"(r), [x] "s"(x), [dr] "v"(dr), [cr] "v"(cm.re),
          [ci] "v"(cm.im)
        : "vcc");
#else
    const double rm = mask_keep(d > thr, r);
    const double xr = rm * x, xr2 = xr * rm, xdr2 = xr2 * dr;
    A2.re = fma(rm, cm.re, A2.re);
    A2.im = fma(rm, cm.im, A2.im);
    B1.re = fma(xr, cm.re, B1.re);
    B1.im = fma(xr, cm.im, B1.im);
    B2.re = fma(xr2, cm.re, B2.re);
    B2.im = fma(xr2, cm.im, B2.im);
    B3.re = fma(xdr2, cm.re, B3.re);
    B3.im = fma(xdr2, cm.im, B3.im);
#endif
}

// G unoccupied bands n .. n+G-1 of one lane into the band sums: one batch
// inversion over the G*NW denominators, then pairs_term per term.
template <int NW, int G>
__device__ __forceinline__ void pairs_sums_group(int n, int nb, int ng, gptr<double2> aqsn,
                                                 uint32_t goff, gptr<double2> am_col,
                                                 gptr<double> wx, const PairState &ps,
                                                 cplx (&A2)[NW], cplx (&B1)[NW],
                                                 cplx (&B2)[NW], cplx (&B3)[NW])
{
    constexpr int Kt = G * NW;
    double xs[Kt], drs[Kt], dc[Kt], r[Kt];
    // the group's aqsntemp and aqsmtemp loads go first, so that their
    // latency overlaps the reciprocal chain
    cplx an[G], am[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        an[u] = load_row_elem(aqsn + (size_t)(n + u) * ng, ng, goff);
        am[u] = cload(am_col + (size_t)(n + u) * ng);
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
        for (int w = 0; w < NW; ++w) xs[u * NW + w] = wx[(size_t)w * nb + n + u];
#pragma unroll
    for (int k = 0; k < Kt; ++k) {
        drs[k] = xs[k] - ps.a;
        dc[k] = fma(drs[k], drs[k], ps.wi2);  // unclamped: see batch_reciprocal
    }
    batch_reciprocal<Kt>(dc, r, ps.wide);
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const cplx cM = cmul_conj(am[u], an[u]);  // conj(M) = conj(an) am
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int k = u * NW + w;
            pairs_term(dc[k], ps.thr, r[k], xs[k], drs[k], cM, A2[w], B1[w], B2[w], B3[w]);
        }
    }
}

// Bands [n, n_end) of one lane in the per-band form: K and L (and, for
// occupied bands, KS and LS) per band, then Ge += conj(M) Z and
// Gw += conj(M) W.
template <int NW>
__device__ __forceinline__ void pairs_per_band(int n, int n_end, int nb, int nv, int ng,
                                               const double2 *__restrict__ aqsn,
                                               const double2 *__restrict__ am_col,
                                               const double *__restrict__ wx,
                                               const double2 *__restrict__ gh,
                                               const double2 *__restrict__ xgh,
                                               const double2 *__restrict__ gs,
                                               const PairState &ps, uint32_t goff, cplx &Ge,
                                               cplx &Gw)
{
    constexpr int G = bwd_group(NW);
    const cplx cw = cmake(ps.om.re, -ps.om.im);  // conj(om)
    while (n < n_end) {
        // bands n .. n+cnt-1 form one batch-inverted group
        const bool occ = n < nv;
        const int cnt = (!occ && n + G <= n_end) ? G : 1;
        cplx K[G], L[G];
        if (cnt == G) {
            ch_bands_kl<NW, G, true>(n, nb, wx, gh, xgh, ps.a, ps.b, ps.wi2, ps.thr, ps.wide, K,
                                     L);
        } else {
            cplx K1[1], L1[1];
            ch_bands_kl<NW, 1, true>(n, nb, wx, gh, xgh, ps.a, ps.b, ps.wi2, ps.thr, ps.wide, K1,
                                     L1);
            K[0] = K1[0];
            L[0] = L1[0];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            if (u >= cnt) break;  // wave-uniform
            const int nn = n + u;
            cplx Z = cmul(cw, K[u]);
            cplx W = L[u];
            if (nn < nv) {
                cplx KS, LS;
                sx_band_kl<NW>(nn, nb, wx, gs, ps.a, ps.b, ps.wi2, ps.wtr, ps.thr, KS, LS);
                Z = cadd(Z, KS);
                W = cadd(W, LS);
            }
            const cplx an = load_row_elem(as_global(aqsn) + (size_t)nn * ng, ng, goff);
            const cplx am = cload(am_col + (size_t)nn * ng);
            const cplx cM = cmul_conj(am, an);  // conj(M) = conj(an) am
            cmac(Ge, cM, Z);
            cmac(Gw, cM, W);
        }
        n += cnt;
    }
}

// ---- pairs kernel: dwtilde and dI_eps -------------------------------------
// Workgroup = 256 rows (one 64-row tile per wave) x one G' column p, p
// fastest, so concurrently resident workgroups share one row block.
template <int NW>
__global__ void __launch_bounds__(kBwdThreads)
__attribute__((amdgpu_waves_per_eu(pairs_waves(NW))))
bwd_pairs(int nb, int nv, int ng, int np, long nblocks, const double2 *__restrict__ aqsm,
          const double2 *__restrict__ aqsn, const double2 *__restrict__ ieps,
          const double2 *__restrict__ wt, const double *__restrict__ vcoul,
          const double *__restrict__ wx, const double2 *__restrict__ gh,
          const double2 *__restrict__ xgh, const double2 *__restrict__ gs,
          double2 *__restrict__ grad_wt, double2 *__restrict__ grad_ieps)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const long blk = xcd_remap(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;  // no barriers in this kernel
    const int gb = (int)(blk / np);
    const int p = (int)(blk - (long)gb * np);
    const int g = gb * kRowsPerBlock + wid * kWave + lane;
    const bool valid = g < ng;
    const int gc = valid ? g : ng - 1;
    const PairState ps = load_pair(wt, ieps, vcoul, p, ng, gc, valid);
    const double2 *am_col = aqsm + p;
    const uint32_t goff = (uint32_t)gc * (uint32_t)sizeof(double2);

    cplx Ge = cmake(0.0, 0.0), Gw = cmake(0.0, 0.0);
    // occupied bands
    const int nocc = nv < nb ? nv : nb;
    pairs_per_band<NW>(0, nocc, nb, nv, ng, aqsn, am_col, wx, gh, xgh, gs, ps, goff, Ge, Gw);
    int n = nocc;
    if constexpr (NW <= kPairsSumsMaxNW) {
        cplx A2[NW], B1[NW], B2[NW], B3[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) A2[w] = B1[w] = B2[w] = B3[w] = cmake(0.0, 0.0);
        for (; n + kPairsGroup <= nb; n += kPairsGroup)
            pairs_sums_group<NW, kPairsGroup>(opaque_uniform(n), nb, ng, as_global(aqsn), goff,
                                              as_global(am_col), as_global(wx), ps, A2, B1, B2,
                                              B3);
        // sum_n conj(M) K and sum_n conj(M) L from the band sums
        cplx SK = cmake(0.0, 0.0), SL = cmake(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const cplx h = cload(gh + w);
            const cplx k = cadd(B1[w], cmul(cmake(-ps.a, -ps.b), A2[w]));  // B1 - om A2
            // B1 - 2 (Im om)^2 B2 - 2i (Im om) B3
            const cplx l = cmake(fma(ps.b2, B3[w].im, fma(-ps.wi2x2, B2[w].re, B1[w].re)),
                                 fma(-ps.b2, B3[w].re, fma(-ps.wi2x2, B2[w].im, B1[w].im)));
            cmac(SK, h, k);
            cmac(SL, h, l);
        }
        cmac(Ge, cmake(ps.om.re, -ps.om.im), SK);
        Gw = cadd(Gw, SL);
    }
    // a ragged tail, or every unoccupied band with more frequencies
    pairs_per_band<NW>(n, nb, nb, nv, ng, aqsn, am_col, wx, gh, xgh, gs, ps, goff, Ge, Gw);

    if (valid) {
        const double v = vcoul[g];
        const size_t idx = (size_t)p * ng + g;
        if (grad_ieps) {
            const cplx r = cscale(v, Ge);
            grad_ieps[idx] = make_double2(r.re, r.im);
        }
        if (grad_wt) {
            const cplx r = cscale(v, cmul(cmake(ps.e.re, -ps.e.im), Gw));
            grad_wt[idx] = make_double2(r.re, r.im);
        }
    }
}

// ---- bands kernel: daqsntemp and the daqsmtemp partials -------------------
// LDS of one bands workgroup's daqsmtemp sums: each wave's slab of
// per-lane terms (kBandTile bands x two G' columns) and the waves' row sums
// of up to kAmCols columns.
struct AmStage {
    double2 slab[kBwdWaves][kSlabRows][kWave];
    double2 red[kBwdWaves][kAmRows];
};

// Where a bands workgroup's daqsmtemp sums go: the slab row of band u at
// column p is ((p - p_lo) % 2) kBandTile + u; `chunk` is the first column of
// the rows waiting in red.
struct AmCtx {
    AmStage *st;
    double2 *part;  // am_part: [256-row block][nb][np]
    int wid, lane, gblk, n0, nb, np, p_lo, p_hi, chunk;
};

// This lane's daqsmtemp term of band u at column p: an conj(vcoul conj(e) Z).
__device__ __forceinline__ void am_put(AmCtx &a, int p, int u, cplx an, cplx vz)
{
    const cplx t = cmul_conj(an, vz);
    a.st->slab[a.wid][((p - a.p_lo) & 1) * kBandTile + u][a.lane] = make_double2(t.re, t.im);
}

// After column p: when the slab is full (two columns) or p is the range's
// last column, add each slab row over the wave (lane (tj, tk) adds the
// entries tk, tk + 8, ..., tk + 56 of row tj, then the octet adds its 8
// sums) into red.  An octet thus reads 128 contiguous bytes at a time, and
// the rows start at staggered offsets ((i + tj) mod 8), so that the two
// octets the LDS serves per clock fall in different halves of its banks:
// measured on gfx950 (gpp_mb_lds patterns 2 and 1), such a 16-byte read
// takes 4 LDS cycles with no bank conflict, against 8 cycles (4 of them
// conflict stalls) when each lane reads 8 consecutive entries.  Every
// kAmCols columns, and at the end, add red over the four waves and write
// the partials.  Every wave of the workgroup calls this for the same
// columns.
__device__ __forceinline__ void am_column_done(AmCtx &a, int p)
{
    const int c = (p - a.p_lo) & 1;
    const bool last = p + 1 == a.p_hi;
    if (c == 1 || last) {
        const int rows = (c + 1) * kBandTile;
        const int base = (p - c - a.chunk) * kBandTile;
        wave_lds_sync();
        const int tj = a.lane >> 3, tk = a.lane & (kOctet - 1);
        double sr = 0.0, si = 0.0;
        if (tj < rows) {
#pragma unroll
            for (int i = 0; i < kOctet; ++i) {
                const double2 v = a.st->slab[a.wid][tj][tk + kOctet * ((i + tj) & (kOctet - 1))];
                sr += v.x;
                si += v.y;
            }
        }
        sr = octet_sum(sr);
        si = octet_sum(si);
        if (tk == 0 && tj < rows) a.st->red[a.wid][base + tj] = make_double2(sr, si);
        wave_lds_sync();
    }
    if (p + 1 - a.chunk == kAmCols || last) {
        __syncthreads();
        const int rows = (p + 1 - a.chunk) * kBandTile;
        const int t = threadIdx.x;
        if (t < 2 * rows) {
            const int j = t >> 1, comp = t & 1;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < kBwdWaves; ++k) {
                const double2 v = a.st->red[k][j];
                s += comp ? v.y : v.x;
            }
            const int col = a.chunk + j / kBandTile, n = a.n0 + j % kBandTile;
            if (n < a.nb)
                reinterpret_cast<double *>(a.part + ((size_t)a.gblk * a.nb + n) * a.np + col)[comp] = s;
        }
        __syncthreads();
        a.chunk = p + 1;
    }
}

// Fast form of one workgroup's p loop: every band n0 .. n0+kBandTile-1 is
// unoccupied and below nb.  With u_w = (x_w - om) r_w (r_w the masked
// reciprocal of |x_w - om|^2),
//   K = sum_w gh_w u_w = S - om R,  S = sum_w xgh_w r_w,  R = sum_w gh_w r_w,
// so vcoul conj(e) Z = vcoul conj(e) conj(om) K = c1 S - c2 R with the
// per-pair constants c1 = vcoul conj(e om) and c2 = vcoul conj(e) |om|^2.
template <int NW, bool AM>
__device__ __forceinline__ void bands_fast(int nb, int ng, int n0, int gc, double vc,
                                           gptr<double2> aqsm, gptr<double2> ieps,
                                           gptr<double2> wt, gptr<double> wx,
                                           gptr<double2> gh, gptr<double2> xgh,
                                           const cplx (&an)[kBandTile], AmCtx &amc,
                                           cplx (&acc)[kBandTile])
{
    constexpr int G = bands_group(NW);
    constexpr int Kt = G * NW;
    const int p_lo = amc.p_lo, p_hi = amc.p_hi;
    // om and e of the next column are loaded one iteration ahead, so their
    // latency overlaps this column's arithmetic
    cplx om_next = cload(wt + (size_t)p_lo * ng + gc), e_next = cload(ieps + (size_t)p_lo * ng + gc);
    for (int p = p_lo; p < p_hi; ++p) {
        const int nfirst = opaque_uniform(n0);  // reload x and xgh per p
        const cplx om = om_next, e = e_next;
        const int pn = p + 1 < p_hi ? p + 1 : p;
        om_next = cload(wt + (size_t)pn * ng + gc);
        e_next = cload(ieps + (size_t)pn * ng + gc);
        const double a = om.re, b = om.im;
        const double wi2 = b * b;
        const double wtr = fma(a, a, wi2);
        const double thr = branch_a_threshold(wtr);
        const bool wide = wi2 >= kMinUnclampedWi2;
        const cplx vce = cmake(vc * e.re, -(vc * e.im));  // vcoul conj(e)
        const cplx c1 = cmul(vce, cmake(a, -b));
        const cplx c2 = cscale(wtr, vce);
#pragma unroll
        for (int u0 = 0; u0 < kBandTile; u0 += G) {
            const int n = nfirst + u0;
            double xs[Kt], dc[Kt], r[Kt];
            bool isA[Kt];
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int w = 0; w < NW; ++w) xs[u * NW + w] = wx[(size_t)w * nb + n + u];
#pragma unroll
            for (int k = 0; k < Kt; ++k) {
                const double dr = xs[k] - a;
                const double wd = fma(dr, dr, wi2);
                isA[k] = wd > thr;
                dc[k] = wd;  // unclamped: see batch_reciprocal
            }
            batch_reciprocal<Kt>(dc, r, wide);
#pragma unroll
            for (int u = 0; u < G; ++u) {
#if GPP_EXEC_MASK == 2
                // the first frequency starts S and R through a select, the
                // others add under an execution mask written by the compare
                const double r0 = mask_keep(isA[u * NW], r[u * NW]);
                const cplx xg0 = cload(xgh + n + u);
                const cplx g0 = cload(gh);
                cplx S = cmake(r0 * xg0.re, r0 * xg0.im), R = cmake(r0 * g0.re, r0 * g0.im);
#pragma unroll
                for (int w = 1; w < NW; ++w) {
                    const int k = u * NW + w;
                    const cplx xg = cload(xgh + (size_t)w * nb + n + u);
                    const cplx g = cload(gh + w);
                    unsigned long long saved;
                    asm("s_mov_b64 %[sv], exec\n\t"
                        "v_cmpx_gt_f64_e32 vcc, %[d], %[thr]\n\t"
                        "v_fma_f64 %[sr], %[r], %[xr], %[sr]\n\t"
                        "v_fma_f64 %[si], %[r], %[xi], %[si]\n\t"
                        "v_fma_f64 %[rr], %[r], %[gr], %[rr]\n\t"
                        "v_fma_f64 %[ri], %[r], %[gi], %[ri]\n\t"
                        "s_mov_b64 exec, %[sv]"
                        : [sv] "=&s"(saved), [sr] "+v"(S.re), [si] "+v"(S.im), [rr] "+v"(R.re),
                          [ri] "+v"(R.im)
                        : [d] "v"(dc[k]), [thr] "v"(thr), [r] "v"(r[k]), [xr] "s"(xg.re),
                          [xi] "s"(xg.im), [gr] "s"(g.re), [gi] "s"(g.im)
                        : "vcc");
                }
#else
                cplx S = cmake(0.0, 0.0), R = cmake(0.0, 0.0);
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const int k = u * NW + w;
                    const double re = mask_keep(isA[k], r[k]);
                    const cplx xg = cload(xgh + (size_t)w * nb + n + u);
                    const cplx g = cload(gh + w);
                    S.re = fma(re, xg.re, S.re);
                    S.im = fma(re, xg.im, S.im);
                    R.re = fma(re, g.re, R.re);
                    R.im = fma(re, g.im, R.im);
                }
#endif
                const cplx vZ = cmake(c1.re * S.re - c1.im * S.im - c2.re * R.re + c2.im * R.im,
                                      c1.re * S.im + c1.im * S.re - c2.re * R.im - c2.im * R.re);
                const cplx am = cload(aqsm + (size_t)(n + u) * ng + p);
                cmac(acc[u0 + u], am, vZ);
                if constexpr (AM) am_put(amc, p, u0 + u, an[u0 + u], vZ);
            }
            // one group's reciprocal chain at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (AM) am_column_done(amc, p);
    }
}

// Generic form: occupied bands (exchange terms) and a ragged last tile.
template <int NW, bool AM>
__device__ __forceinline__ void bands_generic(int nb, int nv, int ng, int n0, int gc, bool valid,
                                              const double2 *__restrict__ aqsm,
                                              const double2 *__restrict__ ieps,
                                              const double2 *__restrict__ wt,
                                              const double *__restrict__ vcoul,
                                              const double *__restrict__ wx,
                                              const double2 *__restrict__ gh,
                                              const double2 *__restrict__ gs,
                                              const cplx (&an)[kBandTile], AmCtx &amc,
                                              cplx (&acc)[kBandTile])
{
    constexpr int G = bands_group(NW);
    for (int p = amc.p_lo; p < amc.p_hi; ++p) {
        const PairState ps = load_pair(wt, ieps, vcoul, p, ng, gc, valid);
        const cplx vce = cmake(ps.ve.re, -ps.ve.im);           // vcoul conj(e)
        const cplx vcw = cmul(vce, cmake(ps.om.re, -ps.om.im));  // vcoul conj(e om)
#pragma unroll
        for (int u0 = 0; u0 < kBandTile; u0 += G) {
            const int n = n0 + u0;
            cplx K[G], L[G];
            const bool full = n + G <= nb && n >= nv;
            if (full) {
                ch_bands_kl<NW, G, false>(n, nb, wx, gh, nullptr, ps.a, ps.b, ps.wi2, ps.thr,
                                          ps.wide, K, L);
            } else {
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    K[u] = cmake(0.0, 0.0);
                    if (n + u < nb) {
                        cplx K1[1], L1[1];
                        ch_bands_kl<NW, 1, false>(n + u, nb, wx, gh, nullptr, ps.a, ps.b,
                                                  ps.wi2, ps.thr, ps.wide, K1, L1);
                        K[u] = K1[0];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int nn = n + u;
                cplx vZ = cmake(0.0, 0.0);
                if (nn < nb) {
                    // vcoul conj(e) Z = vcoul conj(e om) K [+ vcoul conj(e) KS]
                    vZ = cmul(vcw, K[u]);
                    if (nn < nv) {
                        cplx KS, LS;
                        sx_band_kl<NW>(nn, nb, wx, gs, ps.a, ps.b, ps.wi2, ps.wtr, ps.thr, KS, LS);
                        cmac(vZ, vce, KS);
                    }
                    const cplx am = cload(aqsm + (size_t)nn * ng + p);
                    cmac(acc[u0 + u], am, vZ);
                }
                if constexpr (AM) am_put(amc, p, u0 + u, an[u0 + u], vZ);
            }
        }
        if constexpr (AM) am_column_done(amc, p);
    }
}

// Workgroup = kBandTile bands x 256 rows (one 64-row tile per wave) x one
// segment of the G' range; band tile fastest (neighbouring workgroups
// share the rows of wtilde/I_eps), then row block, then segment.  One
// segment writes daqsntemp itself, several write partial sums (grad_an may
// be NULL: daqsmtemp only).  With AM, also the daqsmtemp partials of the
// workgroup's bands, rows and columns.
template <int NW, bool AM>
__global__ void __launch_bounds__(kBwdThreads)
__attribute__((amdgpu_waves_per_eu(AM ? GPP_BWD_BANDS_AM_WAVES : GPP_BWD_BANDS_WAVES)))
bwd_bands(int nb, int nv, int ng, int np, long nwg, int nbt, int ngb, int nps,
          const double2 *__restrict__ aqsm, const double2 *__restrict__ aqsn,
          const double2 *__restrict__ ieps, const double2 *__restrict__ wt,
          const double *__restrict__ vcoul, const double *__restrict__ wx,
          const double2 *__restrict__ gh, const double2 *__restrict__ xgh,
          const double2 *__restrict__ gs, double2 *__restrict__ grad_an,
          double2 *__restrict__ am_part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const long wg = xcd_remap(blockIdx.x, gridDim.x);
    if (wg >= nwg) return;  // the whole workgroup leaves together
    const long per_seg = (long)ngb * nbt;
    const int seg = (int)(wg / per_seg);
    const long in_seg = wg - (long)seg * per_seg;
    const int gblk = (int)(in_seg / nbt);
    const int n0 = (int)(in_seg - (long)gblk * nbt) * kBandTile;
    double2 *const dst = grad_an ? grad_an + (size_t)seg * nb * ng : nullptr;
    const int g = gblk * kRowsPerBlock + wid * kWave + lane;
    const bool valid = g < ng;
    const int gc = valid ? g : ng - 1;

    AmCtx amc;
    amc.st = nullptr;
    if constexpr (AM) {
        __shared__ AmStage stage;
        amc.st = &stage;
    }
    amc.part = am_part;
    amc.wid = wid;
    amc.lane = lane;
    amc.gblk = gblk;
    amc.n0 = n0;
    amc.nb = nb;
    amc.np = np;
    amc.p_lo = (int)((long)np * seg / nps);
    amc.p_hi = (int)((long)np * (seg + 1) / nps);
    amc.chunk = amc.p_lo;

    cplx an[kBandTile];
#pragma unroll
    for (int u = 0; u < kBandTile; ++u) {
        an[u] = cmake(0.0, 0.0);
        if (AM && n0 + u < nb) an[u] = cload(aqsn + (size_t)(n0 + u) * ng + gc);
    }
    cplx acc[kBandTile];
#pragma unroll
    for (int u = 0; u < kBandTile; ++u) acc[u] = cmake(0.0, 0.0);
    if (n0 >= nv && n0 + kBandTile <= nb)
        bands_fast<NW, AM>(nb, ng, n0, gc, valid ? vcoul[gc] : 0.0, as_global(aqsm),
                           as_global(ieps), as_global(wt), as_global(wx), as_global(gh),
                           as_global(xgh), an, amc, acc);
    else
        bands_generic<NW, AM>(nb, nv, ng, n0, gc, valid, aqsm, ieps, wt, vcoul, wx, gh, gs, an,
                              amc, acc);
    if (dst && valid) {
#pragma unroll
        for (int u = 0; u < kBandTile; ++u) {
            const int n = n0 + u;
            if (n < nb) dst[(size_t)n * ng + g] = make_double2(acc[u].re, acc[u].im);
        }
    }
}

// daqsmtemp[n][p] = sum over row blocks of the partials (p < np), 0 for
// columns np..ncouls-1.  One thread per output element, fixed order.  The
// nb * np sums come first in the grid and the zero columns after them, so
// that the workgroups which read run together instead of one in twenty
// across the whole grid.
__global__ void reduce_am(int nb, int ng, int np, int ngb, const double2 *__restrict__ part,
                          double2 *__restrict__ grad_am)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nsum = (long)nb * np;
    if (i < nsum) {
        const int n = (int)(i / np), col = (int)(i - (long)n * np);
        double re = 0.0, im = 0.0;
        // unrolled so that eight loads are in flight; the additions keep
        // their order
#pragma unroll 8
        for (int b = 0; b < ngb; ++b) {
            const double2 v = part[((size_t)b * nb + n) * np + col];
            re += v.x;
            im += v.y;
        }
        grad_am[(size_t)n * ng + col] = make_double2(re, im);
        return;
    }
    const long j = i - nsum, nz = ng - np;
    if (nz <= 0 || j >= (long)nb * nz) return;
    const int n = (int)(j / nz);
    grad_am[(size_t)n * ng + np + (j - (long)n * nz)] = make_double2(0.0, 0.0);
}

// daqsntemp = sum of the nps segment partials, in segment order.
__global__ void reduce_an(long nbg, int nps, const double2 *__restrict__ part,
                          double2 *__restrict__ grad_an)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbg) return;
    double re = 0.0, im = 0.0;
#pragma unroll 4
    for (int s = 0; s < nps; ++s) {
        const double2 v = part[(size_t)s * nbg + i];
        re += v.x;
        im += v.y;
    }
    grad_an[i] = make_double2(re, im);
}

__global__ void fill_zero_n(double2 *a, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = make_double2(0.0, 0.0);
}

BwdGeometry bwd_geometry(const Dims32 &d)
{
    BwdGeometry geo{};
    geo.gh_elems = d.nw;
    geo.xgh_elems = (size_t)d.nw * d.nb;
    if (d.nb > 0 && d.ng > 0 && d.np > 0) {
        geo.ngb = (d.ng + kRowsPerBlock - 1) / kRowsPerBlock;
        geo.pair_blocks = (long)geo.ngb * d.np;
        geo.nbt = (d.nb + kBandTile - 1) / kBandTile;
        geo.ngt = geo.ngb * kBwdWaves;
        // Split the p loop into segments when one pass has too few waves:
        // every wave walks its whole p range, so the last partial round of
        // a short grid leaves most SIMDs idle.  Aim at kBandsRounds rounds
        // of the MI355X's resident bands waves, each segment at least
        // kMinSegCols columns long.
        const long per_seg = (long)geo.ngt * geo.nbt;
        const long want = (long)kBandsRounds * kBandsWaveSlots;
        long nps = (want + per_seg - 1) / per_seg;
        const long max_nps = d.np / kMinSegCols > 1 ? d.np / kMinSegCols : 1;
        geo.nps = (int)(nps < max_nps ? nps : max_nps);
        geo.band_tiles = per_seg * geo.nps;
        geo.band_blocks = (long)geo.ngb * geo.nbt * geo.nps;
        geo.am_part_elems = (size_t)geo.ngb * d.nb * d.np;
        geo.an_part_elems = geo.nps > 1 ? (size_t)geo.nps * d.nb * d.ng : 0;
    }
    // complex elements, each 16 bytes; sections 256-byte aligned
    auto up = [](size_t e) { return (e * sizeof(double2) + 255) / 256 * 256; };
    geo.workspace_bytes = up(geo.gh_elems) + up(geo.xgh_elems) + up(geo.am_part_elems) +
                          up(geo.an_part_elems);
    if (geo.workspace_bytes == 0) geo.workspace_bytes = 256;
    return geo;
}

template <int NW>
static hipError_t launch_bwd_nw(const Dims32 &d, const BwdGeometry &geo, const DevInputs &in,
                                const double2 *ga, const double2 *gs, const BwdOutputs &out,
                                char *ws, hipStream_t st)
{
    auto up = [](size_t e) { return (e * sizeof(double2) + 255) / 256 * 256; };
    double2 *gh = reinterpret_cast<double2 *>(ws);
    double2 *xgh = reinterpret_cast<double2 *>(ws + up(geo.gh_elems));
    double2 *am_part = reinterpret_cast<double2 *>(ws + up(geo.gh_elems) + up(geo.xgh_elems));
    double2 *an_part = reinterpret_cast<double2 *>(ws + up(geo.gh_elems) + up(geo.xgh_elems) +
                                                   up(geo.am_part_elems));
    const long prep = (long)d.nw * d.nb > d.nw ? (long)d.nw * d.nb : d.nw;
    hipLaunchKernelGGL(bwd_prepare, dim3((unsigned)((prep + 255) / 256)), dim3(256), 0, st,
                       d.nb, d.nw, in.wx, ga, gh, xgh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (out.grad_wt || out.grad_ieps) {
        hipLaunchKernelGGL(bwd_pairs<NW>, dim3((unsigned)geo.pair_blocks), dim3(kBwdThreads), 0,
                           st, d.nb, d.nv, d.ng, d.np, geo.pair_blocks, in.aqsm, in.aqsn,
                           in.ieps, in.wt, in.vcoul, in.wx, gh, xgh, gs, out.grad_wt,
                           out.grad_ieps);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (out.grad_an || out.grad_am) {
        double2 *an_dst = !out.grad_an ? nullptr : (geo.nps > 1 ? an_part : out.grad_an);
        if (out.grad_am)
            hipLaunchKernelGGL((bwd_bands<NW, true>), dim3((unsigned)geo.band_blocks),
                               dim3(kBwdThreads), 0, st, d.nb, d.nv, d.ng, d.np, geo.band_blocks,
                               geo.nbt, geo.ngb, geo.nps, in.aqsm, in.aqsn, in.ieps, in.wt,
                               in.vcoul, in.wx, gh, xgh, gs, an_dst, am_part);
        else
            hipLaunchKernelGGL((bwd_bands<NW, false>), dim3((unsigned)geo.band_blocks),
                               dim3(kBwdThreads), 0, st, d.nb, d.nv, d.ng, d.np, geo.band_blocks,
                               geo.nbt, geo.ngb, geo.nps, in.aqsm, in.aqsn, in.ieps, in.wt,
                               in.vcoul, in.wx, gh, xgh, gs, an_dst, nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (out.grad_an && geo.nps > 1) {
            const long nbg = (long)d.nb * d.ng;
            hipLaunchKernelGGL(reduce_an, dim3((unsigned)((nbg + 255) / 256)), dim3(256), 0, st,
                               nbg, geo.nps, an_part, out.grad_an);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (out.grad_am) {
        const long n = (long)d.nb * d.ng;
        hipLaunchKernelGGL(reduce_am, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d.nb,
                           d.ng, d.np, geo.ngb, am_part, out.grad_am);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_bwd(const Dims32 &d, const DevInputs &in, const double2 *ga,
                      const double2 *gs, const BwdOutputs &out, void *workspace, hipStream_t st)
{
    const BwdGeometry geo = bwd_geometry(d);
    if (geo.pair_blocks == 0) {
        // an empty sum: every requested gradient is zero
        const long npg = (long)d.np * d.ng, nbg = (long)d.nb * d.ng;
        double2 *outs[4] = {out.grad_wt, out.grad_ieps, out.grad_an, out.grad_am};
        const long lens[4] = {npg, npg, nbg, nbg};
        for (int k = 0; k < 4; ++k) {
            if (!outs[k] || lens[k] == 0) continue;
            hipLaunchKernelGGL(fill_zero_n, dim3((unsigned)((lens[k] + 255) / 256)), dim3(256), 0,
                               st, outs[k], lens[k]);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    char *ws = static_cast<char *>(workspace);
    switch (d.nw) {
    case 1: return launch_bwd_nw<1>(d, geo, in, ga, gs, out, ws, st);
    case 2: return launch_bwd_nw<2>(d, geo, in, ga, gs, out, ws, st);
    case 3: return launch_bwd_nw<3>(d, geo, in, ga, gs, out, ws, st);
    case 4: return launch_bwd_nw<4>(d, geo, in, ga, gs, out, ws, st);
    case 5: return launch_bwd_nw<5>(d, geo, in, ga, gs, out, ws, st);
    case 6: return launch_bwd_nw<6>(d, geo, in, ga, gs, out, ws, st);
    case 7: return launch_bwd_nw<7>(d, geo, in, ga, gs, out, ws, st);
    case 8: return launch_bwd_nw<8>(d, geo, in, ga, gs, out, ws, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gpp
