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
// Kernels: bwd_pairs (lane = g, wave-uniform p, bands serial) writes
// dwtilde and dI_eps and, per workgroup of 256 rows, partial sums of
// daqsmtemp.  Slabs of unoccupied bands form K and L from four factored
// sums per band (see the slab loop); occupied bands and ragged slabs form
// u and u^2 per term.  The per-lane daqsmtemp terms of kSlab bands are parked in a
// per-wave LDS slab and summed together (8 lanes per band, then a DPP sum
// over the 8), instead of one 64-lane shuffle reduction per band.
// bwd_bands (lane = g, a wave owns kBandTile bands and walks every p)
// writes daqsntemp; reduce_am sums the daqsmtemp partials in a fixed order
// and zero-fills columns >= ngpown.  No atomics: results are bitwise
// reproducible.
#include "gpp_device.h"
#include "gpp_internal.h"

namespace gpp {

constexpr int kBwdWaves = 4;
constexpr int kBwdThreads = kBwdWaves * kWave;
constexpr int kRowsPerBlock = kBwdWaves * kWave;  // g rows per pairs workgroup
// Bands per batch-inverted group: 3, or 1 with more than four frequencies,
// so that a group never holds more than 12 denominators (the range for
// which batch_reciprocal's (Im om)^2 >= 2^-60 lane test keeps every prefix
// product normal).
constexpr int bwd_group(int nw) { return nw <= 4 ? 3 : 1; }
constexpr int kChunk = 48;                         // bands per LDS flush (multiple of kSlab)
constexpr int kSlab = 6;                           // bands per in-wave transpose (two groups)
constexpr int kOctet = 8;                          // lanes that share one band's row sum
// Minimum waves per SIMD the compiler must allow (register cap) for the
// pairs and bands kernels; 1 leaves the allocation to the compiler.  Pairs:
// 3 waves (up to 168 VGPRs; the factored slab loop needs about 160, and a
// 4-wave cap spills it, 5-6 % slower on the nb256/ng16384/np819 adjoint
// workload).  Bands: 5 waves = 96 VGPRs, about 1.3 % faster there than the
// compiler's own choice.
#ifndef GPP_BWD_PAIRS_WAVES
#define GPP_BWD_PAIRS_WAVES 3
#endif
#ifndef GPP_BWD_BANDS_WAVES
#define GPP_BWD_BANDS_WAVES 5
#endif
#ifndef GPP_BWD_BAND_TILE
#define GPP_BWD_BAND_TILE 3
#endif
constexpr int kBandTile = GPP_BWD_BAND_TILE;       // bands per bands-kernel wave
// Bands-kernel p-range split (see bwd_geometry): resident bands waves of the
// MI355X (256 CUs x 4 SIMDs x GPP_BWD_BANDS_WAVES), rounds of them to aim
// at, and the shortest segment.
#ifndef GPP_BWD_BANDS_ROUNDS
#define GPP_BWD_BANDS_ROUNDS 16
#endif
constexpr long kBandsWaveSlots = 256L * 4 * GPP_BWD_BANDS_WAVES;
constexpr int kBandsRounds = GPP_BWD_BANDS_ROUNDS;
constexpr int kMinSegCols = 64;
static_assert(kBandTile % bwd_group(1) == 0 && kBandTile % bwd_group(8) == 0,
              "band tile must be whole groups");

// Upstream gradient scaled for the kernels: gh[w] = ga[w]/2 and
// xgh[w][n] = wx[w][n] ga[w]/2, written once by bwd_prepare.
__global__ void bwd_prepare(int nb, int nw, const double *__restrict__ wx,
                            const double2 *__restrict__ ga, double2 *__restrict__ gh,
                            double2 *__restrict__ xgh)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) gh[i] = make_double2(0.5 * ga[i].x, 0.5 * ga[i].y);
    if (i < nw * nb) {
        const int w = i / nb;
        const double x = wx[i];
        xgh[i] = make_double2(0.5 * x * ga[w].x, 0.5 * x * ga[w].y);
    }
}

// Lane exchange inside a row of 16 lanes (DPP), both halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
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

// Exchange term of an occupied band: ssx = e sigma, d ssx/d om = e delta.
__device__ inline void sx_sigma_delta(double x, double a, double b, double wi2, double wtr,
                                      double thr, cplx &sigma, cplx &delta)
{
    const cplx om = cmake(a, b);
    const double dr = x - a;
    const double wd = fma(dr, dr, wi2);
    const cplx d = cmake(dr, -b);    // x - om
    const cplx s = cmake(x + a, b);  // x + om
    if (wd > thr) {                  // A: sigma = om^2/(d s), delta = 2 om x^2/(d s)^2
        const cplx ds = cmul(d, s);
        sigma = cdiv(cmul(om, om), ds);
        delta = cdiv(cscale(2.0 * x * x, om), cmul(ds, ds));
    } else if (branch_b_holds(wtr, wd)) {  // B: sigma = -om/(2s), delta = -x/(2 s^2)
        const cplx s2 = cscale(-2.0, s);
        sigma = cdiv(om, s2);
        delta = cdiv(cmake(x, 0.0), cmul(s2, s));
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

// Batch-inverted reciprocals of the BU*NW terms of BU bands starting at
// band n for one lane, dr = x - Re om and the denominators dc.  With MASK
// the reciprocals of terms off branch A are cleared (mask_keep); without
// it the caller applies the branch itself (dc against the threshold).
template <int NW, int BU, bool MASK = true>
__device__ __forceinline__ void group_reciprocals(int n, int nb, const double *__restrict__ wx,
                                                  double a, double wi2, double thr, bool wide,
                                                  double (&r)[BU * NW], double (&drs)[BU * NW],
                                                  double (&dc)[BU * NW])
{
    constexpr int Kt = BU * NW;
    bool isA[Kt];
#pragma unroll
    for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int w = 0; w < NW; ++w) drs[u * NW + w] = wx[(size_t)w * nb + n + u] - a;
#pragma unroll
    for (int k = 0; k < Kt; ++k) {
        const double wd = fma(drs[k], drs[k], wi2);
        isA[k] = wd > thr;
        dc[k] = wd;  // unclamped: see batch_reciprocal
    }
    batch_reciprocal<Kt>(dc, r, wide);
    if (MASK) {
#pragma unroll
        for (int k = 0; k < Kt; ++k) r[k] = mask_keep(isA[k], r[k]);
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

// ---- pairs kernel: dwtilde, dI_eps and daqsmtemp partials -----------------
template <int NW>
__global__ void __launch_bounds__(kBwdThreads)
__attribute__((amdgpu_waves_per_eu(GPP_BWD_PAIRS_WAVES)))
bwd_pairs(int nb, int nv, int ng, int np, long nblocks, const double2 *__restrict__ aqsm,
          const double2 *__restrict__ aqsn, const double2 *__restrict__ ieps,
          const double2 *__restrict__ wt, const double *__restrict__ vcoul,
          const double *__restrict__ wx, const double2 *__restrict__ gh,
          const double2 *__restrict__ xgh, const double2 *__restrict__ gs,
          double2 *__restrict__ grad_wt, double2 *__restrict__ grad_ieps,
          double2 *__restrict__ am_part)
{
    // Per-wave transpose slab for the daqsmtemp terms of up to kSlab bands
    // (8 rows so that every lane's read below stays inside its wave's slab),
    // and per-wave band sums awaiting the workgroup flush.
    __shared__ double2 slab[kBwdWaves][kOctet][kWave];
    __shared__ double2 red[kBwdWaves][kChunk];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const long blk = xcd_remap(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;  // whole workgroup leaves together
    // p fastest: concurrently resident workgroups share one 256-row block
    const int gb = (int)(blk / np);
    const int p = (int)(blk - (long)gb * np);
    const int g = gb * kRowsPerBlock + wid * kWave + lane;
    const bool valid = g < ng;
    const int gc = valid ? g : ng - 1;
    const PairState ps = load_pair(wt, ieps, vcoul, p, ng, gc, valid);
    const cplx cw = cmake(ps.om.re, -ps.om.im);  // conj(om)
    const double2 *am_col = aqsm + p;
    const uint32_t goff = (uint32_t)gc * (uint32_t)sizeof(double2);
    // transpose roles: lane = (band j of the slab, segment k of 8 lanes)
    const int tj = lane >> 3, tk = lane & (kOctet - 1);

    cplx Ge = cmake(0.0, 0.0), Gw = cmake(0.0, 0.0);
    for (int c0 = 0; c0 < nb; c0 += kChunk) {
        const int c1 = c0 + kChunk < nb ? c0 + kChunk : nb;
        for (int b0 = c0; b0 < c1; b0 += kSlab) {
            const int b1 = b0 + kSlab < c1 ? b0 + kSlab : c1;
            int n = b0;
            if (b0 >= nv && b1 - b0 == kSlab) {
                // A whole slab of unoccupied bands: no exchange terms, whole
                // groups, and K, L from factored sums.  With r_w the masked
                // reciprocal of |x_w - om|^2 and dr_w = x_w - Re om, every
                // branch-A term has |x_w - om|^2 r_w = 1, so
                //   u_w^2 = r_w - 2 (Im om)^2 r_w^2 - 2i (Im om) dr_w r_w^2,
                //   K = S - om R,  L = S - 2 (Im om)^2 T - 2i (Im om) U,
                //   S = sum_w xgh_w r_w,  R = sum_w gh_w r_w,
                //   T = sum_w xgh_w r_w^2,  U = sum_w xgh_w dr_w r_w^2:
                // four complex-by-real multiply-adds per term.
#pragma unroll 1
                for (int q0 = 0; q0 < kSlab; q0 += bwd_group(NW)) {
                    constexpr int Kt = bwd_group(NW) * NW;
                    double r[Kt], drs[Kt], dcs[Kt];
                    const int ng0 = opaque_uniform(__builtin_amdgcn_readfirstlane(b0 + q0));
                    group_reciprocals<NW, bwd_group(NW), GPP_EXEC_MASK != 2>(
                        ng0, nb, wx, ps.a, ps.wi2, ps.thr, ps.wide, r, drs, dcs);
#pragma unroll
                    for (int u = 0; u < bwd_group(NW); ++u) {
                        const int nn = ng0 + u;
                        cplx S = cmake(0.0, 0.0), R = S, T = S, U = S;
#pragma unroll
                        for (int w = 0; w < NW; ++w) {
                            const int k = u * NW + w;
                            const cplx g = cload(gh + w);
                            const cplx xg = cload(xgh + (size_t)w * nb + nn);
#if GPP_EXEC_MASK == 2
                            if (w > 0) {
                                // later frequencies add under an execution
                                // mask written by the branch-A compare
                                unsigned long long saved;
                                double q, dq;
                                asm("s_mov_b64 %[sv], exec\n\t"
                                    "v_cmpx_gt_f64_e32 vcc, %[d], %[thr]\n\t"
                                    "v_mul_f64 %[q], %[r], %[r]\n\t"
                                    "v_fma_f64 %[sr], %[r], %[xr], %[sr]\n\t"
                                    "v_fma_f64 %[si], %[r], %[xi], %[si]\n\t"
                                    "v_fma_f64 %[rr], %[r], %[gr], %[rr]\n\t"
                                    "v_fma_f64 %[ri], %[r], %[gi], %[ri]\n\t"
                                    "v_mul_f64 %[dq], %[dr], %[q]\n\t"
                                    "v_fma_f64 %[tr], %[q], %[xr], %[tr]\n\t"
                                    "v_fma_f64 %[ti], %[q], %[xi], %[ti]\n\t"
                                    "v_fma_f64 %[ur], %[dq], %[xr], %[ur]\n\t"
                                    "v_fma_f64 %[ui], %[dq], %[xi], %[ui]\n\t"
                                    "s_mov_b64 exec, %[sv]"
                                    : [sv] "=&s"(saved), [q] "=&v"(q), [dq] "=&v"(dq),
                                      [sr] "+v"(S.re), [si] "+v"(S.im), [rr] "+v"(R.re),
                                      [ri] "+v"(R.im), [tr] "+v"(T.re), [ti] "+v"(T.im),
                                      [ur] "+v"(U.re), [ui] "+v"(U.im)
                                    : [d] "v"(dcs[k]), [thr] "v"(ps.thr), [r] "v"(r[k]),
                                      [dr] "v"(drs[k]), [xr] "s"(xg.re), [xi] "s"(xg.im),
                                      [gr] "s"(g.re), [gi] "s"(g.im)
                                    : "vcc");
                                continue;
                            }
                            // the first frequency starts the sums through a select
                            r[k] = mask_keep(dcs[k] > ps.thr, r[k]);
#endif
                            const double q = r[k] * r[k];
                            const double dq = drs[k] * q;
                            S.re = fma(r[k], xg.re, S.re);
                            S.im = fma(r[k], xg.im, S.im);
                            R.re = fma(r[k], g.re, R.re);
                            R.im = fma(r[k], g.im, R.im);
                            T.re = fma(q, xg.re, T.re);
                            T.im = fma(q, xg.im, T.im);
                            U.re = fma(dq, xg.re, U.re);
                            U.im = fma(dq, xg.im, U.im);
                        }
                        // Z = conj(om) (S - om R),  W = L
                        const cplx Z = cmake(fma(ps.a, S.re, fma(ps.b, S.im, -ps.wtr * R.re)),
                                             fma(ps.a, S.im, fma(-ps.b, S.re, -ps.wtr * R.im)));
                        const cplx W = cmake(fma(ps.b2, U.im, fma(-ps.wi2x2, T.re, S.re)),
                                             fma(-ps.b2, U.re, fma(-ps.wi2x2, T.im, S.im)));
                        const cplx an = load_row_elem(as_global(aqsn) + (size_t)nn * ng, ng, goff);
                        const cplx am = cload(am_col + (size_t)nn * ng);
                        const cplx cM = cmul_conj(am, an);  // conj(M) = conj(an) am
                        cmac(Ge, cM, Z);
                        cmac(Gw, cM, W);
                        if (am_part) {
                            const cplx t = cmul(ps.ve, cmul_conj(an, Z));
                            slab[wid][nn - b0][lane] = make_double2(t.re, t.im);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                n = b1;
            }
            while (n < b1) {
                // bands n .. n+cnt-1 form one batch-inverted group
                const bool occ = n < nv;
                const int cnt = (!occ && n + bwd_group(NW) <= b1) ? bwd_group(NW) : 1;
                cplx K[bwd_group(NW)], L[bwd_group(NW)];
                if (cnt == bwd_group(NW)) {
                    ch_bands_kl<NW, bwd_group(NW), true>(n, nb, wx, gh, xgh, ps.a, ps.b, ps.wi2,
                                                     ps.thr, ps.wide, K, L);
                } else {
                    cplx K1[1], L1[1];
                    ch_bands_kl<NW, 1, true>(n, nb, wx, gh, xgh, ps.a, ps.b, ps.wi2, ps.thr,
                                             ps.wide, K1, L1);
                    K[0] = K1[0];
                    L[0] = L1[0];
                }
#pragma unroll
                for (int u = 0; u < bwd_group(NW); ++u) {
                    if (u >= cnt) break;  // wave-uniform
                    const int nn = n + u;
                    cplx Z = cmul(cw, K[u]);
                    cplx W = L[u];
                    if (nn < nv) {
                        cplx KS, LS;
                        sx_band_kl<NW>(nn, nb, wx, gs, ps.a, ps.b, ps.wi2, ps.wtr, ps.thr, KS,
                                       LS);
                        Z = cadd(Z, KS);
                        W = cadd(W, LS);
                    }
                    const cplx an = load_row_elem(as_global(aqsn) + (size_t)nn * ng, ng, goff);
                    const cplx am = cload(am_col + (size_t)nn * ng);
                    const cplx cM = cmul_conj(am, an);  // conj(M) = conj(an) am
                    cmac(Ge, cM, Z);
                    cmac(Gw, cM, W);
                    if (am_part) {
                        // this lane's term of daqsmtemp[nn][p]: ve an conj(Z)
                        const cplx t = cmul(ps.ve, cmul_conj(an, Z));
                        slab[wid][nn - b0][lane] = make_double2(t.re, t.im);
                    }
                }
                n += cnt;
            }
            if (am_part) {
                // Row sums of the slab: lane (tj, tk) adds 8 entries of row tj
                // (rotated so the 8 lanes of an octet hit distinct banks), then
                // the octet adds its 8 partial sums.
                wave_lds_sync();
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int i = 0; i < kOctet; ++i) {
                    const double2 v = slab[wid][tj][kOctet * tk + ((i + tk + tj) & (kOctet - 1))];
                    sr += v.x;
                    si += v.y;
                }
                sr = octet_sum(sr);
                si = octet_sum(si);
                if (tk == 0 && tj < b1 - b0) red[wid][b0 - c0 + tj] = make_double2(sr, si);
                wave_lds_sync();
            }
        }
        if (am_part) {
            __syncthreads();
            const int t = threadIdx.x;
            if (t < 2 * (c1 - c0)) {
                const int j = t >> 1, c = t & 1;
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < kBwdWaves; ++k) {
                    const double2 v = red[k][j];
                    s += c ? v.y : v.x;
                }
                double *dst = reinterpret_cast<double *>(
                    am_part + ((size_t)gb * nb + c0 + j) * np + p);
                dst[c] = s;
            }
            __syncthreads();
        }
    }
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

// ---- bands kernel: daqsntemp --------------------------------------------
// Fast form of one wave's p loop: every band n0 .. n0+kBandTile-1 is
// unoccupied and below nb.  With u_w = (x_w - om) r_w (r_w the masked
// reciprocal of |x_w - om|^2),
//   K = sum_w gh_w u_w = S - om R,  S = sum_w xgh_w r_w,  R = sum_w gh_w r_w,
// so vcoul conj(e) Z = vcoul conj(e) conj(om) K = c1 S - c2 R with the
// per-pair constants c1 = vcoul conj(e om) and c2 = vcoul conj(e) |om|^2.
template <int NW>
__device__ __forceinline__ void bands_fast(int nb, int ng, int p_lo, int p_hi, int n0, int gc,
                                           double vc,
                                           gptr<double2> aqsm, gptr<double2> ieps,
                                           gptr<double2> wt, gptr<double> wx,
                                           gptr<double2> gh, gptr<double2> xgh,
                                           cplx (&acc)[kBandTile])
{
    constexpr int Kt = bwd_group(NW) * NW;
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
        for (int u0 = 0; u0 < kBandTile; u0 += bwd_group(NW)) {
            const int n = nfirst + u0;
            double xs[Kt], dc[Kt], r[Kt];
            bool isA[Kt];
#pragma unroll
            for (int u = 0; u < bwd_group(NW); ++u)
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
            for (int u = 0; u < bwd_group(NW); ++u) {
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
            }
            // one group's reciprocal chain at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Generic form: occupied bands (exchange terms) and a ragged last tile.
template <int NW>
__device__ __forceinline__ void bands_generic(int nb, int nv, int ng, int p_lo, int p_hi, int n0,
                                              int gc,
                                              bool valid, const double2 *__restrict__ aqsm,
                                              const double2 *__restrict__ ieps,
                                              const double2 *__restrict__ wt,
                                              const double *__restrict__ vcoul,
                                              const double *__restrict__ wx,
                                              const double2 *__restrict__ gh,
                                              const double2 *__restrict__ gs,
                                              cplx (&acc)[kBandTile])
{
    for (int p = p_lo; p < p_hi; ++p) {
        const PairState ps = load_pair(wt, ieps, vcoul, p, ng, gc, valid);
        const cplx vce = cmake(ps.ve.re, -ps.ve.im);           // vcoul conj(e)
        const cplx vcw = cmul(vce, cmake(ps.om.re, -ps.om.im));  // vcoul conj(e om)
#pragma unroll
        for (int u0 = 0; u0 < kBandTile; u0 += bwd_group(NW)) {
            const int n = n0 + u0;
            if (n >= nb) break;  // wave-uniform
            cplx K[bwd_group(NW)], L[bwd_group(NW)];
            const bool full = n + bwd_group(NW) <= nb && n >= nv;
            if (full) {
                ch_bands_kl<NW, bwd_group(NW), false>(n, nb, wx, gh, nullptr, ps.a, ps.b, ps.wi2,
                                                  ps.thr, ps.wide, K, L);
            } else {
#pragma unroll
                for (int u = 0; u < bwd_group(NW); ++u) {
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
            for (int u = 0; u < bwd_group(NW); ++u) {
                const int nn = n + u;
                if (nn < nb) {
                    // vcoul conj(e) Z = vcoul conj(e om) K [+ vcoul conj(e) KS]
                    cplx vZ = cmul(vcw, K[u]);
                    if (nn < nv) {
                        cplx KS, LS;
                        sx_band_kl<NW>(nn, nb, wx, gs, ps.a, ps.b, ps.wi2, ps.wtr, ps.thr, KS, LS);
                        cmac(vZ, vce, KS);
                    }
                    const cplx am = cload(aqsm + (size_t)nn * ng + p);
                    cmac(acc[u0 + u], am, vZ);
                }
            }
        }
    }
}

template <int NW>
__global__ void __launch_bounds__(kBwdThreads)
__attribute__((amdgpu_waves_per_eu(GPP_BWD_BANDS_WAVES)))
bwd_bands(int nb, int nv, int ng, int np, long ntiles, int nbt, int ngt, int nps,
          const double2 *__restrict__ aqsm, const double2 *__restrict__ ieps,
          const double2 *__restrict__ wt, const double *__restrict__ vcoul,
          const double *__restrict__ wx, const double2 *__restrict__ gh,
          const double2 *__restrict__ xgh, const double2 *__restrict__ gs,
          double2 *__restrict__ grad_an)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const long tile = (long)xcd_remap(blockIdx.x, gridDim.x) * kBwdWaves + wid;
    if (tile >= ntiles) return;  // wave-uniform; no barriers below
    // band tile fastest (neighbouring waves share the g rows of wtilde/I_eps),
    // then g tile, then segment of the p range
    const long per_seg = (long)ngt * nbt;
    const int seg = (int)(tile / per_seg);
    const long in_seg = tile - (long)seg * per_seg;
    const int gt = (int)(in_seg / nbt);
    const int n0 = (int)(in_seg - (long)gt * nbt) * kBandTile;
    const int p_lo = (int)((long)np * seg / nps), p_hi = (int)((long)np * (seg + 1) / nps);
    // one segment writes the gradient itself, several write partial sums
    double2 *const dst = grad_an + (size_t)seg * nb * ng;
    const int g = gt * kWave + lane;
    const bool valid = g < ng;
    const int gc = valid ? g : ng - 1;

    cplx acc[kBandTile];
#pragma unroll
    for (int u = 0; u < kBandTile; ++u) acc[u] = cmake(0.0, 0.0);
    if (n0 >= nv && n0 + kBandTile <= nb)
        bands_fast<NW>(nb, ng, p_lo, p_hi, n0, gc, valid ? vcoul[gc] : 0.0, as_global(aqsm),
                       as_global(ieps), as_global(wt), as_global(wx), as_global(gh),
                       as_global(xgh), acc);
    else
        bands_generic<NW>(nb, nv, ng, p_lo, p_hi, n0, gc, valid, aqsm, ieps, wt, vcoul, wx, gh,
                          gs, acc);
    if (valid) {
#pragma unroll
        for (int u = 0; u < kBandTile; ++u) {
            const int n = n0 + u;
            if (n < nb) dst[(size_t)n * ng + g] = make_double2(acc[u].re, acc[u].im);
        }
    }
}

// daqsmtemp[n][p] = sum over row blocks of the partials (p < np), 0 for
// columns np..ncouls-1.  One thread per output element, fixed order.
__global__ void reduce_am(int nb, int ng, int np, int ngb, const double2 *__restrict__ part,
                          double2 *__restrict__ grad_am)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nb * ng) return;
    const int n = (int)(i / ng), col = (int)(i - (long)n * ng);
    double re = 0.0, im = 0.0;
    if (col < np) {
        for (int b = 0; b < ngb; ++b) {
            const double2 v = part[((size_t)b * nb + n) * np + col];
            re += v.x;
            im += v.y;
        }
    }
    grad_am[i] = make_double2(re, im);
}

// daqsntemp = sum of the nps segment partials, in segment order.
__global__ void reduce_an(long nbg, int nps, const double2 *__restrict__ part,
                          double2 *__restrict__ grad_an)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbg) return;
    double re = 0.0, im = 0.0;
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
        geo.ngt = (d.ng + kWave - 1) / kWave;
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
        geo.band_blocks = (geo.band_tiles + kBwdWaves - 1) / kBwdWaves;
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
    const int prep = d.nw * d.nb > d.nw ? d.nw * d.nb : d.nw;
    hipLaunchKernelGGL(bwd_prepare, dim3((prep + 255) / 256), dim3(256), 0, st, d.nb, d.nw,
                       in.wx, ga, gh, xgh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool want_pairs = out.grad_wt || out.grad_ieps || out.grad_am;
    if (want_pairs) {
        hipLaunchKernelGGL(bwd_pairs<NW>, dim3((unsigned)geo.pair_blocks), dim3(kBwdThreads), 0,
                           st, d.nb, d.nv, d.ng, d.np, geo.pair_blocks, in.aqsm, in.aqsn,
                           in.ieps, in.wt, in.vcoul, in.wx, gh, xgh, gs, out.grad_wt,
                           out.grad_ieps, out.grad_am ? am_part : nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (out.grad_am) {
        const long n = (long)d.nb * d.ng;
        hipLaunchKernelGGL(reduce_am, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d.nb,
                           d.ng, d.np, geo.ngb, am_part, out.grad_am);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (out.grad_an) {
        double2 *an_dst = geo.nps > 1 ? an_part : out.grad_an;
        hipLaunchKernelGGL(bwd_bands<NW>, dim3((unsigned)geo.band_blocks), dim3(kBwdThreads), 0,
                           st, d.nb, d.nv, d.ng, d.np, geo.band_tiles, geo.nbt, geo.ngt, geo.nps,
                           in.aqsm, in.ieps, in.wt, in.vcoul, in.wx, gh, xgh, gs, an_dst);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (geo.nps > 1) {
            const long nbg = (long)d.nb * d.ng;
            hipLaunchKernelGGL(reduce_an, dim3((unsigned)((nbg + 255) / 256)), dim3(256), 0, st,
                               nbg, geo.nps, an_part, out.grad_an);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
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
