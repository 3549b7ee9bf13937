// gpp_fwd_tile.h -- the forward work of one wave tile (one or several G'
// columns x 64 consecutive G rows), shared by the plain forward and the
// persistent batched kernel so both run the same arithmetic.  See
// gpp_fwd.hip for the derivation.
#pragma once

#include "gpp_device.h"

// 1: the columns of a multi-column tile share one batch inversion per band
// group; 0: one inversion per column.
#ifndef GPP_FWD_JOINT_INV
#define GPP_FWD_JOINT_INV 1
#endif

namespace gpp {

// Column tiles per block of the tile walk: 0 walks each g-tile through all
// column tiles in turn; Q > 0 walks blocks of Q column tiles through all
// g-tiles, so that the block's aqsmtemp columns (Q * cols * 16 bytes per
// band: 2 MB at 128 two-column tiles and 512 bands, half an XCD's L2) stay
// in the L2 while the g-tiles' aqsntemp rows stream past, each row fetched
// once per block.  Measured with band chunks of 512 on MI355X: Q = 128
// took the HBM-side traffic of the 1024-band forward from 45.3 GB (Q = 64)
// to 39.1 GB and its time, the 512-band one's and the 64-state batched
// workload's down by 0.4-0.9 %; Q = 160 and 192 (2.5 and 3 MB) thrashed
// the L2 (85 and 98 GB) and ran slower.
#ifndef GPP_FWD_COL_BLOCK
#define GPP_FWD_COL_BLOCK 128
#endif

// (g-tile, column tile, band chunk) of a tile index, a bijection on
// [0, gtiles * npt * nchunk).  Within a block of Q column tiles the walk
// takes band chunk by band chunk, each through all g-tiles.  The results
// are wave-uniform and made scalar explicitly, since the divisions run on
// the vector unit and a column index left in vector registers would turn
// the tile's aqsmtemp loads into vector loads.
__device__ inline void tile_coords(long tile, int npt, int gtiles, int nchunk, int &gt, int &pt,
                                   int &ck)
{
#if GPP_FWD_COL_BLOCK > 0
    constexpr int Q = GPP_FWD_COL_BLOCK;
    const long per = (long)Q * gtiles * nchunk;
    const int c = (int)(tile / per);
    long r = tile - (long)c * per;
    const int c0 = c * Q;
    const int qc = npt - c0 < Q ? npt - c0 : Q;  // the last block may be short
    const long per_chunk = (long)qc * gtiles;
    ck = (int)(r / per_chunk);
    r -= (long)ck * per_chunk;
    gt = (int)(r / qc);
    pt = c0 + (int)(r - (long)gt * qc);
#else
    const long per_chunk = (long)gtiles * npt;
    ck = (int)(tile / per_chunk);
    const long r = tile - (long)ck * per_chunk;
    gt = (int)(r / npt);
    pt = (int)(r - (long)gt * npt);
#endif
    gt = __builtin_amdgcn_readfirstlane(gt);
    pt = __builtin_amdgcn_readfirstlane(pt);
    ck = __builtin_amdgcn_readfirstlane(ck);
}

// CH-only accumulation for BU consecutive unoccupied bands starting at n.
// aqsntemp[n][g] is read through a buffer descriptor for the row (scalar
// registers) plus the lane's 32-bit byte offset, so the per-band address
// arithmetic stays on the scalar unit.  The denominators go into the batch
// inversion unclamped: every one is at least (Im om)^2, and a lane with
// (Im om)^2 below kMinUnclampedWi2 (wide == false) inverts one by one; a
// masked term's reciprocal (possibly infinite or NaN there) never reaches
// the sums (ch_term).
// The group's aqsntemp values of this lane (one per band).
template <int BU>
__device__ __forceinline__ void load_an(int n, int ng, gptr<double2> aqsn, uint32_t goff,
                                        cplx (&an)[BU])
{
#pragma unroll
    for (int u = 0; u < BU; ++u) an[u] = load_row_elem(aqsn + (size_t)(n + u) * ng, ng, goff);
}

// an conj(am) for a lane's aqsntemp value and a wave-uniform aqsmtemp
// value; the sign sits on the uniform factor, so it folds into an operand
// modifier instead of costing a vector instruction.
__device__ __forceinline__ cplx qm_of(cplx an, cplx am) {
    const double nai = -am.im;
    return cmake(fma(an.re, am.re, an.im * am.im), fma(an.im, am.re, an.re * nai));
}

// One Coulomb-hole term: P1 += r x qm and P2 += r qm when the term is on
// branch A (isA).  With GPP_EXEC_MASK the test is the wave's execution mask
// around the accumulation, laid out as the common case so that no skip
// branch is emitted; otherwise the reciprocal is cleared with mask_keep.
__device__ __forceinline__ void ch_term(bool isA, double r, double x, cplx qm, cplx &P1,
                                        cplx &P2) {
#if GPP_EXEC_MASK
    if (__builtin_expect(isA, 1)) {
        const double rx = r * x;
        P1.re = fma(rx, qm.re, P1.re);
        P1.im = fma(rx, qm.im, P1.im);
        P2.re = fma(r, qm.re, P2.re);
        P2.im = fma(r, qm.im, P2.im);
    }
#else
    const double re = mask_keep(isA, r);
    const double rx = re * x;
    P1.re = fma(rx, qm.re, P1.re);
    P1.im = fma(rx, qm.im, P1.im);
    P2.re = fma(re, qm.re, P2.re);
    P2.im = fma(re, qm.im, P2.im);
#endif
}

// ch_term on the denominator d against the branch-A threshold thr.  With
// GPP_EXEC_MASK == 2 the compare writes the execution mask itself
// (v_cmpx), so the term's five vector instructions wait on one vector
// result instead of a compare, a scalar mask update and the exec write;
// the mask is restored before the block ends.
__device__ __forceinline__ void ch_term_dt(double d, double thr, double r, double x, cplx qm,
                                           cplx &P1, cplx &P2) {
#if GPP_EXEC_MASK == 2
    unsigned long long saved;
    double rx;
    // Not volatile: the block touches no memory and restores exec, and a
    // volatile block would count as a possible store, which keeps the
    // compiler from turning later wave-uniform loads into scalar loads.
    asm(
        "s_mov_b64 %[sv], exec\n\t"
        "v_cmpx_gt_f64_e32 vcc, %[d], %[thr]\n\t"
        "v_mul_f64 %[rx], %[r], %[x]\n\t"
        "v_fma_f64 %[p2r], %[r], %[qr], %[p2r]\n\t"
        "v_fma_f64 %[p2i], %[r], %[qi], %[p2i]\n\t"
        "v_fma_f64 %[p1r], %[rx], %[qr], %[p1r]\n\t"
        "v_fma_f64 %[p1i], %[rx], %[qi], %[p1i]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [sv] "=&s"(saved), [rx] "=&v"(rx), [p1r] "+v"(P1.re), [p1i] "+v"(P1.im),
          [p2r] "+v"(P2.re), [p2i] "+v"(P2.im)
        : [d] "v"(d), [thr] "v"(thr), [r] "v"(r), [x] "s"(x), [qr] "v"(qm.re), [qi] "v"(qm.im)
        : "vcc");
#else
    ch_term(d > thr, r, x, qm, P1, P2);
#endif
}

template <int NW, int BU>
__device__ __forceinline__ void ch_group_an(int n, int nb, int ng, const cplx (&an)[BU],
                                            gptr<double2> am_col, gptr<double> wx, double a,
                                            double wi2, double thr, bool wide, cplx (&P1)[NW],
                                            cplx (&P2)[NW])
{
    constexpr int K = BU * NW;
    cplx qm[BU];
    double xs[K], d[K], r[K];
#pragma unroll
    for (int u = 0; u < BU; ++u) {
        qm[u] = qm_of(an[u], cload(am_col + (size_t)(n + u) * ng));
#pragma unroll
        for (int w = 0; w < NW; ++w) xs[u * NW + w] = wx[(size_t)w * nb + n + u];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double dr = xs[k] - a;
        d[k] = fma(dr, dr, wi2);
    }
    batch_reciprocal<K>(d, r, wide);
#pragma unroll
    for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int k = u * NW + w;
            ch_term_dt(d[k], thr, r[k], xs[k], qm[u], P1[w], P2[w]);
        }
}

// As ch_group_an for NC columns at once: the BU*NW*NC denominators of the
// group share one batch inversion, which takes NC-1 fewer hardware
// reciprocals and Newton steps for NC-1 more multiplies per link of the
// prefix chain.  wide must hold for every column of the lane.
template <int NW, int BU, int NC>
__device__ __forceinline__ void ch_group_cols(int n, int nb, int ng, const cplx (&an)[BU],
                                              gptr<double2> aqsm, const int (&pc)[NC],
                                              gptr<double> wx, const double (&a)[NC],
                                              const double (&wi2)[NC], const double (&thr)[NC],
                                              bool wide, cplx (&P1)[NC][NW],
                                              cplx (&P2)[NC][NW])
{
    constexpr int KB = BU * NW;  // terms of one column
    constexpr int K = NC * KB;
    double xs[KB], d[K], r[K];
    cplx qm[NC][BU];
#pragma unroll
    for (int u = 0; u < BU; ++u) {
#pragma unroll
        for (int w = 0; w < NW; ++w) xs[u * NW + w] = wx[(size_t)w * nb + n + u];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            qm[c][u] = qm_of(an[u], cload(aqsm + pc[c] + (size_t)(n + u) * ng));
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const double dr = xs[k] - a[c];
            d[c * KB + k] = fma(dr, dr, wi2[c]);
        }
    }
    batch_reciprocal<K>(d, r, wide);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int u = 0; u < BU; ++u)
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int k = c * KB + u * NW + w;
                ch_term_dt(d[k], thr[c], r[k], xs[u * NW + w], qm[c][u], P1[c][w], P2[c][w]);
            }
}

template <int NW, int BU>
__device__ __forceinline__ void ch_group(int n, int nb, int ng, gptr<double2> aqsn,
                                         uint32_t goff, gptr<double2> am_col,
                                         gptr<double> wx, double a, double wi2, double thr,
                                         bool wide, cplx (&P1)[NW], cplx (&P2)[NW])
{
    cplx an[BU];
    load_an<BU>(n, ng, aqsn, goff, an);
    ch_group_an<NW, BU>(n, nb, ng, an, am_col, wx, a, wi2, thr, wide, P1, P2);
}

// Frequencies W0 .. W0+G-1 of one occupied band (see occupied_bands).
template <int NW, int W0, int G>
__device__ __forceinline__ void occupied_freqs(int n, int nb, gptr<double> wx, double a, double b,
                                               double wi2, double wtr, double thr, bool wide,
                                               cplx om2, cplx qm, cplx (&P1)[NW],
                                               cplx (&P2)[NW], cplx (&SX)[NW])
{
    double xs[G], wd[G], ws[G], r[G], rs[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        xs[k] = wx[(size_t)(W0 + k) * nb + n];
        const double dr = xs[k] - a, sp = xs[k] + a;
        wd[k] = fma(dr, dr, wi2);  // |x - om|^2, the branch's wdiffr
        ws[k] = fma(sp, sp, wi2);  // |x + om|^2
    }
    if constexpr (G > 1) {
        batch_reciprocal<G>(wd, r, wide);
        batch_reciprocal<G>(ws, rs, wide);
    } else {
        r[0] = rcp_nr2(wd[0]);
        rs[0] = rcp_nr2(ws[0]);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const int w = W0 + k;
        const double x = xs[k];
        const double dr = x - a, sp = x + a;
        const bool isA = wd[k] > thr;
        const double rc = isA ? r[k] : 0.0;
        const double rx = rc * x;
        P1[w].re = fma(rx, qm.re, P1[w].re);
        P1[w].im = fma(rx, qm.im, P1[w].im);
        P2[w].re = fma(rc, qm.re, P2[w].re);
        P2[w].im = fma(rc, qm.im, P2[w].im);
        // both branches' values carry rs: A = r om^2 conj(d s), B = -om conj(s) / 2
        const cplx na = cscale(r[k], cmul(om2, cmake(fma(dr, sp, wi2), om2.im)));
        const cplx nb2 = cmake(-0.5 * fma(a, sp, wi2), -0.5 * (b * x));
        const bool isB = branch_b_holds(wtr, wd[k]);
        cplx t;
        t.re = rs[k] * (isA ? na.re : (isB ? nb2.re : 0.0));
        t.im = rs[k] * (isA ? na.im : (isB ? nb2.im : 0.0));
        cmac(SX[w], qm, t);
    }
}

// Frequencies per batch-inverted group of an occupied band: all three at
// up to three frequencies; one at a time beyond, where the groups'
// reciprocals would raise the kernel's register count above the hot loop's.
#ifndef GPP_OCC_GROUP
#define GPP_OCC_GROUP 0
#endif
constexpr int occ_group(int nw) { return GPP_OCC_GROUP ? GPP_OCC_GROUP : (nw <= 3 ? nw : 1); }

template <int NW, int W0>
__device__ __forceinline__ void occupied_groups(int n, int nb, gptr<double> wx, double a, double b,
                                                double wi2, double wtr, double thr, bool wide,
                                                cplx om2, cplx qm, cplx (&P1)[NW],
                                                cplx (&P2)[NW], cplx (&SX)[NW])
{
    constexpr int G = NW - W0 < occ_group(NW) ? NW - W0 : occ_group(NW);
    occupied_freqs<NW, W0, G>(n, nb, wx, a, b, wi2, wtr, thr, wide, om2, qm, P1, P2, SX);
    if constexpr (W0 + G < NW)
        occupied_groups<NW, W0 + G>(n, nb, wx, a, b, wi2, wtr, thr, wide, om2, qm, P1, P2, SX);
}

// Occupied bands n0 <= n < n1 (all below nvband) of one lane and one
// column: Coulomb-hole terms into P1/P2 and screened-exchange terms
// (ssx / e) into SX.  With d = x - om and s = x + om, the exchange term is
//   A:  om^2 / (d s) = om^2 conj(d s) r rs,     r = 1/|d|^2, rs = 1/|s|^2
//   B:  -om / (2 s)  = -om conj(s) rs / 2
// where d s = x^2 - om^2 has real part fma(Re d, Re s, (Im om)^2) (both
// factors exact to rounding even where x is near -Re om) and imaginary
// part -2 Re om Im om, and om conj(s) = (fma(Re om, Re s, (Im om)^2),
// Im om x).  The band's reciprocals of |d|^2 and of |s|^2 come from two
// batch inversions per group of frequencies (both are at least
// (Im om)^2, like the hot loop's denominators); the branch picks each
// term's value by selects, so a value computed for another branch never
// reaches the sums.
template <int NW>
__device__ __forceinline__ void occupied_bands(int n0, int n1, int nb, int ng,
                                               gptr<double2> an_col, gptr<double2> am_col,
                                               gptr<double> wx, cplx om, double wi2, double wtr,
                                               double thr, cplx (&P1)[NW], cplx (&P2)[NW],
                                               cplx (&SX)[NW])
{
    const double a = om.re, b = om.im;
    const cplx om2 = cmake(fma(a, a, -wi2), 2.0 * a * b);  // om^2
    const bool wide = wi2 >= kMinUnclampedWi2;
    for (int n = n0; n < n1; ++n) {
        const cplx an = cload(an_col + (size_t)n * ng);
        const cplx am = cload(am_col + (size_t)n * ng);
        const cplx qm = cmul_conj(an, am);
        occupied_groups<NW, 0>(n, nb, wx, a, b, wi2, wtr, thr, wide, om2, qm, P1, P2, SX);
    }
}

// One tile: lane g = gt*64 + lane of column p, bands n_lo <= n < n_hi.  On
// return ach[w] holds this lane's Coulomb-hole contribution (still to be
// summed over the wave) and asx[w] the wave's screened-exchange total
// (wave-uniform).  Must be called by all 64 lanes of a wave together (wave
// reductions inside).
template <int NW, int BU>
__device__ __forceinline__ void fwd_tile_body(int nb, int nv, int n_lo, int n_hi, int ng, int p,
                                              int gt, int lane,
                                              gptr<double2> aqsm, gptr<double2> aqsn,
                                              gptr<double2> ieps, gptr<double2> wt,
                                              gptr<double> vcoul, gptr<double> wx,
                                              cplx (&ach)[NW], cplx (&asx)[NW])
{
    const int g = gt * kWave + lane;
    const bool valid = g < ng;
    const int gc = valid ? g : ng - 1;  // clamped, contribution zeroed

    const cplx om = cload(wt + (size_t)p * ng + gc);
    const double a = om.re, b = om.im;
    const double wi2 = b * b;
    const double wtr = fma(a, a, wi2);
    const double thr = branch_a_threshold(wtr);

    cplx P1[NW], P2[NW], SX[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) P1[w] = P2[w] = SX[w] = cmake(0.0, 0.0);

    const gptr<double2> an_col = aqsn + gc;
    const gptr<double2> am_col = aqsm + p;
    const uint32_t goff = (uint32_t)gc * (uint32_t)sizeof(double2);
    const cplx e = cload(ieps + (size_t)p * ng + gc);
    const double v = valid ? vcoul[gc] : 0.0;
    const cplx ev = cscale(v, e);

    // occupied bands: screened exchange (SX) and Coulomb hole (CH)
    const int occ_hi = nv < n_hi ? nv : n_hi;
    occupied_bands<NW>(n_lo, occ_hi, nb, ng, an_col, am_col, wx, om, wi2, wtr, thr, P1, P2, SX);
    // The exchange sums are finished here and reduced over the wave into
    // scalar registers, so they hold no vector registers in the hot loop.
    if (occ_hi > n_lo) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const cplx t = cmul(ev, SX[w]);
            asx[w] = cmake(wave_sum_uniform(t.re), wave_sum_uniform(t.im));
        }
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) asx[w] = cmake(0.0, 0.0);
    }

    // unoccupied bands: CH only -- the hot loop
    const bool wide = wi2 >= kMinUnclampedWi2;
    int n = nv > n_lo ? nv : n_lo;
    for (; n + BU <= n_hi; n += BU)
        ch_group<NW, BU>(n, nb, ng, aqsn, goff, am_col, wx, a, wi2, thr, wide, P1, P2);
    for (; n < n_hi; ++n)
        ch_group<NW, 1>(n, nb, ng, aqsn, goff, am_col, wx, a, wi2, thr, wide, P1, P2);

#pragma unroll
    for (int w = 0; w < NW; ++w) {
        // S = om P1 - wtr P2
        cplx S = cmul(om, P1[w]);
        S.re = fma(-wtr, P2[w].re, S.re);
        S.im = fma(-wtr, P2[w].im, S.im);
        ach[w] = cscale(0.5, cmul(ev, S));
    }
}

// NC consecutive G' columns p0 .. p0+NC-1 of one 64-row tile per wave,
// bands n_lo <= n < n_hi: each aqsntemp element a lane loads serves all of
// them, which divides the vector-memory traffic of the hot loop by NC.
// Columns at or beyond np repeat p0 and their contribution is dropped.
// Outputs as fwd_tile_body, for the NC columns together.
template <int NW, int BU, int NC>
__device__ __forceinline__ void fwd_tile_body_cols(int nb, int nv, int n_lo, int n_hi, int ng,
                                                   int np, int p0, int gt, int lane,
                                                   gptr<double2> aqsm,
                                                   gptr<double2> aqsn, gptr<double2> ieps,
                                                   gptr<double2> wt, gptr<double> vcoul,
                                                   gptr<double> wx, cplx (&ach)[NW],
                                                   cplx (&asx)[NW])
{
    const int g = gt * kWave + lane;
    const bool valid = g < ng;
    const int gc = valid ? g : ng - 1;  // clamped, contribution zeroed

    int pc[NC];
    bool has[NC];
    cplx om[NC];
    double a[NC], wi2[NC], thr[NC];
    bool wide[NC];
    cplx P1[NC][NW], P2[NC][NW];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        has[c] = p0 + c < np;
        pc[c] = has[c] ? p0 + c : p0;
        om[c] = cload(wt + (size_t)pc[c] * ng + gc);
        a[c] = om[c].re;
        wi2[c] = om[c].im * om[c].im;
        thr[c] = branch_a_threshold(fma(a[c], a[c], wi2[c]));
        wide[c] = wi2[c] >= kMinUnclampedWi2;
#pragma unroll
        for (int w = 0; w < NW; ++w) P1[c][w] = P2[c][w] = cmake(0.0, 0.0);
    }
    const gptr<double2> an_col = aqsn + gc;
    const uint32_t goff = (uint32_t)gc * (uint32_t)sizeof(double2);
    const double v = valid ? vcoul[gc] : 0.0;

    // occupied bands, column by column; the exchange sums of all columns
    // are reduced over the wave into scalar registers before the hot loop
    const int occ_hi = nv < n_hi ? nv : n_hi;
    if (occ_hi > n_lo) {
        cplx sx[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) sx[w] = cmake(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            cplx SX[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) SX[w] = cmake(0.0, 0.0);
            occupied_bands<NW>(n_lo, occ_hi, nb, ng, an_col, aqsm + pc[c], wx, om[c], wi2[c],
                               fma(a[c], a[c], wi2[c]), thr[c], P1[c], P2[c], SX);
            const double vc = has[c] ? v : 0.0;
            const cplx ev = cscale(vc, cload(ieps + (size_t)pc[c] * ng + gc));
#pragma unroll
            for (int w = 0; w < NW; ++w) cmac(sx[w], ev, SX[w]);
        }
#pragma unroll
        for (int w = 0; w < NW; ++w)
            asx[w] = cmake(wave_sum_uniform(sx[w].re), wave_sum_uniform(sx[w].im));
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) asx[w] = cmake(0.0, 0.0);
    }

    // unoccupied bands: CH only
    int n = nv > n_lo ? nv : n_lo;
#if GPP_FWD_JOINT_INV
    bool wide_all = true;
#pragma unroll
    for (int c = 0; c < NC; ++c) wide_all = wide_all && wide[c];
    for (; n + BU <= n_hi; n += BU) {
        cplx an[BU];
        load_an<BU>(n, ng, aqsn, goff, an);
        ch_group_cols<NW, BU, NC>(n, nb, ng, an, aqsm, pc, wx, a, wi2, thr, wide_all, P1, P2);
    }
    for (; n < n_hi; ++n) {
        cplx an[1];
        load_an<1>(n, ng, aqsn, goff, an);
        ch_group_cols<NW, 1, NC>(n, nb, ng, an, aqsm, pc, wx, a, wi2, thr, wide_all, P1, P2);
    }
#else
    for (; n + BU <= n_hi; n += BU) {
        cplx an[BU];
        load_an<BU>(n, ng, aqsn, goff, an);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            ch_group_an<NW, BU>(n, nb, ng, an, aqsm + pc[c], wx, a[c], wi2[c], thr[c], wide[c],
                                P1[c], P2[c]);
            // one column's reciprocal chain at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    for (; n < n_hi; ++n) {
        cplx an[1];
        load_an<1>(n, ng, aqsn, goff, an);
#pragma unroll
        for (int c = 0; c < NC; ++c)
            ch_group_an<NW, 1>(n, nb, ng, an, aqsm + pc[c], wx, a[c], wi2[c], thr[c], wide[c],
                               P1[c], P2[c]);
    }
#endif

#pragma unroll
    for (int w = 0; w < NW; ++w) ach[w] = cmake(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double vc = has[c] ? v : 0.0;
        const cplx ev = cscale(vc, cload(ieps + (size_t)pc[c] * ng + gc));
        const double wtr = fma(a[c], a[c], wi2[c]);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            // S = om P1 - wtr P2
            cplx S = cmul(om[c], P1[c][w]);
            S.re = fma(-wtr, P2[c][w].re, S.re);
            S.im = fma(-wtr, P2[c][w].im, S.im);
            const cplx t = cscale(0.5, cmul(ev, S));
            ach[w] = cadd(ach[w], t);
        }
    }
}

}  // namespace gpp
