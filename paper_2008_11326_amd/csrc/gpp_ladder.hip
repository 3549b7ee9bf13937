// gpp_ladder.hip -- the optimisation steps of the paper's Sec. III (v0-v8)
// as gfx950 kernels of the forward reduction, for timing each step against
// the others and against the production kernel (entry points declared in
// include/gpp_ladder.h).
//
// Every step computes the reduction of include/gpp.h.  What changes from
// step to step is what the paper changes:
//   divides      v0: IEEE complex divides; v1 on: one reciprocal (rcp_nr2)
//                of |denominator|^2 per complex divide
//   branch       v0-v1: if A / else if B / else zero; v2 on: outputs preset
//                to zero, if A / else if B
//   predicate    v0-v2: moduli by square roots, A <=> |x-om| > 0.5 and
//                |om| < 500 |x-om|, B <=> |om| > 1e-6 |x-om| (the abs() form
//                multiplied out, so an exact pole needs no quotient); v3 on:
//                the exact squared, cross-multiplied predicate of gpp.h
//   mapping      v0-v3: one thread per (n, p, g), g fastest, grid-stride
//                (the collapsed three-loop nest); v4 on: one thread per
//                (p, g), bands serial inside the thread
//   frequencies  v0-v4: all frequencies of a (n, p, g) in one thread; v5
//                on: one launch per frequency, recomputing M each time
//   blocking     v6 on: the aqsntemp rows of kBandBlock bands staged in LDS
//                and shared by the four waves (four G' columns) of a
//                workgroup
//   layout       v7 on: aqsmtemp read from a [ngpown][number_bands] copy
//                (band-contiguous per G' column), made inside the call
//   registers    v8: the kernel held to 80 VGPRs (6 waves per SIMD, one
//                step above its natural 5, at the price of a few spills)
// and then two steps toward the production kernel: m1 (v4's mapping with
// the Coulomb-hole sum factored, lad_factored) and m2 (m1 with batch
// inversion), before the production forward itself.
// Each workgroup writes one partial row of 4*nfreq doubles; the forward's
// fixed-order two-stage reduction adds them.  No atomics.
#include <math.h>

#include "gpp_device.h"
#include "gpp_internal.h"
#include "gpp_ladder.h"

namespace gpp {
namespace {

enum class Div { Ieee, Rcp };
enum class Pred { Abs, Square };
enum class Br { Three, Two };

constexpr int kLadThreads = 256;
constexpr int kLadWaves = kLadThreads / kWave;
constexpr int kBandBlock = 16;      // bands per LDS block (v6-v8)
constexpr long kCollapseBlocks = 2048;  // grid of the grid-stride kernels (8 per CU)

// a / b (complex).  Only called where b != 0.
template <Div D>
__device__ __forceinline__ cplx cdiv_step(cplx a, cplx b)
{
    const double den = fma(b.re, b.re, b.im * b.im);
    const double nr = fma(a.re, b.re, a.im * b.im);
    const double ni = fma(a.im, b.re, -(a.re * b.im));
    if (D == Div::Ieee) return cmake(nr / den, ni / den);
    const double r = rcp_nr2(den);
    return cmake(nr * r, ni * r);
}

// The frequencies [w0, w0 + NWK) of one (n, p, g): with y = vcoul/2 * M * e,
// acc gets y sch into (re, im) of achtemp and 2 y ssx (occupied bands) into
// (re, im) of asxtemp, per frequency.  wxn points at wx_array[0][n].
template <int NWK, Div D, Pred P, Br B>
__device__ __forceinline__ void lad_terms(cplx y, cplx om, bool occ, const double *wxn, int nb,
                                          int w0, double (&acc)[4 * NWK])
{
    const double a = om.re, b = om.im;
    const double wi2 = b * b;
    const double wtr = fma(a, a, wi2);
    const double thr = P == Pred::Square ? branch_a_threshold(wtr) : 0.0;
    const double omr = P == Pred::Abs ? sqrt(wtr) : 0.0;  // |om|
#pragma unroll
    for (int w = 0; w < NWK; ++w) {
        const double x = wxn[(size_t)(w0 + w) * nb];
        const cplx d = cmake(x - a, -b);  // x - om
        bool isA, isB;
        if (P == Pred::Abs) {
            const double wdr = sqrt(fma(d.re, d.re, wi2));  // |x - om|
            isA = wdr > 0.5 && omr < 500.0 * wdr;
            isB = omr > 1e-6 * wdr;
        } else {
            const double wd = fma(d.re, d.re, wi2);
            isA = wd > thr;
            isB = branch_b_holds(wtr, wd);
        }
        cplx sch, ssx;
        if (B == Br::Two) sch = ssx = cmake(0.0, 0.0);
        if (isA) {
            sch = cdiv_step<D>(om, d);
            ssx = occ ? cdiv_step<D>(cmul(om, om), cmul(d, cmake(x + a, b))) : cmake(0.0, 0.0);
        } else if (isB) {
            sch = cmake(0.0, 0.0);
            ssx = occ ? cdiv_step<D>(om, cmake(-2.0 * (x + a), -2.0 * b)) : cmake(0.0, 0.0);
        } else if (B == Br::Three) {
            sch = ssx = cmake(0.0, 0.0);
        }
        const cplx ts = cmul(y, sch), tx = cmul(y, ssx);
        acc[4 * w + 0] += ts.re;
        acc[4 * w + 1] += ts.im;
        acc[4 * w + 2] += 2.0 * tx.re;
        acc[4 * w + 3] += 2.0 * tx.im;
    }
}

// Sum acc over the workgroup (wave shuffles, then LDS over the waves) and
// write it to columns [col, col + W) of this workgroup's partial row.
template <int W>
__device__ __forceinline__ void lad_block_store(double (&acc)[W], double *__restrict__ row,
                                                int col)
{
    __shared__ double red[kLadWaves][W];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const double s = wave_sum(acc[j]);
        if (lane == 0) red[wid][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < W) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kLadWaves; ++k) s += red[k][threadIdx.x];
        row[col + threadIdx.x] = s;
    }
}

// v0-v3: thread <-> (n, p, g), flat index f = (n np + p) ng + g, grid-stride.
// The indices advance by the stride incrementally (Sg = S mod ng, and the
// carry into p and n), so no per-iteration 64-bit division.
template <int NW, Div D, Pred P, Br B>
__global__ void __launch_bounds__(kLadThreads)
lad_collapse3(int nb, int nv, int ng, int np, int sg, int sp, int sn, DevInputs in,
              double *__restrict__ partials)
{
    double acc[4 * NW];
#pragma unroll
    for (int j = 0; j < 4 * NW; ++j) acc[j] = 0.0;
    const long f0 = (long)blockIdx.x * kLadThreads + threadIdx.x;
    int g = (int)(f0 % ng);
    const long q = f0 / ng;
    int p = (int)(q % np);
    int n = (int)(q / np);
    while (n < nb) {
        const cplx an = cload(in.aqsn + (size_t)n * ng + g);
        const cplx am = cload(in.aqsm + (size_t)n * ng + p);
        const cplx om = cload(in.wt + (size_t)p * ng + g);
        const cplx e = cload(in.ieps + (size_t)p * ng + g);
        const double v = in.vcoul[g];
        const cplx y = cscale(0.5 * v, cmul(cmul_conj(an, am), e));
        lad_terms<NW, D, P, B>(y, om, n < nv, in.wx + n, nb, 0, acc);
        g += sg;
        int carry = 0;
        if (g >= ng) {
            g -= ng;
            carry = 1;
        }
        p += sp + carry;
        if (p >= np) {
            p -= np;
            ++n;
        }
        n += sn;
    }
    lad_block_store<4 * NW>(acc, partials + (size_t)blockIdx.x * 4 * NW, 0);
}

// v4 (NWK = nw, w0 = 0) and v5 (NWK = 1, one launch per w0): thread <-> (p, g)
// with f = p ng + g; bands serial.  Row width 4 nw; this launch fills its
// frequencies' columns.
template <int NWK, Div D, Pred P, Br B>
__global__ void __launch_bounds__(kLadThreads)
lad_bandinner(int nb, int nv, int ng, int np, int w0, int nw, DevInputs in,
              double *__restrict__ partials)
{
    double acc[4 * NWK];
#pragma unroll
    for (int j = 0; j < 4 * NWK; ++j) acc[j] = 0.0;
    const long f = (long)blockIdx.x * kLadThreads + threadIdx.x;
    if (f < (long)np * ng) {
        const int p = (int)(f / ng), g = (int)(f - (long)p * ng);
        const cplx om = cload(in.wt + (size_t)p * ng + g);
        const cplx ev = cscale(0.5 * in.vcoul[g], cload(in.ieps + (size_t)p * ng + g));
        for (int n = 0; n < nb; ++n) {
            const cplx an = cload(in.aqsn + (size_t)n * ng + g);
            const cplx am = cload(in.aqsm + (size_t)n * ng + p);
            lad_terms<NWK, D, P, B>(cmul(cmul_conj(an, am), ev), om, n < nv, in.wx + n, nb, w0,
                                    acc);
        }
    }
    lad_block_store<4 * NWK>(acc, partials + (size_t)blockIdx.x * 4 * nw, 4 * w0);
}

// v6-v8, one launch per frequency w0: workgroup = 4 waves = 4 consecutive G'
// columns x the same 64 G rows (workgroup index: g-tile major, column block
// minor).  The aqsntemp rows of kBandBlock bands go through LDS once for the
// 4 waves.  With SWAPPED, aqsmtemp comes from amT[p][n].
template <bool SWAPPED>
__device__ __forceinline__ void lad_blocked_body(int nb, int nv, int ng, int np, int w0, int nw,
                                                 int npb, const DevInputs &in,
                                                 const double2 *__restrict__ amT,
                                                 double *__restrict__ partials)
{
    __shared__ double2 an_s[kBandBlock][kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int gt = (int)(blockIdx.x / npb), pb = (int)(blockIdx.x - (long)gt * npb);
    const int p = pb * kLadWaves + wid, g = gt * kWave + lane;
    const bool live = p < np && g < ng;
    const int pc = p < np ? p : np - 1, gc = g < ng ? g : ng - 1;
    const cplx om = cload(in.wt + (size_t)pc * ng + gc);
    const cplx ev =
        cscale(live ? 0.5 * in.vcoul[gc] : 0.0, cload(in.ieps + (size_t)pc * ng + gc));
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int n0 = 0; n0 < nb; n0 += kBandBlock) {
        __syncthreads();  // the previous block's rows are no longer read
#pragma unroll
        for (int k = 0; k < kBandBlock / kLadWaves; ++k) {
            const int j = wid + kLadWaves * k, n = n0 + j;
            an_s[j][lane] = n < nb ? in.aqsn[(size_t)n * ng + gc] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const int nend = nb - n0 < kBandBlock ? nb - n0 : kBandBlock;
        for (int j = 0; j < nend; ++j) {
            const int n = n0 + j;
            const double2 a2 = an_s[j][lane];
            const cplx an = cmake(a2.x, a2.y);
            const cplx am = SWAPPED ? cload(amT + (size_t)pc * nb + n)
                                    : cload(in.aqsm + (size_t)n * ng + pc);
            lad_terms<1, Div::Rcp, Pred::Square, Br::Two>(cmul(cmul_conj(an, am), ev), om,
                                                          n < nv, in.wx + n, nb, w0, acc);
        }
    }
    lad_block_store<4>(acc, partials + (size_t)blockIdx.x * 4 * nw, 4 * w0);
}

template <bool SWAPPED>
__global__ void __launch_bounds__(kLadThreads)
lad_blocked(int nb, int nv, int ng, int np, int w0, int nw, int npb, DevInputs in,
            const double2 *__restrict__ amT, double *__restrict__ partials)
{
    lad_blocked_body<SWAPPED>(nb, nv, ng, np, w0, nw, npb, in, amT, partials);
}

__global__ void __launch_bounds__(kLadThreads) __attribute__((amdgpu_waves_per_eu(6)))
lad_blocked_capped(int nb, int nv, int ng, int np, int w0, int nw, int npb, DevInputs in,
                   const double2 *__restrict__ amT, double *__restrict__ partials)
{
    lad_blocked_body<true>(nb, nv, ng, np, w0, nw, npb, in, amT, partials);
}

// m1 (BATCH = false) and m2 (BATCH = true): v4's mapping (thread <-> (p, g),
// bands serial, every frequency in registers) with the production
// forward's Coulomb-hole factoring: om/(x - om) = r (x om - |om|^2) with
// r = 1/|x - om|^2, so each lane keeps P1 = sum r x Qm and P2 = sum r Qm
// (Qm = aqsntemp conj(aqsmtemp) per band) and applies om, |om|^2, e and
// vcoul once at the end.  Occupied bands take v4's exact per-term path.  m1
// takes one reciprocal (rcp_nr2) per term; m2 batch-inverts the
// denominators of 3 bands x NW frequencies and masks with the high-word
// clear, as the production kernel does.
template <int NW, bool BATCH>
__global__ void __launch_bounds__(kLadThreads)
lad_factored(int nb, int nv, int ng, int np, DevInputs in, double *__restrict__ partials)
{
    double acc[4 * NW];
#pragma unroll
    for (int j = 0; j < 4 * NW; ++j) acc[j] = 0.0;
    const long f = (long)blockIdx.x * kLadThreads + threadIdx.x;
    if (f < (long)np * ng) {
        const int p = (int)(f / ng), g = (int)(f - (long)p * ng);
        const cplx om = cload(in.wt + (size_t)p * ng + g);
        const cplx ev = cscale(0.5 * in.vcoul[g], cload(in.ieps + (size_t)p * ng + g));
        const double a = om.re, wi2 = om.im * om.im;
        const double wtr = fma(a, a, wi2);
        const double thr = branch_a_threshold(wtr);
        for (int n = 0; n < nv; ++n) {
            const cplx an = cload(in.aqsn + (size_t)n * ng + g);
            const cplx am = cload(in.aqsm + (size_t)n * ng + p);
            lad_terms<NW, Div::Rcp, Pred::Square, Br::Two>(cmul(cmul_conj(an, am), ev), om, true,
                                                          in.wx + n, nb, 0, acc);
        }
        cplx P1[NW], P2[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) P1[w] = P2[w] = cmake(0.0, 0.0);
        int n = nv;
        if (BATCH) {
            constexpr int K = 3 * NW;
            const bool wide = wi2 >= kMinUnclampedWi2;
            for (; n + 3 <= nb; n += 3) {
                cplx qm[3];
                double xs[K], dc[K], r[K];
                bool isA[K];
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    qm[u] = cmul_conj(cload(in.aqsn + (size_t)(n + u) * ng + g),
                                      cload(in.aqsm + (size_t)(n + u) * ng + p));
#pragma unroll
                    for (int w = 0; w < NW; ++w) xs[u * NW + w] = in.wx[(size_t)w * nb + n + u];
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double dr = xs[k] - a;
                    const double wd = fma(dr, dr, wi2);
                    isA[k] = wd > thr;
                    dc[k] = wd;
                }
                batch_reciprocal<K>(dc, r, wide);
#pragma unroll
                for (int u = 0; u < 3; ++u)
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const int k = u * NW + w;
                        const double re = mask_keep(isA[k], r[k]);
                        const double rx = re * xs[k];
                        P1[w].re = fma(rx, qm[u].re, P1[w].re);
                        P1[w].im = fma(rx, qm[u].im, P1[w].im);
                        P2[w].re = fma(re, qm[u].re, P2[w].re);
                        P2[w].im = fma(re, qm[u].im, P2[w].im);
                    }
            }
        }
        for (; n < nb; ++n) {  // m1: every unoccupied band; m2: the ragged tail
            const cplx qm = cmul_conj(cload(in.aqsn + (size_t)n * ng + g),
                                      cload(in.aqsm + (size_t)n * ng + p));
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const double x = in.wx[(size_t)w * nb + n];
                const double dr = x - a;
                const double wd = fma(dr, dr, wi2);
                const double r = wd > thr ? rcp_nr2(wd) : 0.0;
                const double rx = r * x;
                P1[w].re = fma(rx, qm.re, P1[w].re);
                P1[w].im = fma(rx, qm.im, P1[w].im);
                P2[w].re = fma(r, qm.re, P2[w].re);
                P2[w].im = fma(r, qm.im, P2[w].im);
            }
        }
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            cplx S = cmul(om, P1[w]);
            S.re = fma(-wtr, P2[w].re, S.re);
            S.im = fma(-wtr, P2[w].im, S.im);
            const cplx ch = cmul(ev, S);
            acc[4 * w + 0] += ch.re;
            acc[4 * w + 1] += ch.im;
        }
    }
    lad_block_store<4 * NW>(acc, partials + (size_t)blockIdx.x * 4 * NW, 0);
}

// amT[p][n] = aqsmtemp[n][p] for p < np (one thread per element, writes
// coalesced).
__global__ void lad_transpose_am(int nb, int ng, int np, const double2 *__restrict__ aqsm,
                                 double2 *__restrict__ amT)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)np * nb) return;
    const int p = (int)(i / nb), n = (int)(i - (long)p * nb);
    amT[i] = aqsm[(size_t)n * ng + p];
}

const char *const kNames[GPP_LADDER_STEPS] = {
    "v0 collapse-3, IEEE divides, abs predicates, 3-way branch",
    "v1 collapse-3, reciprocals, abs predicates, 3-way branch",
    "v2 collapse-3, reciprocals, abs predicates, 2-way branch",
    "v3 collapse-3, reciprocals, squared predicates, 2-way branch",
    "v4 band loop inside the thread, all frequencies in registers",
    "v5 band loop inside the thread, one launch per frequency",
    "v6 as v5 with aqsntemp rows staged in LDS for 4 G' columns",
    "v7 as v6 with band-contiguous aqsmtemp (transposed copy)",
    "v8 as v7 with an 80-VGPR cap (6 waves per SIMD)",
    "m1 v4 with the Coulomb-hole sum factored (P1/P2), one reciprocal per term",
    "m2 as m1 with batch inversion over 3 bands and high-word masking",
    "production gpp_sigma_fwd",
};

struct LadderGeometry {
    long rows = 0;       // partial rows (workgroups of the main kernel)
    size_t amT_bytes = 0;
    size_t partial_bytes = 0, stage_bytes = 0, workspace_bytes = 0;
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

LadderGeometry ladder_geometry(int step, const Dims32 &d)
{
    LadderGeometry geo;
    const long total = (long)d.nb * d.np * d.ng;
    if (total > 0) {
        if (step <= 3) {
            const long need = (total + kLadThreads - 1) / kLadThreads;
            geo.rows = need < kCollapseBlocks ? need : kCollapseBlocks;
        } else if (step <= 5 || step >= 9) {
            geo.rows = ((long)d.np * d.ng + kLadThreads - 1) / kLadThreads;
        } else {
            geo.rows = (long)((d.ng + kWave - 1) / kWave) * ((d.np + kLadWaves - 1) / kLadWaves);
        }
        if (step == 7 || step == 8) geo.amT_bytes = up256((size_t)d.np * d.nb * sizeof(double2));
    }
    geo.partial_bytes = up256((size_t)geo.rows * 4 * d.nw * sizeof(double));
    geo.stage_bytes = up256(reduce_stage_bytes(d.nw, geo.rows));
    geo.workspace_bytes = geo.amT_bytes + geo.partial_bytes + geo.stage_bytes;
    if (geo.workspace_bytes == 0) geo.workspace_bytes = 256;
    return geo;
}

template <int NW>
hipError_t launch_collapse(int step, const Dims32 &d, const LadderGeometry &geo,
                           const DevInputs &in, double *partials, hipStream_t st)
{
    const long S = geo.rows * kLadThreads;
    const int sg = (int)(S % d.ng);
    const long sq = S / d.ng;
    const int sp = (int)(sq % d.np), sn = (int)(sq / d.np);
    const dim3 grid((unsigned)geo.rows), blk(kLadThreads);
    switch (step) {
    case 0:
        hipLaunchKernelGGL((lad_collapse3<NW, Div::Ieee, Pred::Abs, Br::Three>), grid, blk, 0, st,
                           d.nb, d.nv, d.ng, d.np, sg, sp, sn, in, partials);
        break;
    case 1:
        hipLaunchKernelGGL((lad_collapse3<NW, Div::Rcp, Pred::Abs, Br::Three>), grid, blk, 0, st,
                           d.nb, d.nv, d.ng, d.np, sg, sp, sn, in, partials);
        break;
    case 2:
        hipLaunchKernelGGL((lad_collapse3<NW, Div::Rcp, Pred::Abs, Br::Two>), grid, blk, 0, st,
                           d.nb, d.nv, d.ng, d.np, sg, sp, sn, in, partials);
        break;
    default:
        hipLaunchKernelGGL((lad_collapse3<NW, Div::Rcp, Pred::Square, Br::Two>), grid, blk, 0,
                           st, d.nb, d.nv, d.ng, d.np, sg, sp, sn, in, partials);
        break;
    }
    return hipGetLastError();
}

template <int NW>
hipError_t launch_bandinner_all(const Dims32 &d, const LadderGeometry &geo, const DevInputs &in,
                                double *partials, hipStream_t st)
{
    hipLaunchKernelGGL((lad_bandinner<NW, Div::Rcp, Pred::Square, Br::Two>),
                       dim3((unsigned)geo.rows), dim3(kLadThreads), 0, st, d.nb, d.nv, d.ng, d.np,
                       0, d.nw, in, partials);
    return hipGetLastError();
}

hipError_t launch_ladder(int step, const Dims32 &d, const DevInputs &in, double2 *ach,
                         double2 *asx, char *ws, hipStream_t st)
{
    const LadderGeometry geo = ladder_geometry(step, d);
    double2 *amT = reinterpret_cast<double2 *>(ws);
    double *partials = reinterpret_cast<double *>(ws + geo.amT_bytes);
    double *stage = reinterpret_cast<double *>(ws + geo.amT_bytes + geo.partial_bytes);
    if (geo.rows == 0) return launch_reduce_partials(d.nw, nullptr, 0, nullptr, ach, asx, st);
    hipError_t e = hipSuccess;
    if (step <= 3) {
        switch (d.nw) {
        case 1: e = launch_collapse<1>(step, d, geo, in, partials, st); break;
        case 2: e = launch_collapse<2>(step, d, geo, in, partials, st); break;
        case 3: e = launch_collapse<3>(step, d, geo, in, partials, st); break;
        default: e = launch_collapse<4>(step, d, geo, in, partials, st); break;
        }
    } else if (step == 4) {
        switch (d.nw) {
        case 1: e = launch_bandinner_all<1>(d, geo, in, partials, st); break;
        case 2: e = launch_bandinner_all<2>(d, geo, in, partials, st); break;
        case 3: e = launch_bandinner_all<3>(d, geo, in, partials, st); break;
        default: e = launch_bandinner_all<4>(d, geo, in, partials, st); break;
        }
    } else if (step == 9 || step == 10) {
        const dim3 grid((unsigned)geo.rows), blk(kLadThreads);
        switch (d.nw * 2 + (step == 10)) {
        case 2: hipLaunchKernelGGL((lad_factored<1, false>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        case 3: hipLaunchKernelGGL((lad_factored<1, true>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        case 4: hipLaunchKernelGGL((lad_factored<2, false>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        case 5: hipLaunchKernelGGL((lad_factored<2, true>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        case 6: hipLaunchKernelGGL((lad_factored<3, false>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        case 7: hipLaunchKernelGGL((lad_factored<3, true>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        case 8: hipLaunchKernelGGL((lad_factored<4, false>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        default: hipLaunchKernelGGL((lad_factored<4, true>), grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, in, partials); break;
        }
        e = hipGetLastError();
    } else if (step == 5) {
        for (int w = 0; w < d.nw && e == hipSuccess; ++w) {
            hipLaunchKernelGGL((lad_bandinner<1, Div::Rcp, Pred::Square, Br::Two>),
                               dim3((unsigned)geo.rows), dim3(kLadThreads), 0, st, d.nb, d.nv,
                               d.ng, d.np, w, d.nw, in, partials);
            e = hipGetLastError();
        }
    } else {
        const int npb = (d.np + kLadWaves - 1) / kLadWaves;
        if (step >= 7) {
            const long n = (long)d.np * d.nb;
            hipLaunchKernelGGL(lad_transpose_am, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                               st, d.nb, d.ng, d.np, in.aqsm, amT);
            e = hipGetLastError();
        }
        for (int w = 0; w < d.nw && e == hipSuccess; ++w) {
            const dim3 grid((unsigned)geo.rows), blk(kLadThreads);
            if (step == 6)
                hipLaunchKernelGGL(lad_blocked<false>, grid, blk, 0, st, d.nb, d.nv, d.ng, d.np,
                                   w, d.nw, npb, in, amT, partials);
            else if (step == 7)
                hipLaunchKernelGGL(lad_blocked<true>, grid, blk, 0, st, d.nb, d.nv, d.ng, d.np, w,
                                   d.nw, npb, in, amT, partials);
            else
                hipLaunchKernelGGL(lad_blocked_capped, grid, blk, 0, st, d.nb, d.nv, d.ng, d.np,
                                   w, d.nw, npb, in, amT, partials);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    return launch_reduce_partials(d.nw, partials, geo.rows, stage, ach, asx, st);
}

}  // namespace
}  // namespace gpp

extern "C" {

int32_t gpp_ladder_steps(void) { return GPP_LADDER_STEPS; }

const char *gpp_ladder_name(int32_t step)
{
    return step >= 0 && step < GPP_LADDER_STEPS ? gpp::kNames[step] : nullptr;
}

size_t gpp_ladder_workspace(int32_t step, const gpp_dims *dims)
{
    gpp::Dims32 d;
    if (step < 0 || step >= GPP_LADDER_STEPS || gpp::check_dims(dims, &d) != GPP_OK) return 0;
    if (step == GPP_LADDER_STEPS - 1) return gpp_sigma_fwd_workspace(dims);
    if (d.nw > GPP_LADDER_MAX_NFREQ) return 0;
    return gpp::ladder_geometry(step, d).workspace_bytes;
}

gpp_status gpp_ladder_fwd(int32_t step, const gpp_dims *dims, const gpp_inputs *inputs,
                          double *achtemp, double *asxtemp, void *workspace,
                          size_t workspace_bytes, void *stream)
{
    gpp::g_last_error[0] = '\0';
    if (step < 0 || step >= GPP_LADDER_STEPS)
        return gpp::fail(GPP_ERR_INVALID, "ladder step %d outside [0, %d)", (int)step,
                         GPP_LADDER_STEPS);
    if (step == GPP_LADDER_STEPS - 1)
        return gpp_sigma_fwd(dims, inputs, achtemp, asxtemp, workspace, workspace_bytes, stream);
    gpp::Dims32 d;
    gpp::DevInputs din;
    gpp_status s;
    if ((s = gpp::check_dims(dims, &d))) return s;
    if (d.nw > GPP_LADDER_MAX_NFREQ)
        return gpp::fail(GPP_ERR_INVALID, "ladder steps 0-%d take nfreq <= %d, got %d",
                         GPP_LADDER_STEPS - 2, GPP_LADDER_MAX_NFREQ, d.nw);
    if ((s = gpp::check_inputs(d, inputs, &din))) return s;
    if ((s = gpp::check_array("achtemp", achtemp, d.nw, 16)) ||
        (s = gpp::check_array("asxtemp", asxtemp, d.nw, 16)))
        return s;
    const size_t need = gpp::ladder_geometry(step, d).workspace_bytes;
    if (!workspace || workspace_bytes < need)
        return gpp::fail(GPP_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu%s", need,
                         workspace_bytes, workspace ? "" : " (NULL)");
    if (gpp::misaligned(workspace, 16))
        return gpp::fail(GPP_ERR_INVALID, "workspace is not 16-byte aligned");
    if ((s = gpp::check_device("gpp_ladder_fwd"))) return s;
    hipError_t e = gpp::launch_ladder(step, d, din, reinterpret_cast<double2 *>(achtemp),
                                      reinterpret_cast<double2 *>(asxtemp),
                                      static_cast<char *>(workspace),
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return gpp::hip_fail(e, "gpp_ladder_fwd launch");
    return GPP_OK;
}

}  // extern "C"
