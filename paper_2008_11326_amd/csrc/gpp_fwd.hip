// gpp_fwd.hip -- forward GPP reduction on gfx950 (fp64 vector ALU, no MFMA).
//
// Work decomposition.  A wave owns one G' column p and 64 consecutive G
// rows g (one per lane) and walks every band n sequentially, as in the
// band-inner loop order of Sec. III v4 (bands serial per thread keeps the
// g-fastest arrays coalesced and reads wtilde/I_eps once).  Within a wave
// p and n are uniform, so aqsmtemp[n][p] and wx_array[w][n] are scalar
// loads; the frequencies are register-blocked (all NW in one pass, no
// redundant recompute as in v5).
//
// Per lane, e = I_eps[p][g] and vcoul[g] are constant over the band loop,
// so they multiply once at the end.  For a branch-A term,
//   om / (x - om) = (x om - |om|^2) / |x - om|^2 = r (x om - wtr),
// so with Qm = aqsntemp[n][g] conj(aqsmtemp[n][p]) the lane accumulates
//   P1[w] += (r x) Qm,  P2[w] += r Qm
// and ends with  achtemp += vcoul/2 * e * (om P1 - wtr P2).  The branch-A
// test is a single compare against a per-(p,g) threshold that reproduces
// the specification exactly (gpp_device.h); r = 1/wdiffr is a hardware
// reciprocal plus two Newton steps (the v1 idea: no IEEE divide), and
// masked terms select r = 0.  Occupied bands (n < nvband) also evaluate the
// screened-exchange term with full complex arithmetic.
//
// Each workgroup (4 waves) writes one partial per output; a second kernel
// sums the partials in a fixed order (the separate reduction kernel of
// Sec. II-A), so results are bitwise reproducible.
#include "gpp_device.h"
#include "gpp_internal.h"

namespace gpp {

constexpr int kFwdWaves = 4;
constexpr int kFwdThreads = kFwdWaves * kWave;

template <int NW>
__global__ void __launch_bounds__(kFwdThreads)
fwd_tiles(int nb, int nv, int ng, int np, long ntiles,
          const double2 *__restrict__ aqsm, const double2 *__restrict__ aqsn,
          const double2 *__restrict__ ieps, const double2 *__restrict__ wt,
          const double *__restrict__ vcoul, const double *__restrict__ wx,
          double2 *__restrict__ partials)
{
    __shared__ double red[kFwdWaves][4 * NW];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const long tile = (long)xcd_remap(blockIdx.x, gridDim.x) * kFwdWaves + wid;

    cplx ach[NW], asx[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) ach[w] = asx[w] = cmake(0.0, 0.0);

    if (tile < ntiles) {
        // consecutive tiles share a g-tile (and so the same aqsntemp rows)
        const int gt = (int)(tile / np);
        const int p = (int)(tile - (long)gt * np);
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

        const double2 *an_col = aqsn + gc;
        const double2 *am_col = aqsm + p;

        // occupied bands: exchange (SX) and Coulomb-hole (CH) terms
        for (int n = 0; n < nv; ++n) {
            const cplx an = cload(an_col + (size_t)n * ng);
            const cplx am = cload(am_col + (size_t)n * ng);
            const cplx qm = cmul_conj(an, am);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const double x = wx[(size_t)w * nb + n];
                const double dr = x - a;
                const double wd = fma(dr, dr, wi2);
                const bool isA = wd > thr;
                const double r = isA ? rcp_nr2(wd) : 0.0;
                const double rx = r * x;
                P1[w].re = fma(rx, qm.re, P1[w].re);
                P1[w].im = fma(rx, qm.im, P1[w].im);
                P2[w].re = fma(r, qm.re, P2[w].re);
                P2[w].im = fma(r, qm.im, P2[w].im);
                // ssx / e
                const cplx d = cmake(dr, -b);     // x - om
                const cplx s = cmake(x + a, b);   // x + om
                cplx t = cmake(0.0, 0.0);
                if (isA) {
                    t = cdiv(cmul(om, om), cmul(d, s));
                } else if (branch_b_holds(wtr, wd)) {
                    t = cdiv(om, cmake(-2.0 * s.re, -2.0 * s.im));
                }
                cmac(SX[w], qm, t);
            }
        }
        // unoccupied bands: CH only -- the hot loop
#pragma unroll 2
        for (int n = nv; n < nb; ++n) {
            const cplx an = cload(an_col + (size_t)n * ng);
            const cplx am = cload(am_col + (size_t)n * ng);
            const cplx qm = cmul_conj(an, am);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const double x = wx[(size_t)w * nb + n];
                const double dr = x - a;
                const double wd = fma(dr, dr, wi2);
                const double rr = rcp_nr2(wd);
                const double r = wd > thr ? rr : 0.0;
                const double rx = r * x;
                P1[w].re = fma(rx, qm.re, P1[w].re);
                P1[w].im = fma(rx, qm.im, P1[w].im);
                P2[w].re = fma(r, qm.re, P2[w].re);
                P2[w].im = fma(r, qm.im, P2[w].im);
            }
        }

        const cplx e = cload(ieps + (size_t)p * ng + gc);
        const double v = valid ? vcoul[gc] : 0.0;
        const cplx ev = cscale(v, e);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            // S = om P1 - wtr P2
            cplx S = cmul(om, P1[w]);
            S.re = fma(-wtr, P2[w].re, S.re);
            S.im = fma(-wtr, P2[w].im, S.im);
            ach[w] = cscale(0.5, cmul(ev, S));
            asx[w] = cmul(ev, SX[w]);
        }
    }

    // wave then workgroup reduction in a fixed order
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        double v0 = wave_sum(ach[w].re), v1 = wave_sum(ach[w].im);
        double v2 = wave_sum(asx[w].re), v3 = wave_sum(asx[w].im);
        if (lane == 0) {
            red[wid][4 * w + 0] = v0;
            red[wid][4 * w + 1] = v1;
            red[wid][4 * w + 2] = v2;
            red[wid][4 * w + 3] = v3;
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 * NW) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kFwdWaves; ++k) s += red[k][threadIdx.x];
        // partial layout: [block][2 * NW] complex; slot w = achtemp[w],
        // slot NW + w = asxtemp[w]
        const int w = threadIdx.x / 4, c = threadIdx.x % 4;
        const int slot = (c < 2) ? w : NW + w;
        double *dst = reinterpret_cast<double *>(partials + (size_t)blockIdx.x * 2 * NW + slot);
        dst[c & 1] = s;
    }
}

// Sum `nparts` partials of 2*nw complex slots in a fixed order: thread t
// takes parts t, t+256, ... in increasing order, then a fixed tree.
__global__ void __launch_bounds__(256)
reduce_partials(const double2 *__restrict__ partials, long nparts, int nslots,
                double2 *__restrict__ out_a, double2 *__restrict__ out_b, int nw)
{
    __shared__ double sre[256], sim[256];
    for (int k = 0; k < nslots; ++k) {
        double re = 0.0, im = 0.0;
        for (long i = threadIdx.x; i < nparts; i += 256) {
            double2 v = partials[(size_t)i * nslots + k];
            re += v.x;
            im += v.y;
        }
        sre[threadIdx.x] = re;
        sim[threadIdx.x] = im;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                sre[threadIdx.x] += sre[threadIdx.x + h];
                sim[threadIdx.x] += sim[threadIdx.x + h];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double2 r = make_double2(sre[0], sim[0]);
            if (k < nw) out_a[k] = r; else out_b[k - nw] = r;
        }
        __syncthreads();
    }
}

__global__ void fill_zero(double2 *a, double2 *b, int nw)
{
    int i = threadIdx.x;
    if (i < nw) {
        a[i] = make_double2(0.0, 0.0);
        b[i] = make_double2(0.0, 0.0);
    }
}

FwdGeometry fwd_geometry(const Dims32 &d)
{
    FwdGeometry geo{};
    if (d.nb == 0 || d.ng == 0 || d.np == 0) return geo;
    const long gtiles = (d.ng + kWave - 1) / kWave;
    geo.ntiles = gtiles * d.np;
    geo.nblocks = (geo.ntiles + kFwdWaves - 1) / kFwdWaves;
    geo.partial_bytes = (size_t)geo.nblocks * 2 * d.nw * sizeof(double2);
    return geo;
}

template <int NW>
static void launch_fwd_nw(const Dims32 &d, const FwdGeometry &geo, const DevInputs &in,
                          double2 *partials, hipStream_t st)
{
    hipLaunchKernelGGL(fwd_tiles<NW>, dim3((unsigned)geo.nblocks), dim3(kFwdThreads), 0, st,
                       d.nb, d.nv, d.ng, d.np, geo.ntiles, in.aqsm, in.aqsn, in.ieps,
                       in.wt, in.vcoul, in.wx, partials);
}

hipError_t launch_fwd(const Dims32 &d, const DevInputs &in, double2 *ach, double2 *asx,
                      void *workspace, hipStream_t st)
{
    const FwdGeometry geo = fwd_geometry(d);
    if (geo.nblocks == 0) {
        hipLaunchKernelGGL(fill_zero, dim3(1), dim3(64), 0, st, ach, asx, d.nw);
        return hipGetLastError();
    }
    double2 *partials = static_cast<double2 *>(workspace);
    switch (d.nw) {
    case 1: launch_fwd_nw<1>(d, geo, in, partials, st); break;
    case 2: launch_fwd_nw<2>(d, geo, in, partials, st); break;
    case 3: launch_fwd_nw<3>(d, geo, in, partials, st); break;
    case 4: launch_fwd_nw<4>(d, geo, in, partials, st); break;
    case 5: launch_fwd_nw<5>(d, geo, in, partials, st); break;
    case 6: launch_fwd_nw<6>(d, geo, in, partials, st); break;
    case 7: launch_fwd_nw<7>(d, geo, in, partials, st); break;
    case 8: launch_fwd_nw<8>(d, geo, in, partials, st); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(256), 0, st, partials, geo.nblocks,
                       2 * d.nw, ach, asx, d.nw);
    return hipGetLastError();
}

}  // namespace gpp
