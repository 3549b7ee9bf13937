// gpp_fwd.hip -- forward GPP reduction on gfx950 (fp64 vector ALU, no MFMA).
//
// Work decomposition.  A wave owns two G' columns (one with more than three
// frequencies) and 64 consecutive G rows g (one per lane) and walks every
// band n sequentially, as in the band-inner loop order of Sec. III v4
// (bands serial per thread keeps the g-fastest arrays coalesced and reads
// wtilde/I_eps once); each aqsntemp[n][g] a lane loads serves both
// columns.  Within a wave p and n are uniform, so aqsmtemp[n][p] and
// wx_array[w][n] are scalar loads; the frequencies are register-blocked
// (all NW in one pass, none of v5's recompute).
//
// Per lane, e = I_eps[p][g] and vcoul[g] are constant over the band loop,
// so they multiply once at the end.  For a branch-A term,
//   om / (x - om) = (x om - |om|^2) / |x - om|^2 = r (x om - wtr),
// so with Qm = aqsntemp[n][g] conj(aqsmtemp[n][p]) the lane accumulates
//   P1[w] += (r x) Qm,  P2[w] += r Qm
// and ends with  achtemp += vcoul/2 * e * (om P1 - wtr P2).  The branch-A
// test is one compare against a per-(p,g) threshold that reproduces the
// specification exactly (gpp_device.h).  r = 1/wdiffr needs no IEEE divide
// (the v1 idea); the 2*BU*NW reciprocals of a group of BU bands and both
// columns come from a single hardware reciprocal by batch inversion
// (gpp_device.h: unclamped denominators, a lane test on (Im om)^2 for the
// product's range), and the branch-A test is the execution mask around
// each term's four fused multiply-adds, so a masked term adds nothing and
// costs no select.  Occupied bands (n < nvband) also evaluate the
// screened-exchange term, from batch-inverted |x - om|^2 and |x + om|^2
// instead of a complex divide (gpp_fwd_tile.h).  Above 512 bands each
// tile's band loop is split into chunks, each a tile of its own.
//
// Each workgroup (4 waves) writes one partial per output into the
// workspace; two reduction kernels then sum the partials in a fixed order
// (the separate reduction kernel of Sec. II-A), so results are bitwise
// reproducible.
#include "gpp_device.h"
#include "gpp_fwd_tile.h"
#include "gpp_internal.h"

namespace gpp {

constexpr int kFwdWaves = 4;
constexpr int kFwdThreads = kFwdWaves * kWave;
// G' columns per wave tile and bands per batch-inverted group (K = columns
// x bands x nfreq reciprocals from one hardware reciprocal) come from
// fwd_cols and fwd_bands, and a cap on VGPRs through a minimum number of
// waves per SIMD from fwd_min_waves (gpp_internal.h), all chosen by
// measurement on MI355X.  At nfreq 3, two columns per wave let each
// aqsntemp load serve both: 153 VGPRs when measured, 156 with the
// divide-free exchange term (3 waves per SIMD either way) with 2-band
// groups, 2.8-3.1 % faster than one column with 3-band groups (105 VGPRs,
// 4 waves); three columns need about 200 VGPRs (2 waves) and measured
// 3-30 % slower.
constexpr int kRedThreads = 256;
constexpr long kRedBlocks = 512;  // first reduction stage

template <int NW, int BU>
__global__ void __launch_bounds__(kFwdThreads)
__attribute__((amdgpu_waves_per_eu(fwd_min_waves(NW))))
fwd_tiles(int nb, int nv, int ng, int np, long ntiles, int nchunk, int chunk_bands,
          const double2 *__restrict__ aqsm, const double2 *__restrict__ aqsn,
          const double2 *__restrict__ ieps, const double2 *__restrict__ wt,
          const double *__restrict__ vcoul, const double *__restrict__ wx,
          double *__restrict__ partials)
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
        constexpr int C = fwd_cols(NW);
        const int npt = (np + C - 1) / C;  // column tiles per g-tile
        int gt, pt, ck;
        tile_coords(tile, npt, (ng + kWave - 1) / kWave, nchunk, gt, pt, ck);
        const int n_lo = ck * chunk_bands;
        const int n_hi = nb - n_lo < chunk_bands ? nb : n_lo + chunk_bands;
        if (C == 1) {
            fwd_tile_body<NW, BU>(nb, nv, n_lo, n_hi, ng, pt, gt, lane, as_global(aqsm),
                                  as_global(aqsn), as_global(ieps), as_global(wt),
                                  as_global(vcoul), as_global(wx), ach, asx);
        } else {
            fwd_tile_body_cols<NW, BU, C>(nb, nv, n_lo, n_hi, ng, np, C * pt, gt, lane,
                                          as_global(aqsm), as_global(aqsn), as_global(ieps),
                                          as_global(wt), as_global(vcoul), as_global(wx), ach,
                                          asx);
        }
    }

    // wave then workgroup reduction in a fixed order; partial row layout
    // [4 w + 0..3] = achtemp[w].re, .im, asxtemp[w].re, .im
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        // asx[] already holds wave totals (or zeros)
        const double v0 = wave_sum(ach[w].re), v1 = wave_sum(ach[w].im);
        const double v2 = asx[w].re, v3 = asx[w].im;
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
        partials[(size_t)blockIdx.x * 4 * NW + threadIdx.x] = s;
    }
}

// Quasiparticle quantities from the final sums fin[4 w + 0..3] = achtemp[w]
// re, im, asxtemp[w] re, im, for nfreq odd and at least 3 (the caller
// checks): Sigma(E_w) = achtemp[w] - asxtemp[w] (asxtemp is the unsigned
// exchange sum), dSigma/dE at the middle frequency m by the central
// difference of its neighbours, Z = 1/(1 - Re dSigma/dE) and the linearised
// quasiparticle energy E + Z (Re Sigma(E) - V_xc).  out = Sigma re, im,
// dSigma/dE re, im, Z, E_qp.
template <int NW>
__device__ inline void qp_epilogue(const double *fin, const QpArgs &qp)
{
    if constexpr (NW >= 3 && NW % 2 == 1) {
        constexpr int m = (NW - 1) / 2;
        const double sr = fin[4 * m] - fin[4 * m + 2], si = fin[4 * m + 1] - fin[4 * m + 3];
        const double hi_r = fin[4 * (m + 1)] - fin[4 * (m + 1) + 2];
        const double hi_i = fin[4 * (m + 1) + 1] - fin[4 * (m + 1) + 3];
        const double lo_r = fin[4 * (m - 1)] - fin[4 * (m - 1) + 2];
        const double lo_i = fin[4 * (m - 1) + 1] - fin[4 * (m - 1) + 3];
        const double span = 2.0 * qp.step;
        const double dr = (hi_r - lo_r) / span, di = (hi_i - lo_i) / span;
        const double z = 1.0 / (1.0 - dr);
        qp.out[0] = sr;
        qp.out[1] = si;
        qp.out[2] = dr;
        qp.out[3] = di;
        qp.out[4] = z;
        qp.out[5] = qp.energy + z * (sr - qp.vxc);
    }
}

// Sum rows of W doubles: block b takes rows [b*chunk, (b+1)*chunk), thread
// t rows t, t+256, ... of it (coalesced: neighbouring threads read
// neighbouring rows), then a fixed wave/workgroup tree.  With final set,
// writes the result as achtemp/asxtemp instead of a row, and with qp.out
// set also the quasiparticle quantities (qp_epilogue).
template <int NW>
__global__ void __launch_bounds__(kRedThreads)
reduce_rows(const double *__restrict__ in, long nrows, long chunk, double *__restrict__ out,
            double2 *__restrict__ ach, double2 *__restrict__ asx, int final_stage, QpArgs qp)
{
    constexpr int W = 4 * NW;
    __shared__ double red[kRedThreads / kWave][W];
    __shared__ double fin[W];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const long lo = (long)blockIdx.x * chunk;
    const long hi = lo + chunk < nrows ? lo + chunk : nrows;
    double acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = 0.0;
    for (long i = lo + threadIdx.x; i < hi; i += kRedThreads) {
        const double *row = in + (size_t)i * W;
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] += row[j];
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) red[wid][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < W) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kRedThreads / kWave; ++k) s += red[k][threadIdx.x];
        if (!final_stage) {
            out[(size_t)blockIdx.x * W + threadIdx.x] = s;
        } else {
            const int w = threadIdx.x / 4, c = threadIdx.x % 4;
            double *dst = reinterpret_cast<double *>(c < 2 ? ach + w : asx + w);
            dst[c & 1] = s;
            fin[threadIdx.x] = s;
        }
    }
    if (final_stage && qp.out) {  // uniform: kernel arguments
        __syncthreads();
        if (threadIdx.x == 0) qp_epilogue<NW>(fin, qp);
    }
}

// Zero outputs of an empty sum (and its quasiparticle quantities: Sigma = 0,
// Z = 1, E_qp = E - V_xc).
template <int NW>
__global__ void fill_zero(double2 *a, double2 *b, QpArgs qp)
{
    __shared__ double fin[4 * NW];
    int i = threadIdx.x;
    if (i < NW) {
        a[i] = make_double2(0.0, 0.0);
        b[i] = make_double2(0.0, 0.0);
    }
    if (i < 4 * NW) fin[i] = 0.0;
    if (qp.out) {
        __syncthreads();
        if (i == 0) qp_epilogue<NW>(fin, qp);
    }
}

static hipError_t launch_fill_zero(int nw, double2 *a, double2 *b, const QpArgs &qp,
                                   hipStream_t st)
{
    switch (nw) {
#define GPP_Z(N)                                                                      \
    case N: hipLaunchKernelGGL(fill_zero<N>, dim3(1), dim3(64), 0, st, a, b, qp); break;
        GPP_Z(1) GPP_Z(2) GPP_Z(3) GPP_Z(4) GPP_Z(5) GPP_Z(6) GPP_Z(7) GPP_Z(8)
#undef GPP_Z
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

FwdGeometry fwd_geometry(const Dims32 &d)
{
    FwdGeometry geo{};
    if (d.nb == 0 || d.ng == 0 || d.np == 0) return geo;
    const long gtiles = (d.ng + kWave - 1) / kWave;
    const int cols = fwd_cols(d.nw);
    fwd_band_chunks(d.nb, d.nw, geo.nchunk, geo.chunk_bands);
    geo.ntiles = gtiles * ((d.np + cols - 1) / cols) * geo.nchunk;
    geo.nblocks = (geo.ntiles + kFwdWaves - 1) / kFwdWaves;
    geo.red_blocks = geo.nblocks < kRedBlocks ? geo.nblocks : kRedBlocks;
    geo.red_chunk = (geo.nblocks + geo.red_blocks - 1) / geo.red_blocks;
    const size_t row = 4 * sizeof(double) * d.nw;
    geo.partial_bytes = (size_t)geo.nblocks * row;
    geo.stage_bytes = (size_t)geo.red_blocks * row;
    geo.workspace_bytes = geo.partial_bytes + geo.stage_bytes;
    return geo;
}

template <int NW>
static hipError_t launch_fwd_nw(const Dims32 &d, const FwdGeometry &geo, const DevInputs &in,
                                double2 *ach, double2 *asx, double *ws, hipStream_t st,
                                const QpArgs &qp)
{
    double *partials = ws;
    double *stage = ws + (size_t)geo.nblocks * 4 * NW;
    constexpr int BU = fwd_bands(NW);
    hipLaunchKernelGGL((fwd_tiles<NW, BU>), dim3((unsigned)geo.nblocks),
                       dim3(kFwdThreads), 0, st, d.nb, d.nv, d.ng, d.np, geo.ntiles, geo.nchunk,
                       geo.chunk_bands, in.aqsm, in.aqsn, in.ieps, in.wt, in.vcoul, in.wx,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_rows<NW>, dim3((unsigned)geo.red_blocks), dim3(kRedThreads), 0,
                       st, partials, geo.nblocks, geo.red_chunk, stage, ach, asx, 0, QpArgs());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_rows<NW>, dim3(1), dim3(kRedThreads), 0, st, stage,
                       geo.red_blocks, geo.red_blocks, nullptr, ach, asx, 1, qp);
    return hipGetLastError();
}

size_t reduce_stage_bytes(int nw, long nrows)
{
    const long blocks = nrows < kRedBlocks ? nrows : kRedBlocks;
    return (size_t)blocks * 4 * sizeof(double) * nw;
}

template <int NW>
static hipError_t launch_reduce_nw(const double *partials, long nrows, double *stage,
                                   double2 *ach, double2 *asx, hipStream_t st)
{
    const long blocks = nrows < kRedBlocks ? nrows : kRedBlocks;
    const long chunk = (nrows + blocks - 1) / blocks;
    hipLaunchKernelGGL(reduce_rows<NW>, dim3((unsigned)blocks), dim3(kRedThreads), 0, st,
                       partials, nrows, chunk, stage, ach, asx, 0, QpArgs());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_rows<NW>, dim3(1), dim3(kRedThreads), 0, st, stage, blocks,
                       blocks, nullptr, ach, asx, 1, QpArgs());
    return hipGetLastError();
}

hipError_t launch_reduce_partials(int nw, const double *partials, long nrows, double *stage,
                                  double2 *ach, double2 *asx, hipStream_t st)
{
    if (nrows <= 0) return launch_fill_zero(nw, ach, asx, QpArgs(), st);
    switch (nw) {
    case 1: return launch_reduce_nw<1>(partials, nrows, stage, ach, asx, st);
    case 2: return launch_reduce_nw<2>(partials, nrows, stage, ach, asx, st);
    case 3: return launch_reduce_nw<3>(partials, nrows, stage, ach, asx, st);
    case 4: return launch_reduce_nw<4>(partials, nrows, stage, ach, asx, st);
    case 5: return launch_reduce_nw<5>(partials, nrows, stage, ach, asx, st);
    case 6: return launch_reduce_nw<6>(partials, nrows, stage, ach, asx, st);
    case 7: return launch_reduce_nw<7>(partials, nrows, stage, ach, asx, st);
    case 8: return launch_reduce_nw<8>(partials, nrows, stage, ach, asx, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fwd(const Dims32 &d, const DevInputs &in, double2 *ach, double2 *asx,
                      void *workspace, hipStream_t st, const QpArgs &qp)
{
    const FwdGeometry geo = fwd_geometry(d);
    if (geo.nblocks == 0) return launch_fill_zero(d.nw, ach, asx, qp, st);
    double *ws = static_cast<double *>(workspace);
    switch (d.nw) {
    case 1: return launch_fwd_nw<1>(d, geo, in, ach, asx, ws, st, qp);
    case 2: return launch_fwd_nw<2>(d, geo, in, ach, asx, ws, st, qp);
    case 3: return launch_fwd_nw<3>(d, geo, in, ach, asx, ws, st, qp);
    case 4: return launch_fwd_nw<4>(d, geo, in, ach, asx, ws, st, qp);
    case 5: return launch_fwd_nw<5>(d, geo, in, ach, asx, ws, st, qp);
    case 6: return launch_fwd_nw<6>(d, geo, in, ach, asx, ws, st, qp);
    case 7: return launch_fwd_nw<7>(d, geo, in, ach, asx, ws, st, qp);
    case 8: return launch_fwd_nw<8>(d, geo, in, ach, asx, ws, st, qp);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace gpp
