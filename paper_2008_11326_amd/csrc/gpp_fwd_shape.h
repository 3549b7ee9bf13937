// gpp_fwd_shape.h -- tile shape of the forward tile kernels per frequency
// count, shared by the plain forward, the batched flat grid and the
// batched plan's tile counts (host and device code).
#pragma once

namespace gpp {

// G' columns per wave tile, and bands per batch-inverted group, so that a group holds
// columns x bands x nfreq <= 12 denominators.  More columns let each
// aqsntemp load serve more terms; the accumulators (columns x nfreq x 4
// doubles) bound how many fit.  Pairs (columns, bands) for nfreq = 1..8;
// nfreq 3 takes GPP_FWD_COLS x GPP_FWD_BANDS.  Measured on MI355X at 512
// bands, 32768 rows, 1638 columns (best of 3 alternating rounds): nfreq 2
// with three columns 2 % faster than with two; nfreq 5 and 6 with 2-band
// groups 20 % and 15 % faster than 1-band ones; nfreq 1 with 2 x 2 faster
// than 2 x 6, 3 x 4, 4 x 3 or 6 x 2; nfreq 4 with 1 x 2 faster than 1 x 3
// or 2 x 1.
#ifndef GPP_FWD_COLS
#define GPP_FWD_COLS 2
#endif
#ifndef GPP_FWD_BANDS
#define GPP_FWD_BANDS 2
#endif
#ifndef GPP_FWD_SHAPE
#define GPP_FWD_SHAPE 2, 2, 3, 2, GPP_FWD_COLS, GPP_FWD_BANDS, 1, 2, 1, 2, 1, 2, 1, 1, 1, 1
#endif
constexpr int kFwdShape[16] = {GPP_FWD_SHAPE};
constexpr int fwd_cols(int nw) { return kFwdShape[2 * (nw - 1)]; }
constexpr int fwd_bands(int nw) { return kFwdShape[2 * (nw - 1) + 1]; }
constexpr bool fwd_shapes_fit()
{
    for (int nw = 1; nw <= 8; ++nw)
        if (fwd_cols(nw) < 1 || fwd_bands(nw) < 1 || fwd_cols(nw) * fwd_bands(nw) * nw > 12)
            return false;
    return true;
}
static_assert(fwd_shapes_fit(), "a forward tile's batch inversion holds at most 12 denominators");
// Minimum waves per SIMD (a VGPR cap) of the forward tile kernels for
// nfreq = 1..8, measured at 512 bands, 32768 rows, 1638 columns (best of 3
// alternating rounds): nfreq 4 capped at 96 VGPRs (5 waves) 1.5 % faster
// than at 103 (4); nfreq 7 and 8 capped at 128 (4 waves; 2 and 24 bytes of
// spills) 9.5 % and 5.1 % faster than at 130 and 144 (3).  nfreq 1 capped
// for 6 waves and nfreq 6 for 4 ran 0.9 % and 16 % slower.
#ifndef GPP_FWD_MIN_WAVES
#define GPP_FWD_MIN_WAVES 1, 1, 1, 5, 1, 1, 4, 4
#endif
constexpr int kFwdMinWaves[8] = {GPP_FWD_MIN_WAVES};
constexpr int fwd_min_waves(int nw) { return kFwdMinWaves[nw - 1]; }

// Band chunks of the plain forward's tiles.  The waves an XCD holds at
// once start and end together, so a value one tile reads comes back to the
// next tiles only after a whole tile's band loop of other traffic (about
// 8 KB per band for the resident tiles of one XCD); splitting the band
// loop into chunks of at most GPP_FWD_CHUNK_BANDS bands keeps that inside
// the XCD's 4 MB L2.  Every chunk of a tile adds its own partial sums (the
// sums are linear in the bands), so chunks cost their own set-up, exchange
// sums and partial row.  0 turns chunking off.  Chunks hold whole band
// groups except the last.
#ifndef GPP_FWD_CHUNK_BANDS
#define GPP_FWD_CHUNK_BANDS 512
#endif
inline void fwd_band_chunks(int nb, int nw, int &nchunk, int &chunk_bands)
{
    nchunk = 1;
    chunk_bands = nb;
    if (GPP_FWD_CHUNK_BANDS <= 0 || nb <= GPP_FWD_CHUNK_BANDS) return;
    const int bu = fwd_bands(nw);
    const int want = (nb + GPP_FWD_CHUNK_BANDS - 1) / GPP_FWD_CHUNK_BANDS;
    int cb = (nb + want - 1) / want;
    cb = (cb + bu - 1) / bu * bu;
    chunk_bands = cb;
    nchunk = (nb + cb - 1) / cb;
}

}  // namespace gpp
