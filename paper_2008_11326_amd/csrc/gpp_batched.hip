// gpp_batched.hip -- persistent forward over many quasiparticle states of
// uneven sizes in one launch (gfx950, fp64).
//
// The tiles of all states (each state's forward tiles: one or two G'
// columns x 64 G rows, G'-column fastest) are concatenated in a schedule order chosen by
// the plan.  Two kernel forms exist: the static one below and a work-queue
// one (batched_queue) whose waves take small chunks of the list from atomic
// counters.  In the static form, persistent wave w takes global tiles
// w, w + W, w + 2W, ...
// (W = resident waves), so at any moment the running waves sit on
// neighbouring tiles of one state -- the same aqsntemp rows and L2
// locality as the plain forward -- and every wave's cost stays within one
// tile of the mean (or, in the XCD-chunked schedule, each XCD takes one
// contiguous, equally costly chunk of the list and its waves round-robin
// inside it).  Each wave keeps running sums for the state it is in and
// writes one partial row for each state it touches, at a slot fixed by
// where its first tile of the state lies (static_slot); a second kernel adds
// each state's rows in a fixed order.  The rows of a state are thus at most
// min(W, its tiles) per XCD range it meets, so the workspace grows with the
// tile count, not with states x waves.  Waves never wait on each other, so
// the grid needs no co-residency and every wave reaches its exit.  The
// per-tile arithmetic is the plain forward's (gpp_fwd_tile.h).
#include "gpp_device.h"
#include "gpp_fwd_tile.h"
#include "gpp_internal.h"

namespace gpp {

#ifndef GPP_BAT_FLAT_RUN
#define GPP_BAT_FLAT_RUN 16
#endif
constexpr int kBatWaves = 4;
constexpr long kFlatRun = GPP_BAT_FLAT_RUN;  // flat form: consecutive workgroups per XCD
constexpr int kBatThreads = kBatWaves * kWave;

// Partial-row slot of a static-schedule wave for schedule position s, whose
// tiles are [b, e) = [st[s].tile_begin, st[s+1].tile_begin).  The waves that
// walk a range of tiles with stride W (all waves over the whole list, or one
// XCD's waves over its chunk [xc[x], xc[x+1])) meet min(W, L) of the state's
// L tiles in that range first, each at a different offset below min(W, L)
// from the range's first tile of the state; that offset numbers the wave's
// row.  The state's rows start at st[s].chunk_begin and take the ranges of
// lower XCDs first, so they fill [chunk_begin[s], chunk_begin[s+1]) exactly
// (the plan computes the same counts).  xc == nullptr: one range.
__device__ __forceinline__ long static_slot(const StateDesc *__restrict__ st, int s, long first,
                                            const long *__restrict__ xc, int xcd, uint32_t per,
                                            uint32_t rem)
{
    const long b = st[s].tile_begin, e = st[s + 1].tile_begin;
    long slot = st[s].chunk_begin, f = b;
    if (xc) {
        for (int x = 0; x < xcd; ++x) {
            const long lo = xc[x] > b ? xc[x] : b, hi = xc[x + 1] < e ? xc[x + 1] : e;
            const long wx = (long)(per + ((uint32_t)x < rem ? 1 : 0)) * 4;
            if (hi > lo) slot += hi - lo < wx ? hi - lo : wx;
        }
        if (xc[xcd] > f) f = xc[xcd];
    }
    return slot + (first - f);
}

// The schedule position k in [lo, nstates) of the state holding item v of
// the list (a tile, or a queue chunk when CHUNK), given that state lo starts
// at or before v: the last k with start(k) <= v, so empty states are never
// returned.  st[nstates] is the sentinel holding the total, which v is below.
template <bool CHUNK>
__device__ __forceinline__ int find_state(const StateDesc *__restrict__ st, int lo, int nstates,
                                          long v)
{
    int hi = nstates;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((CHUNK ? st[mid].chunk_begin : st[mid].tile_begin) <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Write the wave's running sums (wave-uniform values) into partial row
// `slot` and clear them.
template <int NW>
__device__ __forceinline__ void flush_state(long slot, int lane, cplx (&ach)[NW], cplx (&asx)[NW],
                                            double *__restrict__ partials)
{
    if (lane == 0) {
        double *dst = partials + (size_t)slot * (4 * NW);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            dst[4 * w + 0] = ach[w].re;
            dst[4 * w + 1] = ach[w].im;
            dst[4 * w + 2] = asx[w].re;
            dst[4 * w + 3] = asx[w].im;
        }
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) ach[w] = asx[w] = cmake(0.0, 0.0);
}

// The forward work of one tile of state d (its local tile index), as in
// the plain forward: one or two G' columns x 64 G rows.
template <int NW, int BU>
__device__ __forceinline__ void state_tile(const StateDesc &d, long local, int lane,
                                           cplx (&a)[NW], cplx (&x)[NW])
{
    constexpr int C = bat_cols(NW);
    const int npt = (d.np + C - 1) / C;
    const int gt = (int)(local / npt);
    const int pt = (int)(local - (long)gt * npt);
    if (C == 1) {
        fwd_tile_body<NW, BU>(d.nb, d.nv, 0, d.nb, d.ng, pt, gt, lane, as_global(d.aqsm),
                              as_global(d.aqsn), as_global(d.ieps), as_global(d.wt),
                              as_global(d.vcoul), as_global(d.wx), a, x);
    } else {
        fwd_tile_body_cols<NW, BU, C>(d.nb, d.nv, 0, d.nb, d.ng, d.np, C * pt, gt, lane,
                                      as_global(d.aqsm), as_global(d.aqsn), as_global(d.ieps),
                                      as_global(d.wt), as_global(d.vcoul), as_global(d.wx), a,
                                      x);
    }
}

// Register caps: two-column tiles (up to three frequencies) at 3 waves per
// SIMD, one-column tiles with four or more frequencies uncapped.
template <int NW, int BU>
__global__ void __launch_bounds__(kBatThreads)
__attribute__((amdgpu_waves_per_eu(bat_cols(NW) == 2 ? GPP_BAT_WAVES2 : (NW <= 3 ? 4 : 1))))
batched_persistent(const StateDesc *__restrict__ st, int nstates, long total_tiles, int nwaves,
                   double *__restrict__ partials, const long *__restrict__ xcd_chunks)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int wave = (int)xcd_remap(blockIdx.x, gridDim.x) * kBatWaves + wid;
    if (wave >= nwaves) return;  // wave-uniform; no barriers in this kernel

    // Tile sequence of this wave: t0, t0 + step, ... below t_end.  Global
    // round-robin, or (xcd_chunks != NULL) round-robin among the waves of
    // this wave's XCD over that XCD's contiguous chunk of the tile list, so
    // one XCD's L2 serves each g-tile as in the plain forward.
    long t0 = wave, step = nwaves, t_end = total_tiles;
    const uint32_t kXcd = kXcdCount, per = gridDim.x / kXcd, rem = gridDim.x % kXcd;
    const int xcd = (int)(blockIdx.x % kXcd);
    if (xcd_chunks) {
        const uint32_t x = (uint32_t)xcd, i = blockIdx.x / kXcd;
        const long waves_x = (long)(per + (x < rem ? 1 : 0)) * kBatWaves;
        t0 = xcd_chunks[x] + (long)i * kBatWaves + wid;
        step = waves_x;
        t_end = xcd_chunks[x + 1];
    }

    // running sums of the current state, kept wave-uniform (scalar
    // registers): each tile's contribution is summed over the wave as soon
    // as the tile is done, so no vector registers live across tiles
    cplx ach[NW], asx[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) ach[w] = asx[w] = cmake(0.0, 0.0);

    int s = 0;        // schedule position of the state holding tile t
    long first = -1;  // the wave's first tile of state s (-1: none yet)
    for (long t = t0; t < t_end; t += step) {
        if (t >= st[s + 1].tile_begin) {  // st[nstates].tile_begin == total_tiles
            if (first >= 0)
                flush_state<NW>(static_slot(st, s, first, xcd_chunks, xcd, per, rem), lane, ach,
                                asx, partials);
            first = -1;
            // the states in between hold none of this wave's tiles
            s = find_state<false>(st, s + 1, nstates, t);
        }
        if (first < 0) first = t;
        const StateDesc d = st[s];
        cplx a[NW], x[NW];
        state_tile<NW, BU>(d, t - d.tile_begin, lane, a, x);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            ach[w].re = to_uniform(ach[w].re + wave_sum(a[w].re));
            ach[w].im = to_uniform(ach[w].im + wave_sum(a[w].im));
            asx[w].re = to_uniform(asx[w].re + x[w].re);  // x: already wave totals
            asx[w].im = to_uniform(asx[w].im + x[w].im);
        }
    }
    if (first >= 0)
        flush_state<NW>(static_slot(st, s, first, xcd_chunks, xcd, per, rem), lane, ach, asx,
                        partials);
}

// Work-queue form: waves take chunks of chunk_tiles consecutive tiles (never
// crossing a state) from a global counter in increasing order, so the
// chunks in flight stay a contiguous window of the tile list and faster
// CUs take more chunks.  Each chunk writes its own partial row, which makes
// the result independent of which wave ran which chunk.
// With queue_begin != NULL there are kXcdCount queues: queue x hands out
// chunks [queue_begin[x], queue_begin[x+1]) (an equal-cost contiguous region
// of the chunk list) through counter[x]; waves start on their own XCD's
// queue (workgroups reach XCDs round-robin), keeping one XCD's L2 on one
// region, and move on to the other queues once theirs is empty.  Each queue
// is left for good when it runs dry, so a wave makes at most kXcdCount
// failed takes and every wave reaches the exit.
template <int NW, int BU>
__global__ void __launch_bounds__(kBatThreads)
__attribute__((amdgpu_waves_per_eu(bat_cols(NW) == 2 ? GPP_BAT_WAVES2 : (NW <= 3 ? 4 : 1))))
batched_queue(const StateDesc *__restrict__ st, int nstates, long nchunks, int chunk_tiles,
              unsigned long long *__restrict__ counter, const long *__restrict__ queue_begin,
              double *__restrict__ partials)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int nq = queue_begin ? kXcdCount : 1;
    const int q0 = queue_begin ? (int)(blockIdx.x % kXcdCount) : 0;
    int qi = 0;  // queues tried so far
    int s = 0;   // schedule position of the state holding chunk c
    for (;;) {
        const int q = (q0 + qi) % nq;
        const long qlo = queue_begin ? queue_begin[q] : 0;
        const long qhi = queue_begin ? queue_begin[q + 1] : nchunks;
        unsigned long long c0 = 0;
        if (lane == 0) c0 = atomicAdd(counter + q, 1ull);
        const long k = (long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                   (int)(c0 >> 32)) << 32) |
                              (unsigned)__builtin_amdgcn_readfirstlane((int)c0));
        const long c = qlo + k;
        if (c >= qhi) {  // this queue is dry (wave-uniform)
            if (++qi >= nq) break;
            continue;
        }
        if (c < st[s].chunk_begin || c >= st[s + 1].chunk_begin)
            s = find_state<true>(st, c < st[s].chunk_begin ? 0 : s + 1, nstates, c);
        const StateDesc d = st[s];
        const long t0 = d.tile_begin + (c - d.chunk_begin) * chunk_tiles;
        const long tmax = st[s + 1].tile_begin;
        const long t1 = t0 + chunk_tiles < tmax ? t0 + chunk_tiles : tmax;
        cplx ach[NW], asx[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) ach[w] = asx[w] = cmake(0.0, 0.0);
        for (long t = t0; t < t1; ++t) {
            cplx a[NW], x[NW];
            state_tile<NW, BU>(d, t - d.tile_begin, lane, a, x);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                ach[w].re = to_uniform(ach[w].re + wave_sum(a[w].re));
                ach[w].im = to_uniform(ach[w].im + wave_sum(a[w].im));
                asx[w].re = to_uniform(asx[w].re + x[w].re);
                asx[w].im = to_uniform(asx[w].im + x[w].im);
            }
        }
        if (lane == 0) {
            double *dst = partials + (size_t)c * (4 * NW);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                dst[4 * w + 0] = ach[w].re;
                dst[4 * w + 1] = ach[w].im;
                dst[4 * w + 2] = asx[w].re;
                dst[4 * w + 3] = asx[w].im;
            }
        }
    }
}

// Flat form (not persistent): one wave per tile of the plain forward's own
// shape (fwd_cols(NW) G' columns x 64 rows, fwd_tile_body_cols), four
// consecutive tiles of one state per workgroup, each state's tiles padded to
// whole workgroups.  Here chunk_begin is a state's first workgroup:
// workgroup wg finds its state by binary search, and writes one partial row
// (zeros past the state's last tile), which batched_reduce_chunks adds per
// state in a fixed order.  With no loop state to carry it keeps the plain
// forward's registers and two-column tiles.
template <int NW, int BU>
__global__ void __launch_bounds__(kBatThreads)
__attribute__((amdgpu_waves_per_eu(fwd_min_waves(NW))))
batched_flat(const StateDesc *__restrict__ st, int nstates, double *__restrict__ partials)
{
    __shared__ double red[kBatWaves][4 * NW];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // Workgroups reach the XCDs round-robin.  Within each span of
    // 8 * kFlatRun workgroups, XCD x takes the kFlatRun consecutive ones
    // starting at x * kFlatRun (neighbouring tiles share rows in its L2),
    // while across spans every XCD keeps meeting every state of the
    // cost-ordered list (contiguous per-XCD ranges of the whole grid would
    // give the first XCD all the most expensive states).  The last, partial
    // span keeps the identity.
    const long b = blockIdx.x, span = (long)kXcdCount * kFlatRun;
    const long sb = b / span;
    long wg = b;
    if ((sb + 1) * span <= (long)gridDim.x) {
        const long r = b - sb * span;
        wg = sb * span + (r % kXcdCount) * kFlatRun + r / kXcdCount;
    }
    // st[lo].chunk_begin <= wg < st[hi].chunk_begin; st[nstates] is the
    // sentinel holding the total, so the state found owns wg
    int lo = 0, hi = nstates;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (st[mid].chunk_begin <= wg) lo = mid;
        else hi = mid;
    }
    const StateDesc d = st[lo];
    constexpr int C = fwd_cols(NW);
    const int npt = (d.np + C - 1) / C;
    const long ntile = (long)((d.ng + kWave - 1) / kWave) * npt;
    const long local = (wg - d.chunk_begin) * kBatWaves + wid;

    cplx ach[NW], asx[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) ach[w] = asx[w] = cmake(0.0, 0.0);
    if (local < ntile) {
        int gt, pt, ck;
        tile_coords(local, npt, (d.ng + kWave - 1) / kWave, 1, gt, pt, ck);
        if (C == 1) {
            fwd_tile_body<NW, BU>(d.nb, d.nv, 0, d.nb, d.ng, pt, gt, lane, as_global(d.aqsm),
                                  as_global(d.aqsn), as_global(d.ieps), as_global(d.wt),
                                  as_global(d.vcoul), as_global(d.wx), ach, asx);
        } else {
            fwd_tile_body_cols<NW, BU, C>(d.nb, d.nv, 0, d.nb, d.ng, d.np, C * pt, gt, lane,
                                          as_global(d.aqsm), as_global(d.aqsn),
                                          as_global(d.ieps), as_global(d.wt),
                                          as_global(d.vcoul), as_global(d.wx), ach, asx);
        }
    }
    // wave then workgroup sums in a fixed order (row layout as the other forms)
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const double v0 = wave_sum(ach[w].re), v1 = wave_sum(ach[w].im);
        if (lane == 0) {
            red[wid][4 * w + 0] = v0;
            red[wid][4 * w + 1] = v1;
            red[wid][4 * w + 2] = asx[w].re;  // already wave totals
            red[wid][4 * w + 3] = asx[w].im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 * NW) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kBatWaves; ++k) s += red[k][threadIdx.x];
        partials[(size_t)wg * 4 * NW + threadIdx.x] = s;
    }
}

__global__ void zero_counters(unsigned long long *counter, int n)
{
    if ((int)threadIdx.x < n) counter[threadIdx.x] = 0ull;
}

// Per state (one workgroup per schedule position k): the sum of its partial
// rows [chunk_begin[k], chunk_begin[k+1]) (queue chunks, flat workgroups or
// static-schedule slots) in a fixed order.
template <int NW>
__global__ void __launch_bounds__(256)
batched_reduce_chunks(const StateDesc *__restrict__ st, const double *__restrict__ partials,
                      double2 *__restrict__ ach, double2 *__restrict__ asx)
{
    constexpr int R = 4 * NW;
    __shared__ double red[4][R];
    const int k = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const long c0 = st[k].chunk_begin, c1 = st[k + 1].chunk_begin;
    const int s = st[k].out_index;
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    for (long c = c0 + threadIdx.x; c < c1; c += 256) {
#pragma unroll
        for (int j = 0; j < R; ++j) acc[j] += partials[(size_t)c * R + j];
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) red[wid][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < R) {
        const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                         red[3][threadIdx.x];
        const int w = threadIdx.x / 4, c = threadIdx.x % 4;
        double *dst = reinterpret_cast<double *>(c < 2 ? ach + (size_t)s * NW + w
                                                       : asx + (size_t)s * NW + w);
        dst[c & 1] = v;
    }
}

// The kernel of a persistent tile variant, or nullptr where its batch
// inversion would hold more than 12 denominators (columns x bands x
// frequencies), which the plan never asks for.
template <int NW, int BU>
static const void *persistent_ptr(int sched)
{
    if constexpr (bat_cols(NW) * BU * NW <= 12)
        return (sched == kSchedQueue || sched == kSchedXcdQueues)
                   ? reinterpret_cast<const void *>(&batched_queue<NW, BU>)
                   : reinterpret_cast<const void *>(&batched_persistent<NW, BU>);
    return nullptr;
}

const void *batched_kernel(int nw, int bu, int sched)
{
#define GPP_K(NWV)                                                                 \
    case NWV:                                                                      \
        if (sched == kSchedFlat) /* the plain forward's tile shape only */         \
            return bu == fwd_bands(NWV)                                            \
                       ? reinterpret_cast<const void *>(                           \
                             &batched_flat<NWV, fwd_bands(NWV)>)                   \
                       : nullptr;                                                  \
        if (bu == 1) return persistent_ptr<NWV, 1>(sched);                         \
        if (bu == 2) return persistent_ptr<NWV, 2>(sched);                         \
        if (bu == 3) return persistent_ptr<NWV, 3>(sched);                         \
        return nullptr;
    switch (nw) {
        GPP_K(1) GPP_K(2) GPP_K(3) GPP_K(4) GPP_K(5) GPP_K(6) GPP_K(7) GPP_K(8)
    }
#undef GPP_K
    return nullptr;
}

template <int NW>
static void launch_reduce(const BatchedLaunch &L, double2 *ach, double2 *asx, hipStream_t st)
{
    hipLaunchKernelGGL(batched_reduce_chunks<NW>, dim3(L.nstates), dim3(256), 0, st, L.desc,
                       L.partials, ach, asx);
}

hipError_t launch_batched(const BatchedLaunch &L, double2 *ach, double2 *asx, hipStream_t st)
{
    const void *k = batched_kernel(L.nw, L.bu, L.sched);
    if (!k) return hipErrorInvalidValue;
    hipError_t e;
    if (L.sched == kSchedFlat) {
        // L.nchunks workgroups; none for an all-empty plan (the reduction
        // then writes zeros)
        if (L.nchunks > 0) {
            void *args[] = {(void *)&L.desc, (void *)&L.nstates, (void *)&L.partials};
            e = hipLaunchKernel(k, dim3((unsigned)L.nchunks), dim3(kBatThreads), args, 0, st);
        } else {
            e = hipSuccess;
        }
    } else if (L.sched == kSchedQueue || L.sched == kSchedXcdQueues) {
        hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, st, L.counter, kXcdCount);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const long *qb = L.sched == kSchedXcdQueues ? L.queue_begin : nullptr;
        void *args[] = {(void *)&L.desc,    (void *)&L.nstates, (void *)&L.nchunks,
                        (void *)&L.chunk_tiles, (void *)&L.counter, (void *)&qb,
                        (void *)&L.partials};
        e = hipLaunchKernel(k, dim3(L.blocks), dim3(kBatThreads), args, 0, st);
    } else {
        const int nwaves = L.blocks * kBatWaves;
        const long *chunks = L.sched == kSchedXcdChunks ? L.xcd_chunks : nullptr;
        void *args[] = {(void *)&L.desc,     (void *)&L.nstates,  (void *)&L.total_tiles,
                        (void *)&nwaves,     (void *)&L.partials, (void *)&chunks};
        e = hipLaunchKernel(k, dim3(L.blocks), dim3(kBatThreads), args, 0, st);
    }
    if (e != hipSuccess) return e;
    switch (L.nw) {
    case 1: launch_reduce<1>(L, ach, asx, st); break;
    case 2: launch_reduce<2>(L, ach, asx, st); break;
    case 3: launch_reduce<3>(L, ach, asx, st); break;
    case 4: launch_reduce<4>(L, ach, asx, st); break;
    case 5: launch_reduce<5>(L, ach, asx, st); break;
    case 6: launch_reduce<6>(L, ach, asx, st); break;
    case 7: launch_reduce<7>(L, ach, asx, st); break;
    case 8: launch_reduce<8>(L, ach, asx, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gpp
