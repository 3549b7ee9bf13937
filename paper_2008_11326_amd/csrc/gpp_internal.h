// gpp_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gpp.h"
#include "gpp_fwd_shape.h"

namespace gpp {

// Validated loop bounds (every value < 2^31).
struct Dims32 {
    int nb, nv, ng, np, nw;
};

struct DevInputs {
    const double2 *aqsm, *aqsn, *ieps, *wt;
    const double *vcoul, *wx;
};

struct FwdGeometry {
    long ntiles = 0;      // g-tiles x column tiles x band chunks, one per wave
    int nchunk = 1;       // band chunks (fwd_band_chunks)
    int chunk_bands = 0;  // bands per chunk (the last may be shorter)
    long nblocks = 0;     // tile-kernel workgroups of 4 waves (one partial each)
    long red_blocks = 0;  // first reduction stage workgroups
    long red_chunk = 0;   // partial rows per first-stage workgroup
    size_t partial_bytes = 0, stage_bytes = 0, workspace_bytes = 0;
};

struct BwdGeometry {
    int ngb = 0;             // 256-row blocks of the pairs kernel
    long pair_blocks = 0;    // pairs-kernel workgroups (ngb x np)
    int nbt = 0;             // band tiles of the bands kernel
    int ngt = 0;             // 64-row g tiles of the bands kernel
    int nps = 1;             // segments of the bands kernel's p range
    long band_tiles = 0;     // bands-kernel waves (segments x g tiles x band tiles)
    long band_blocks = 0;
    size_t gh_elems = 0, xgh_elems = 0, am_part_elems = 0;  // complex elements
    size_t an_part_elems = 0;  // per-segment daqsntemp partials (nps > 1 only)
    size_t workspace_bytes = 0;
};

// The quasiparticle epilogue of the final reduction stage (gpp_sigma_qp):
// out = device double[6] or nullptr (plain forward); step = spacing of the
// frequencies, energy = E of the middle one, vxc = the exchange-correlation
// value subtracted in the linearised quasiparticle equation.
struct QpArgs {
    double *out = nullptr;
    double step = 0.0, energy = 0.0, vxc = 0.0;
};

struct BwdOutputs {
    double2 *grad_am, *grad_an, *grad_ieps, *grad_wt;  // NULL = not wanted
};

// One state of a batched call, in schedule order (device-side table with
// one extra sentinel entry whose tile_begin is the total tile count).
struct StateDesc {
    const double2 *aqsm, *aqsn, *ieps, *wt;
    const double *vcoul, *wx;
    int nb, nv, ng, np;
    long tile_begin;   // first global tile of this state
    long chunk_begin;  // first partial row of this state: work-queue chunk, flat-form
                       // workgroup or static-schedule slot, by schedule
    int out_index;     // position in the caller's state order
    int pad;
};

// How the persistent waves walk the concatenated tile list.
enum BatchedSchedule {
    kSchedRoundRobin = 0,  // wave w: tiles w, w + W, ...
    kSchedXcdChunks = 1,   // one equal-cost contiguous chunk per XCD
    kSchedQueue = 2,       // waves take chunk_tiles-tile chunks from a counter
    kSchedXcdQueues = 3,   // one such queue per XCD over its own region, with stealing
    kSchedFlat = 4,        // not persistent: one workgroup per four tiles of one state
};
constexpr int kSchedCount = 5;

struct BatchedLaunch {
    int nw, bu, blocks, sched;
    const StateDesc *desc;
    int nstates;
    long total_tiles;
    const long *xcd_chunks;  // kSchedXcdChunks: kXcdCount + 1 boundaries
    long nchunks;            // kSchedQueue
    int chunk_tiles;         // kSchedQueue
    unsigned long long *counter;  // queue schedules: kXcdCount counters, zeroed by the launch
    const long *queue_begin;      // kSchedXcdQueues: kXcdCount + 1 chunk boundaries
    double *partials;
};

const void *batched_kernel(int nw, int bu, int sched);
hipError_t launch_batched(const BatchedLaunch &L, double2 *ach, double2 *asx, hipStream_t st);
constexpr int kXcdCount = 8;

// The same for the batched persistent forward's tiles, and the register cap
// (minimum waves per SIMD) of its two-column form.  The batched kernel keeps
// one column: with two, its persistent loop runs out of scalar registers,
// the per-band aqsmtemp and aqsntemp loads become per-lane vector loads, and
// it measured 30 % slower (640-690 ms against 494 ms on 64 states).
#ifndef GPP_BAT_COLS
#define GPP_BAT_COLS 1
#endif
#ifndef GPP_BAT_WAVES2
#define GPP_BAT_WAVES2 3
#endif
constexpr int bat_cols(int nw) { return nw <= 3 ? GPP_BAT_COLS : 1; }

// host-side validation and error reporting shared by the entry points
extern thread_local char g_last_error[512];
gpp_status fail(gpp_status s, const char *fmt, ...);
gpp_status hip_fail(hipError_t e, const char *where);
gpp_status check_dims(const gpp_dims *d, Dims32 *out);
gpp_status check_array(const char *name, const void *p, int64_t elems, size_t align);
gpp_status check_inputs(const Dims32 &d, const gpp_inputs *in, DevInputs *out);
gpp_status check_fwd_grid(const Dims32 &d, const char *who);
gpp_status check_bwd_grid(const Dims32 &d, const char *who);
bool misaligned(const void *p, size_t a);
// GPP_OK when the current HIP device is a gfx950, else GPP_ERR_UNSUPPORTED
// (no device, or another target) with a message naming `who`.  The device's
// answer is cached after the first query.
gpp_status check_device(const char *who);

FwdGeometry fwd_geometry(const Dims32 &d);
BwdGeometry bwd_geometry(const Dims32 &d);
hipError_t launch_bwd(const Dims32 &d, const DevInputs &in, const double2 *ga,
                      const double2 *gs, const BwdOutputs &out, void *workspace, hipStream_t st);
// Fixed-order two-stage sum of nrows partial rows of 4*nw doubles (achtemp
// re/im, asxtemp re/im per frequency) into achtemp/asxtemp; the first stage
// writes reduce_stage_bytes(nw, nrows) bytes to stage.
size_t reduce_stage_bytes(int nw, long nrows);
hipError_t launch_reduce_partials(int nw, const double *partials, long nrows, double *stage,
                                  double2 *ach, double2 *asx, hipStream_t st);
hipError_t launch_fwd(const Dims32 &d, const DevInputs &in, double2 *ach, double2 *asx,
                      void *workspace, hipStream_t st, const QpArgs &qp = QpArgs());

}  // namespace gpp
