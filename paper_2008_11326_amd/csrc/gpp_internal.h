// gpp_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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
    long ntiles = 0;      // (ceil(ng/64) g-tiles) x (np columns), one per wave
    long nblocks = 0;     // tile-kernel workgroups of 4 waves (one partial each)
    long red_blocks = 0;  // first reduction stage workgroups
    long red_chunk = 0;   // partial rows per first-stage workgroup
    size_t partial_bytes = 0, stage_bytes = 0, workspace_bytes = 0;
};

struct BwdGeometry {
    int ngb = 0;             // 256-row blocks of the pairs kernel
    long pair_blocks = 0;    // pairs-kernel workgroups (ngb x np)
    int nbt = 0;             // band tiles of the bands kernel
    long band_tiles = 0;     // bands-kernel waves (g tiles x band tiles)
    long band_blocks = 0;
    size_t gh_elems = 0, xgh_elems = 0, am_part_elems = 0;  // complex elements
    size_t workspace_bytes = 0;
};

struct BwdOutputs {
    double2 *grad_am, *grad_an, *grad_ieps, *grad_wt;  // NULL = not wanted
};

FwdGeometry fwd_geometry(const Dims32 &d);
BwdGeometry bwd_geometry(const Dims32 &d);
hipError_t launch_bwd(const Dims32 &d, const DevInputs &in, const double2 *ga,
                      const double2 *gs, const BwdOutputs &out, void *workspace, hipStream_t st);
hipError_t launch_fwd(const Dims32 &d, const DevInputs &in, double2 *ach, double2 *asx,
                      void *workspace, hipStream_t st);

}  // namespace gpp
