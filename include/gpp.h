/*
 * gpp.h -- C ABI of the MI355X (gfx950) GPP self-energy library, libgpp.so.
 *
 * The operation (paper Sec. II-A, pseudo-code of the GPP kernel, with the
 * branch skeleton of Sec. III v2 and squared compares of v3):
 *
 *   achtemp[w] = sum_{n<NB} sum_{p<NP} sum_{g<NG}  vcoul[g]/2 * M * sch(n,p,g,w)
 *   asxtemp[w] = sum_{n<NV} sum_{p<NP} sum_{g<NG}  vcoul[g]   * M * ssx(n,p,g,w)
 *   M = aqsntemp[n][g] * conj(aqsmtemp[n][p]),  x = wx_array[w][n],
 *   om = wtilde_array[p][g],  e = I_eps_array[p][g]
 *
 *   dr = x - Re om, wi2 = (Im om)^2, wdiffr = fma(dr, dr, wi2),
 *   wtr = fma(Re om, Re om, wi2)                       (all fp64, round-to-nearest)
 *   branch A: wdiffr > 0.25 and wtr < fl(250000 * wdiffr)
 *             sch = e om / (x - om),  ssx = e om^2 / ((x - om)(x + om))
 *   branch B: not A and wtr > fl(1e-12 * wdiffr)
 *             sch = 0,                ssx = -e om / (2 (x + om))
 *   branch C: otherwise sch = ssx = 0
 *
 * NB = number_bands, NV = nvband (occupied bands), NG = ncouls (G rows),
 * NP = ngpown (G' columns held by this process), NW = nfreq.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *    tensors) unless marked "host".  Complex arrays are interleaved
 *    (re, im) fp64 pairs, row-major with the last index fastest; complex
 *    pointers must be 16-byte aligned, real ones 8-byte aligned.
 *  - The caller owns every buffer, including the workspace; the library
 *    keeps no pointer after a call returns.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default
 *    stream) and the call returns without synchronising.  Outputs are
 *    overwritten, never accumulated into.
 *  - Arguments are validated before anything is enqueued; a failed check
 *    returns GPP_ERR_INVALID (or GPP_ERR_WORKSPACE) and touches nothing.
 *    Then the current HIP device must be a gfx950: otherwise (another
 *    target, or no device at all) the call returns GPP_ERR_UNSUPPORTED and
 *    enqueues nothing.  The answer is cached per device after the first
 *    query, so the check costs one hipGetDevice per call.
 *    HIP runtime failures return GPP_ERR_HIP.  gpp_last_error() gives a
 *    thread-local message for the most recent failure.  No C++ exception
 *    crosses this interface.
 *  - Inputs must be finite; non-finite inputs give unspecified outputs.
 *  - Results are deterministic: the same inputs, sizes and device give
 *    bitwise-identical outputs (fixed-order reductions, no atomics).
 */
#ifndef GPP_H
#define GPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GPP_OK = 0,
    GPP_ERR_INVALID = 1,     /* bad dims, NULL or misaligned pointer      */
    GPP_ERR_HIP = 2,         /* a HIP runtime call failed                 */
    GPP_ERR_NOMEM = 3,       /* host allocation failed                    */
    GPP_ERR_WORKSPACE = 4,   /* workspace NULL or smaller than required   */
    GPP_ERR_UNSUPPORTED = 5  /* device is not gfx950 / no device          */
} gpp_status;

/* Loop bounds (Sec. II-A).  Requirements: 0 <= nvband <= number_bands,
 * 0 <= ngpown <= ncouls <= GPP_MAX_NCOULS, 1 <= nfreq <= GPP_MAX_NFREQ,
 * number_bands <= GPP_MAX_NBANDS, and each kernel grid a call launches within
 * 2^31 workgroups (number_bands x ncouls x ngpown bounds it; a call beyond
 * returns GPP_ERR_INVALID, its workspace query 0).  number_bands, ncouls or
 * ngpown may be 0 (outputs are then 0). */
typedef struct {
    int64_t number_bands;
    int64_t nvband;
    int64_t ncouls;
    int64_t ngpown;
    int64_t nfreq;
} gpp_dims;

#define GPP_MAX_NFREQ 8
#define GPP_MAX_NCOULS (1 << 26)
#define GPP_MAX_NBANDS (1 << 30)

/* Device input arrays (read only).  A pointer may be NULL only when its
 * array has no elements. */
typedef struct {
    const double *aqsmtemp;     /* complex [number_bands][ncouls]; only the
                                   first ngpown columns are read          */
    const double *aqsntemp;     /* complex [number_bands][ncouls]          */
    const double *I_eps_array;  /* complex [ngpown][ncouls]                */
    const double *wtilde_array; /* complex [ngpown][ncouls]                */
    const double *vcoul;        /* real    [ncouls]                        */
    const double *wx_array;     /* real    [nfreq][number_bands]           */
} gpp_inputs;

/* Bytes of device workspace gpp_sigma_fwd needs for `dims` (host-only
 * computation, no device call).  Returns 0 for invalid dims. */
size_t gpp_sigma_fwd_workspace(const gpp_dims *dims);

/*
 * gpp_sigma_fwd -- the reduction above (Sec. II-A), one G'-column share.
 *   dims, in:        host pointer
 *   achtemp, asxtemp: device, complex [nfreq] each, overwritten
 *   workspace:       device, >= gpp_sigma_fwd_workspace(dims) bytes,
 *                    16-byte aligned; contents unspecified afterwards
 *   stream:          hipStream_t or NULL
 * Three kernels run on `stream`: the tile kernel writes one partial per
 * workgroup into the workspace (above 512 bands, the band loop of each tile
 * is split into chunks of at most 512 bands, each with its own partial),
 * then two fixed-order reduction stages produce the outputs (the separate
 * reduction kernel of Sec. II-A).
 * Masked (branch B/C) Coulomb-hole terms add nothing to the sums (the
 * branch test is the execution mask of their accumulation), so an output
 * none of whose terms is on branch A comes back exactly 0.
 */
gpp_status gpp_sigma_fwd(const gpp_dims *dims, const gpp_inputs *in,
                         double *achtemp, double *asxtemp, void *workspace,
                         size_t workspace_bytes, void *stream);

/*
 * gpp_sigma_fwd_noalloc -- gpp_sigma_fwd for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same operation, kernels and results
 * (bit for bit) as gpp_sigma_fwd; the workspace is a fixed device array of
 * GPP_NOALLOC_SCRATCH_BYTES inside the library, one per device, allocated
 * with the library's code object and held until the process ends.  The
 * call itself allocates nothing: the first call on a device resolves that
 * device's array address (hipGetSymbolAddress, with the device current),
 * so make one call before capturing a graph.
 *   dims, in, achtemp, asxtemp, stream: as gpp_sigma_fwd
 * Sizes whose gpp_sigma_fwd_workspace(dims) exceeds GPP_NOALLOC_SCRATCH_BYTES
 * return GPP_ERR_WORKSPACE and enqueue nothing (96 MiB covers 1024 bands x
 * 65536 rows x 3276 columns at nfreq 3: 80.6 MB).  Every call on one device shares
 * that device's array: calls that overlap in time on one device (different
 * streams, or host threads without ordering) race and give wrong results;
 * calls ordered on one stream are safe.  Nothing in the array needs to
 * start at zero (every partial row a kernel reads was written earlier in
 * the same call).
 */
#define GPP_NOALLOC_SCRATCH_BYTES (96u << 20)
gpp_status gpp_sigma_fwd_noalloc(const gpp_dims *dims, const gpp_inputs *in, double *achtemp,
                                 double *asxtemp, void *stream);

/*
 * gpp_sigma_qp -- gpp_sigma_fwd followed by the quasiparticle step that
 * consumes its outputs in the Sigma module the kernel comes from (Sec.
 * II-A; the paper does not print this step, so the reading below is the
 * library's).  The nfreq frequencies are equally spaced around the state's
 * energy: E_w = energy + (w - m) freq_step, m = (nfreq - 1)/2, i.e.
 * wx_array[w][n] = E_w - e_n.  With Sigma(E_w) = achtemp[w] - asxtemp[w]
 * (asxtemp is the unsigned screened-exchange sum):
 *   qp[0], qp[1]  Sigma(E) = Sigma(E_m), re and im
 *   qp[2], qp[3]  dSigma/dE = (Sigma(E_{m+1}) - Sigma(E_{m-1})) / (2 freq_step)
 *   qp[4]         Z = 1 / (1 - Re dSigma/dE)
 *   qp[5]         E_qp = energy + Z (Re Sigma(E) - vxc), the linearised
 *                 quasiparticle energy for the exchange-correlation value vxc
 *   dims, in:       as gpp_sigma_fwd; nfreq must be odd and at least 3
 *   freq_step:      host, finite and > 0; energy, vxc: host, finite
 *   achtemp, asxtemp: device, complex [nfreq], overwritten (as gpp_sigma_fwd)
 *   qp:             device, double [6], 8-byte aligned, overwritten
 *   workspace:      device, >= gpp_sigma_fwd_workspace(dims) bytes, 16-byte aligned
 * The step runs inside the forward's last reduction kernel (no extra
 * launch).  An empty sum gives Sigma = 0, Z = 1, E_qp = energy - vxc.
 */
gpp_status gpp_sigma_qp(const gpp_dims *dims, const gpp_inputs *in, double freq_step,
                        double energy, double vxc, double *achtemp, double *asxtemp, double *qp,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of device workspace gpp_sigma_bwd needs for `dims` (host-only
 * computation).  It grows as ceil(ncouls/256) * number_bands * ngpown * 16
 * bytes (partial sums of the aqsmtemp gradient), plus, for problems small
 * enough that the aqsntemp-gradient pass splits its G' range into S > 1
 * segments to fill the GPU, S * number_bands * ncouls * 16 bytes (S <= 16
 * when ngpown >= 1024; 4 at 256 bands x 16384 rows).  Returns 0 for invalid
 * dims. */
size_t gpp_sigma_bwd_workspace(const gpp_dims *dims);

/*
 * gpp_sigma_bwd -- adjoint of gpp_sigma_fwd for the loss
 *     L = sum_w Re(conj(grad_achtemp[w]) achtemp[w] + conj(grad_asxtemp[w]) asxtemp[w]),
 * i.e. the vector-Jacobian product of the reduction of Sec. II-A.  Each
 * gradient of a complex input z is dL/dRe z + i dL/dIm z (PyTorch's
 * convention); the branch of Sec. III v2 is piecewise constant and is not
 * differentiated.  vcoul and wx_array get no gradient.
 *   grad_achtemp, grad_asxtemp: device, complex [nfreq]
 *   grad_aqsmtemp:     device, complex [number_bands][ncouls] (columns
 *                      >= ngpown are set to 0), or NULL to skip
 *   grad_aqsntemp:     device, complex [number_bands][ncouls] or NULL
 *   grad_I_eps_array:  device, complex [ngpown][ncouls] or NULL
 *   grad_wtilde_array: device, complex [ngpown][ncouls] or NULL
 *   workspace:         device, >= gpp_sigma_bwd_workspace(dims) bytes,
 *                      256-byte aligned
 * Every term's wdiff, reciprocal and branch are recomputed (nothing is
 * kept from the forward).  Outputs are overwritten; deterministic.
 */
gpp_status gpp_sigma_bwd(const gpp_dims *dims, const gpp_inputs *in,
                         const double *grad_achtemp, const double *grad_asxtemp,
                         double *grad_aqsmtemp, double *grad_aqsntemp,
                         double *grad_I_eps_array, double *grad_wtilde_array,
                         void *workspace, size_t workspace_bytes, void *stream);

/* ---- batched forward over many quasiparticle states ------------------- */

#define GPP_MAX_STATES 65536

/* Opaque plan: the states' sizes, the chosen tile variant and schedule,
 * a device descriptor table and a captured hipGraph. */
typedef struct gpp_plan gpp_plan;

/*
 * gpp_plan_create -- plan a batched forward for `nstates` states whose
 * sizes are dims_host[0..nstates-1] (host array; every state must share
 * nfreq).  Queries the current device (must be gfx950), sizes the
 * persistent grids to the kernels' resident capacity, and allocates the
 * plan's device descriptor table, pinned staging buffer and capture
 * stream.  The schedule is tuned on the first gpp_sigma_batched call (or
 * taken from the tuning cache, see below).  Candidates: the flat grid (the
 * untuned default) and the persistent schedules 0-3 of gpp_plan_info, each
 * with its tile variants; the environment variable GPP_BATCHED_SCHEDULE=<n>
 * keeps only schedule n, and GPP_BATCHED_BANDS=<b> only the persistent
 * candidates with b bands per group (either bypasses the cache; for
 * tests).  *out is NULL on failure.
 */
gpp_status gpp_plan_create(int32_t nstates, const gpp_dims *dims_host, gpp_plan **out);

/* Device workspace bytes gpp_sigma_batched needs with this plan: 256 bytes
 * of queue counters plus one 32*nfreq-byte partial row per tile at most
 * (gpp_plan_info.total_tiles), rounded up to 256 bytes; 0 for NULL. */
size_t gpp_plan_workspace(const gpp_plan *plan);

typedef struct {
    int32_t tuned;            /* 1 once a candidate has been chosen          */
    int32_t from_cache;       /* 1 if the choice came from the tuning cache  */
    int32_t bands_per_group;  /* tile variant of the chosen candidate        */
    int32_t schedule_order;   /* 0 = caller order, 1 = longest tiles first   */
    int32_t workgroups;       /* persistent workgroups (4 waves each); for
                                 the flat schedule, all of its workgroups     */
    int32_t waves;
    int32_t candidates;       /* size of the search space                    */
    int32_t schedule;         /* 0 = global round-robin, 1 = one contiguous
                                 chunk of the tile list per XCD, 2 = work
                                 queue of 2-tile chunks, 3 = one such queue
                                 per XCD (own region first, then stealing),
                                 4 = flat grid (not persistent: one
                                 workgroup per four tiles of the plain
                                 forward's shape)                            */
    int64_t total_tiles;      /* 64-row wave tiles over all states           */
    double tuned_ms;          /* measured time of the chosen candidate       */
} gpp_plan_info;

/* Fill *info (host) with the plan's current choice. */
gpp_status gpp_plan_get_info(const gpp_plan *plan, gpp_plan_info *info);

/*
 * gpp_sigma_batched -- for every state s, the reduction of gpp_sigma_fwd
 * (Sec. II-A) over inputs_host[s] (host array of device-pointer sets),
 * all states in one persistent launch followed by one per-state reduction,
 * replayed from a hipGraph.
 *   achtemp, asxtemp: device, complex [nstates][nfreq], overwritten
 *   workspace:        device, >= gpp_plan_workspace(plan) bytes, 256-byte
 *                     aligned
 * First call (tuning): unless the cache holds a choice for these sizes on
 * this architecture, each candidate (tile variant x state order x
 * tile-to-wave schedule) runs
 * twice on the caller's inputs, timed with events (the call synchronises
 * `stream` then), and the fastest is kept and saved to the cache file
 * $GPP_TUNE_CACHE (default $XDG_CACHE_HOME/gpp/tune.json, else
 * ~/.cache/gpp/tune.json; unreadable or corrupt files are ignored).
 * GPP_AUTOTUNE=off skips timing and uses the default candidate;
 * GPP_TUNE_VERBOSE=1 prints every candidate's time to stderr.
 * Every call: the descriptor table is re-uploaded (async, on `stream`)
 * only when an input pointer changed; the graph is re-captured only when
 * achtemp, asxtemp or workspace changed.  Calls on one plan must be
 * ordered (one stream, or externally synchronised); `stream` must not be
 * capturing.  Results are deterministic for a fixed plan choice.
 */
gpp_status gpp_sigma_batched(gpp_plan *plan, const gpp_inputs *inputs_host,
                             double *achtemp, double *asxtemp, void *workspace,
                             size_t workspace_bytes, void *stream);

/* Release a plan.  Work using it must have completed. */
void gpp_plan_destroy(gpp_plan *plan);

/* Static string for a status code. */
const char *gpp_status_string(gpp_status status);

/* Thread-local message describing the most recent failure on this thread
 * ("" if none).  Valid until the next call on the same thread. */
const char *gpp_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int gpp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GPP_H */
