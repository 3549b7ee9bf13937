// gpp_noalloc.hip -- gpp_sigma_fwd_noalloc: the plain forward for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Its workspace (the tile
// kernel's per-workgroup partial rows and the first reduction stage's rows)
// is a fixed file-scope device array instead of a caller buffer; the
// kernels are the plain forward's own.
#include <mutex>

#include "gpp.h"
#include "gpp_internal.h"

namespace {

// One array per device, allocated with the code object and held until the
// process ends.  In host code `scratch` names a host-side shadow, not the
// device memory: kernels and copies get the address hipGetSymbolAddress
// returns for the current device (scratch_ptr below).
__device__ __align__(256) unsigned char scratch[GPP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices];

// The device address of `scratch` on the current device, resolved once per
// device (with that device current) on the first call there.
gpp_status scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gpp::hip_fail(e, "gpp_sigma_fwd_noalloc: device query");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return gpp::fail(GPP_ERR_UNSUPPORTED, "gpp_sigma_fwd_noalloc: device %d beyond the %d "
                         "the library keeps scratch addresses for", dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gpp::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                 "gpp_sigma_fwd_noalloc: scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GPP_OK;
}

}  // namespace

extern "C" {

gpp_status gpp_sigma_fwd_noalloc(const gpp_dims *dims, const gpp_inputs *in, double *achtemp,
                                 double *asxtemp, void *stream)
{
    gpp::g_last_error[0] = '\0';
    gpp::Dims32 d;
    gpp::DevInputs din;
    gpp_status s;
    if ((s = gpp::check_dims(dims, &d))) return s;
    if ((s = gpp::check_fwd_grid(d, "gpp_sigma_fwd_noalloc"))) return s;
    if ((s = gpp::check_inputs(d, in, &din))) return s;
    if ((s = gpp::check_array("achtemp", achtemp, d.nw, 16)) ||
        (s = gpp::check_array("asxtemp", asxtemp, d.nw, 16)))
        return s;
    const size_t need = gpp::fwd_geometry(d).workspace_bytes;
    if (need > (size_t)GPP_NOALLOC_SCRATCH_BYTES)
        return gpp::fail(GPP_ERR_WORKSPACE,
                         "gpp_sigma_fwd_noalloc: these sizes need %zu bytes of workspace, the "
                         "fixed scratch array holds %zu; use gpp_sigma_fwd with a workspace",
                         need, (size_t)GPP_NOALLOC_SCRATCH_BYTES);
    if ((s = gpp::check_device("gpp_sigma_fwd_noalloc"))) return s;
    void *ws = nullptr;
    if ((s = scratch_ptr(&ws))) return s;
    // every partial row the kernels read is written earlier in the same
    // call, so nothing in the array has to start at zero
    hipError_t e = gpp::launch_fwd(d, din, reinterpret_cast<double2 *>(achtemp),
                                   reinterpret_cast<double2 *>(asxtemp), ws,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return gpp::hip_fail(e, "gpp_sigma_fwd_noalloc launch");
    return GPP_OK;
}

}  // extern "C"
