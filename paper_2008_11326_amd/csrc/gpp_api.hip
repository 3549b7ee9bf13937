// gpp_api.hip -- C ABI entry points of libgpp.so (declared in include/gpp.h).
//
// Every entry point validates its arguments on the host before any HIP
// call, so invalid calls return an error without touching a device.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>

#include "gpp.h"
#include "gpp_internal.h"

namespace gpp {

thread_local char g_last_error[512] = "";

gpp_status fail(gpp_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

gpp_status hip_fail(hipError_t e, const char *where)
{
    return fail(GPP_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int64_t kMax32 = 2147483647;

gpp_status check_dims(const gpp_dims *d, gpp::Dims32 *out)
{
    if (!d) return fail(GPP_ERR_INVALID, "dims is NULL");
    if (d->number_bands < 0 || d->nvband < 0 || d->ncouls < 0 || d->ngpown < 0)
        return fail(GPP_ERR_INVALID, "negative dimension");
    if (d->nfreq < 1 || d->nfreq > GPP_MAX_NFREQ)
        return fail(GPP_ERR_INVALID, "nfreq=%lld outside [1, %d]", (long long)d->nfreq,
                    GPP_MAX_NFREQ);
    if (d->nvband > d->number_bands)
        return fail(GPP_ERR_INVALID, "nvband=%lld > number_bands=%lld",
                    (long long)d->nvband, (long long)d->number_bands);
    if (d->ngpown > d->ncouls)
        return fail(GPP_ERR_INVALID, "ngpown=%lld > ncouls=%lld", (long long)d->ngpown,
                    (long long)d->ncouls);
    // band indices plus a tile's few bands stay far inside 32 bits
    if (d->number_bands > GPP_MAX_NBANDS)
        return fail(GPP_ERR_INVALID, "number_bands=%lld > %d", (long long)d->number_bands,
                    GPP_MAX_NBANDS);
    if (d->ngpown > kMax32) return fail(GPP_ERR_INVALID, "dimension >= 2^31");
    // rows are addressed with 32-bit byte offsets inside the kernels
    if (d->ncouls > GPP_MAX_NCOULS)
        return fail(GPP_ERR_INVALID, "ncouls=%lld > %d", (long long)d->ncouls, GPP_MAX_NCOULS);
    // tile count must index a 32-bit grid
    int64_t gtiles = (d->ncouls + 63) / 64;
    if (gtiles * d->ngpown / 4 + 1 > kMax32)
        return fail(GPP_ERR_INVALID, "ncouls * ngpown too large for one launch");
    out->nb = (int)d->number_bands;
    out->nv = (int)d->nvband;
    out->ng = (int)d->ncouls;
    out->np = (int)d->ngpown;
    out->nw = (int)d->nfreq;
    return GPP_OK;
}

// The forward's tile grid (one workgroup per four tile chunks of at most
// 512 bands) and the adjoint's two grids must each index a 32-bit launch.
gpp_status check_fwd_grid(const gpp::Dims32 &d, const char *who)
{
    if (gpp::fwd_geometry(d).nblocks > kMax32)
        return fail(GPP_ERR_INVALID, "%s: number_bands x ncouls x ngpown too large for one launch",
                    who);
    return GPP_OK;
}

gpp_status check_bwd_grid(const gpp::Dims32 &d, const char *who)
{
    const gpp::BwdGeometry g = gpp::bwd_geometry(d);
    if (g.pair_blocks > kMax32 || g.band_blocks > kMax32)
        return fail(GPP_ERR_INVALID, "%s: number_bands x ncouls x ngpown too large for one launch",
                    who);
    return GPP_OK;
}

bool misaligned(const void *p, size_t a) { return ((uintptr_t)p) % a != 0; }

gpp_status check_array(const char *name, const void *p, int64_t elems, size_t align)
{
    if (elems == 0) return GPP_OK;
    if (!p) return fail(GPP_ERR_INVALID, "%s is NULL", name);
    if (misaligned(p, align))
        return fail(GPP_ERR_INVALID, "%s is not %zu-byte aligned", name, align);
    return GPP_OK;
}

gpp_status check_inputs(const gpp::Dims32 &d, const gpp_inputs *in, gpp::DevInputs *out)
{
    if (!in) return fail(GPP_ERR_INVALID, "inputs is NULL");
    const int64_t nbng = (int64_t)d.nb * d.ng, npng = (int64_t)d.np * d.ng;
    gpp_status s;
    if ((s = check_array("aqsmtemp", in->aqsmtemp, nbng, 16))) return s;
    if ((s = check_array("aqsntemp", in->aqsntemp, nbng, 16))) return s;
    if ((s = check_array("I_eps_array", in->I_eps_array, npng, 16))) return s;
    if ((s = check_array("wtilde_array", in->wtilde_array, npng, 16))) return s;
    if ((s = check_array("vcoul", in->vcoul, d.ng, 8))) return s;
    if ((s = check_array("wx_array", in->wx_array, (int64_t)d.nw * d.nb, 8))) return s;
    out->aqsm = reinterpret_cast<const double2 *>(in->aqsmtemp);
    out->aqsn = reinterpret_cast<const double2 *>(in->aqsntemp);
    out->ieps = reinterpret_cast<const double2 *>(in->I_eps_array);
    out->wt = reinterpret_cast<const double2 *>(in->wtilde_array);
    out->vcoul = in->vcoul;
    out->wx = in->wx_array;
    return GPP_OK;
}

// Devices whose answer is cached (ids beyond this are queried every call).
constexpr int kMaxCachedDevices = 64;

gpp_status check_device(const char *who)
{
    // per device id: 0 = not yet queried, 1 = gfx950, -1 = another target
    static std::atomic<signed char> verdict[kMaxCachedDevices];
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(GPP_ERR_UNSUPPORTED, "%s: no HIP device (%s)", who, hipGetErrorString(e));
    }
    signed char v = (dev >= 0 && dev < kMaxCachedDevices)
                        ? verdict[dev].load(std::memory_order_relaxed)
                        : (signed char)0;
    if (v == 0) {
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
            return hip_fail(e, "device query");
        v = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
        if (dev >= 0 && dev < kMaxCachedDevices) verdict[dev].store(v, std::memory_order_relaxed);
        if (v < 0)
            return fail(GPP_ERR_UNSUPPORTED, "%s: device %d is %s, not gfx950", who, dev,
                        prop.gcnArchName);
    }
    if (v < 0) return fail(GPP_ERR_UNSUPPORTED, "%s: device %d is not gfx950", who, dev);
    return GPP_OK;
}

}  // namespace gpp

using gpp::check_array;
using gpp::check_device;
using gpp::check_dims;
using gpp::check_inputs;
using gpp::fail;
using gpp::g_last_error;
using gpp::hip_fail;
using gpp::misaligned;

extern "C" {

size_t gpp_sigma_fwd_workspace(const gpp_dims *dims)
{
    gpp::Dims32 d;
    if (check_dims(dims, &d) != GPP_OK || check_fwd_grid(d, "gpp_sigma_fwd_workspace") != GPP_OK)
        return 0;
    size_t b = gpp::fwd_geometry(d).workspace_bytes;
    return b ? b : 256;
}

gpp_status gpp_sigma_fwd(const gpp_dims *dims, const gpp_inputs *in, double *achtemp,
                         double *asxtemp, void *workspace, size_t workspace_bytes,
                         void *stream)
{
    g_last_error[0] = '\0';
    gpp::Dims32 d;
    gpp::DevInputs din;
    gpp_status s;
    if ((s = check_dims(dims, &d))) return s;
    if ((s = check_fwd_grid(d, "gpp_sigma_fwd"))) return s;
    if ((s = check_inputs(d, in, &din))) return s;
    if ((s = check_array("achtemp", achtemp, d.nw, 16)) ||
        (s = check_array("asxtemp", asxtemp, d.nw, 16)))
        return s;
    const size_t need = gpp_sigma_fwd_workspace(dims);
    if (!workspace || workspace_bytes < need)
        return fail(GPP_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu%s", need,
                    workspace_bytes, workspace ? "" : " (NULL)");
    if (misaligned(workspace, 16))
        return fail(GPP_ERR_INVALID, "workspace is not 16-byte aligned");
    if ((s = check_device("gpp_sigma_fwd"))) return s;
    hipError_t e = gpp::launch_fwd(d, din, reinterpret_cast<double2 *>(achtemp),
                                   reinterpret_cast<double2 *>(asxtemp), workspace,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_fwd launch");
    return GPP_OK;
}

gpp_status gpp_sigma_qp(const gpp_dims *dims, const gpp_inputs *in, double freq_step,
                        double energy, double vxc, double *achtemp, double *asxtemp, double *qp,
                        void *workspace, size_t workspace_bytes, void *stream)
{
    g_last_error[0] = '\0';
    gpp::Dims32 d;
    gpp::DevInputs din;
    gpp_status s;
    if ((s = check_dims(dims, &d))) return s;
    if (d.nw < 3 || d.nw % 2 == 0)
        return fail(GPP_ERR_INVALID, "nfreq=%d: the quasiparticle step needs an odd number of "
                    "frequencies, at least 3", d.nw);
    if (!(freq_step > 0.0) || !(freq_step <= 1.0e300))
        return fail(GPP_ERR_INVALID, "freq_step must be finite and positive");
    if (!(energy == energy) || !(vxc == vxc) || !(energy - energy == 0.0) ||
        !(vxc - vxc == 0.0))
        return fail(GPP_ERR_INVALID, "energy and vxc must be finite");
    if ((s = check_fwd_grid(d, "gpp_sigma_qp"))) return s;
    if ((s = check_inputs(d, in, &din))) return s;
    if ((s = check_array("achtemp", achtemp, d.nw, 16)) ||
        (s = check_array("asxtemp", asxtemp, d.nw, 16)) || (s = check_array("qp", qp, 6, 8)))
        return s;
    const size_t need = gpp_sigma_fwd_workspace(dims);
    if (!workspace || workspace_bytes < need)
        return fail(GPP_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu%s", need,
                    workspace_bytes, workspace ? "" : " (NULL)");
    if (misaligned(workspace, 16))
        return fail(GPP_ERR_INVALID, "workspace is not 16-byte aligned");
    if ((s = check_device("gpp_sigma_qp"))) return s;
    gpp::QpArgs qa;
    qa.out = qp;
    qa.step = freq_step;
    qa.energy = energy;
    qa.vxc = vxc;
    hipError_t e = gpp::launch_fwd(d, din, reinterpret_cast<double2 *>(achtemp),
                                   reinterpret_cast<double2 *>(asxtemp), workspace,
                                   static_cast<hipStream_t>(stream), qa);
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_qp launch");
    return GPP_OK;
}

size_t gpp_sigma_bwd_workspace(const gpp_dims *dims)
{
    gpp::Dims32 d;
    if (check_dims(dims, &d) != GPP_OK || check_bwd_grid(d, "gpp_sigma_bwd_workspace") != GPP_OK)
        return 0;
    return gpp::bwd_geometry(d).workspace_bytes;
}

gpp_status gpp_sigma_bwd(const gpp_dims *dims, const gpp_inputs *in,
                         const double *grad_achtemp, const double *grad_asxtemp,
                         double *grad_aqsmtemp, double *grad_aqsntemp, double *grad_I_eps_array,
                         double *grad_wtilde_array, void *workspace, size_t workspace_bytes,
                         void *stream)
{
    g_last_error[0] = '\0';
    gpp::Dims32 d;
    gpp::DevInputs din;
    gpp_status s;
    if ((s = check_dims(dims, &d))) return s;
    if ((s = check_bwd_grid(d, "gpp_sigma_bwd"))) return s;
    if ((s = check_inputs(d, in, &din))) return s;
    if ((s = check_array("grad_achtemp", grad_achtemp, d.nw, 16)) ||
        (s = check_array("grad_asxtemp", grad_asxtemp, d.nw, 16)))
        return s;
    // optional outputs: NULL skips, otherwise aligned
    const void *outs[4] = {grad_aqsmtemp, grad_aqsntemp, grad_I_eps_array, grad_wtilde_array};
    const char *names[4] = {"grad_aqsmtemp", "grad_aqsntemp", "grad_I_eps_array",
                            "grad_wtilde_array"};
    for (int k = 0; k < 4; ++k)
        if (outs[k] && misaligned(outs[k], 16))
            return fail(GPP_ERR_INVALID, "%s is not 16-byte aligned", names[k]);
    const size_t need = gpp_sigma_bwd_workspace(dims);
    if (!workspace || workspace_bytes < need)
        return fail(GPP_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu%s", need,
                    workspace_bytes, workspace ? "" : " (NULL)");
    if (misaligned(workspace, 256))
        return fail(GPP_ERR_INVALID, "workspace is not 256-byte aligned");
    if ((s = check_device("gpp_sigma_bwd"))) return s;
    gpp::BwdOutputs out{reinterpret_cast<double2 *>(grad_aqsmtemp),
                        reinterpret_cast<double2 *>(grad_aqsntemp),
                        reinterpret_cast<double2 *>(grad_I_eps_array),
                        reinterpret_cast<double2 *>(grad_wtilde_array)};
    hipError_t e = gpp::launch_bwd(d, din, reinterpret_cast<const double2 *>(grad_achtemp),
                                   reinterpret_cast<const double2 *>(grad_asxtemp), out,
                                   workspace, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "gpp_sigma_bwd launch");
    return GPP_OK;
}

const char *gpp_status_string(gpp_status s)
{
    switch (s) {
    case GPP_OK: return "GPP_OK";
    case GPP_ERR_INVALID: return "GPP_ERR_INVALID: invalid argument";
    case GPP_ERR_HIP: return "GPP_ERR_HIP: HIP runtime error";
    case GPP_ERR_NOMEM: return "GPP_ERR_NOMEM: host allocation failed";
    case GPP_ERR_WORKSPACE: return "GPP_ERR_WORKSPACE: workspace missing or too small";
    case GPP_ERR_UNSUPPORTED: return "GPP_ERR_UNSUPPORTED: unsupported device";
    }
    return "unknown gpp_status";
}

const char *gpp_last_error(void) { return g_last_error; }

int gpp_version(void) { return 100; }

}  // extern "C"
