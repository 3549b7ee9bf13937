// gpp_microbench.hip -- empirical machine ceilings for the roofline: an
// fp64 FMA issue-rate kernel and a streaming copy of known size (the
// reference for scaling hardware byte counters).  Declared in
// include/gpp_microbench.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpp_microbench.h"

namespace {

constexpr int kChains = 16;

// kChains independent dependent-FMA chains per lane; `iters` rounds of one
// FMA per chain.  2 * 64 * kChains * iters fp64 operations per wave.
__global__ void __launch_bounds__(256) mb_fma(double *out, double seed, int iters)
{
    double a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = seed + 1e-3 * threadIdx.x + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], 0.9999999, 1e-9);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// dst[i] = src[i] for n 16-byte elements, grid-stride.
__global__ void __launch_bounds__(256) mb_copy(const double2 *__restrict__ src,
                                               double2 *__restrict__ dst, long n)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

int gpp_mb_fp64_fma(double *out, int blocks, int iters, void *stream, double *flops)
{
    if (!out || blocks <= 0 || iters <= 0) return 1;
    hipLaunchKernelGGL(mb_fma, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, 1.5,
                       iters);
    if (flops) *flops = 2.0 * kChains * (double)iters * 256.0 * blocks;
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

int gpp_mb_copy(const void *src, void *dst, int64_t bytes, int blocks, void *stream)
{
    if (!src || !dst || bytes <= 0 || bytes % 16 || blocks <= 0) return 1;
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return 1;
    hipLaunchKernelGGL(mb_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const double2 *)src, (double2 *)dst, (long)(bytes / 16));
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
