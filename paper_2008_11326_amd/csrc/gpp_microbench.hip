// gpp_microbench.hip -- empirical machine ceilings for the roofline: an
// fp64 FMA issue-rate kernel, a streaming copy of known size (the
// reference for scaling hardware byte counters), a read-bandwidth kernel
// whose window size selects the cache level it measures, and LDS access
// patterns for the bank-conflict counters.  Declared in
// include/gpp_microbench.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpp_internal.h"
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

// Read bandwidth of one level of the memory hierarchy.  Workgroup b reads a
// window of `win` 16-byte elements `reps` times, 256 lanes x 16 B per step,
// four loads in flight per lane.  shared = 0: window b of the buffer (its
// own); shared = 1: the buffer's first window, every workgroup starting at
// its own rotated offset (4096 elements apart) so that the workgroups on one
// CU read different lines.  The sums keep the loads live.
__global__ void __launch_bounds__(256) mb_read(const double2 *__restrict__ buf, long win,
                                               int shared, int reps, double *out)
{
    const double2 *w = buf + (shared ? 0 : (size_t)blockIdx.x * win);
    const long start = shared ? ((long)blockIdx.x * 4096) % win : 0;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < reps; ++r) {
        long i = threadIdx.x;
        for (; i + 3 * 256 < win; i += 4 * 256) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                long j = start + i + k * 256;
                if (j >= win) j -= win;
                const double2 v = w[j];
                s[k] += v.x + v.y;
            }
        }
        for (; i < win; i += 256) {
            long j = start + i;
            if (j >= win) j -= win;
            const double2 v = w[j];
            s[0] += v.x + v.y;
        }
    }
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// LDS access patterns (gpp_mb_lds).  The memory clobber after each round
// keeps the compiler from reusing the previous round's loads or dropping
// overwritten stores, so every round issues its 8 LDS instructions.
__global__ void __launch_bounds__(64) mb_lds(int pattern, int reps, double *out)
{
    __shared__ double2 s[8][64];
    const int l = threadIdx.x, tj = l >> 3, tk = l & 7;
#pragma unroll
    for (int r = 0; r < 8; ++r) s[r][l] = make_double2(64.0 * r + l, 1.0);
    __syncthreads();
    double acc = 0.0;
    if (pattern == 0) {
        for (int i = 0; i < reps; ++i) {
#pragma unroll
            for (int r = 0; r < 8; ++r) s[r][l] = make_double2(64.0 * (8 * i + r) + l, 1.0);
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
        __syncthreads();
        acc = s[l & 7][63 - l].x;
    } else {
        for (int i = 0; i < reps; ++i) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int e = pattern == 1 ? 8 * tk + ((c + tk + tj) & 7)
                              : pattern == 2 ? tk + 8 * ((c + tj) & 7)
                                             : 8 * tk + c;
                const double2 v = s[tj][e];
                acc += v.x + v.y;
            }
            asm volatile("" ::: "memory");
        }
    }
    out[(size_t)blockIdx.x * 64 + l] = acc;
}

}  // namespace

extern "C" {

int gpp_mb_fp64_fma(double *out, int blocks, int iters, void *stream, double *flops)
{
    if (!out || blocks <= 0 || iters <= 0) return 1;
    if (gpp::check_device("gpp_mb_fp64_fma") != GPP_OK) return 5;
    hipLaunchKernelGGL(mb_fma, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, 1.5,
                       iters);
    if (flops) *flops = 2.0 * kChains * (double)iters * 256.0 * blocks;
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

int gpp_mb_copy(const void *src, void *dst, int64_t bytes, int blocks, void *stream)
{
    if (!src || !dst || bytes <= 0 || bytes % 16 || blocks <= 0) return 1;
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return 1;
    if (gpp::check_device("gpp_mb_copy") != GPP_OK) return 5;
    hipLaunchKernelGGL(mb_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const double2 *)src, (double2 *)dst, (long)(bytes / 16));
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

int gpp_mb_read(const void *buf, int64_t window_bytes, int shared, int blocks, int reps,
                double *out, void *stream)
{
    if (!buf || !out || window_bytes <= 0 || window_bytes % 16 || blocks <= 0 || reps <= 0)
        return 1;
    if ((uintptr_t)buf % 16) return 1;
    if (gpp::check_device("gpp_mb_read") != GPP_OK) return 5;
    hipLaunchKernelGGL(mb_read, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const double2 *)buf, (long)(window_bytes / 16), shared ? 1 : 0, reps,
                       out);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

int gpp_mb_lds(int pattern, int blocks, int reps, double *out, void *stream)
{
    if (pattern < 0 || pattern > 3 || blocks <= 0 || reps <= 0 || !out) return 1;
    if ((uintptr_t)out % 8) return 1;
    if (gpp::check_device("gpp_mb_lds") != GPP_OK) return 5;
    hipLaunchKernelGGL(mb_lds, dim3(blocks), dim3(64), 0, (hipStream_t)stream, pattern, reps,
                       out);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
