// gpp_device.h -- device helpers shared by the GPP kernels (gfx950, fp64).
//
// Branch specification (Sec. III v2 three-way branch, v3 squared compares;
// the |delw| test is cross-multiplied so no divide is needed):
//   dr = x - Re om;  wi2 = (Im om)^2;  wdiffr = fma(dr, dr, wi2);
//   wtr = fma(Re om, Re om, wi2)
//   A: wdiffr > kLimitTwo && wtr < fl(kLimitOne * wdiffr)
//   B: !A && wtr > fl(kTolZero * wdiffr)
//   C: otherwise
// Every quantity in a branch decision is computed with exactly these
// roundings; only term *values* may use other (faithful) evaluations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpp {

constexpr double kLimitTwo = 0.25;
constexpr double kLimitOne = 250000.0;
constexpr double kTolZero = 1e-12;
// kLimitOne * kLimitTwo, exact.  For wtr below it, A <=> wdiffr > kLimitTwo:
// rounding is monotone, so wdiffr > 1/4 gives fl(kLimitOne*wdiffr) >= 62500.
constexpr double kFastWtr = 62500.0;
// Smallest (Im om)^2 for which the batch inversion may take the CH
// denominators unclamped: every |x - om|^2 >= (Im om)^2 >= 2^-60, so a
// product of up to 12 of them stays >= 2^-720, far from underflow.
constexpr double kMinUnclampedWi2 = 0x1p-60;

constexpr int kWave = 64;

struct cplx {
    double re, im;
};

// Global-memory pointer types: pointers read from memory (not kernel
// arguments) keep their address space this way, so loads through them
// compile to global or scalar loads rather than flat ones.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)p;
}

__device__ __forceinline__ cplx cmake(double re, double im) { return {re, im}; }
__device__ __forceinline__ cplx cload(const double2 *p) {
    double2 v = *p;
    return {v.x, v.y};
}
// The same wave-uniform integer, opaque to the optimiser: loads indexed by
// it cannot be hoisted out of the loop that calls this.  Used where
// wave-uniform values would otherwise be hoisted into more scalar registers
// than exist (and spilled into vector lanes); reloading them each iteration
// goes through the scalar cache instead.  The base pointer stays visible,
// so the loads remain scalar loads.
__device__ __forceinline__ int opaque_uniform(int v) {
    asm volatile("" : "+s"(v));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ cplx cload(gptr<double2> p) {
    return {p->x, p->y};  // member reads: one 16-byte load after vectorising
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// a * conj(b)
__device__ __forceinline__ cplx cmul_conj(cplx a, cplx b) {
    return {fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -a.re * b.im)};
}
__device__ __forceinline__ cplx cscale(double s, cplx a) { return {s * a.re, s * a.im}; }
// acc += a * b
__device__ __forceinline__ void cmac(cplx &acc, cplx a, cplx b) {
    acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
    acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}

// 1/d for normal d: the hardware estimate refined by two Newton-Raphson
// steps r <- r + r (1 - d r).  Each step squares the relative error; two
// steps from the estimate end within about one ulp.  Not for 0, inf,
// denormal inputs (callers only use it where d > 1/4).
__device__ __forceinline__ double rcp_nr2(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return r;
}

// Newton steps after the hardware estimate for the batch product.  The
// estimate is good to 2^-24.4; one step leaves a relative error below
// 2.2e-15 (2^-48.7, measured over normal inputs with exponents -720..1000,
// the range a batch product can take), which is shared by the K reciprocals
// of the batch.  That is far inside the 1e-12 bar on every output, and saves
// two fused multiply-adds per batch.
#ifndef GPP_BATCH_NEWTON
#define GPP_BATCH_NEWTON 1
#endif
// 1/d for normal d with GPP_BATCH_NEWTON Newton-Raphson steps from the
// hardware estimate.
__device__ __forceinline__ double rcp_batch(double d) {
    double r = __builtin_amdgcn_rcp(d);
#pragma unroll
    for (int i = 0; i < GPP_BATCH_NEWTON; ++i) {
        const double e = fma(-d, r, 1.0);
        r = fma(r, e, r);
    }
    return r;
}

// Batch inversion: r[k] = 1/d[k] for K positive values from one reciprocal
// of their product.  Prefix products c[k] = d[0]...d[k]; then R = 1/c[K-1]
// and, walking back, r[k] = R c[k-1] and R <- R d[k].  Costs 3(K-1)
// multiplies plus one rcp_batch instead of K reciprocals; each r[k] carries
// the error of R plus at most 2K roundings.  The batch path needs every d[k] >= 2^-60 (so that no
// prefix product, K <= 12, leaves the normal range at the bottom; callers
// pass batch_ok = false for a lane without that bound) and c[K-1] < 2^1000
// (an overflowed prefix stays infinite, so this also covers the middle
// ones).  Other lanes take the one-by-one path; a zero there gives an
// infinite or NaN reciprocal, which callers mask.
template <int K>
__device__ __forceinline__ void batch_reciprocal(const double (&d)[K], double (&r)[K],
                                                 bool batch_ok = true) {
    static_assert(K <= 12, "the 2^-60 lane bound keeps products of at most 12 factors normal");
    double c[K];
    c[0] = d[0];
#pragma unroll
    for (int k = 1; k < K; ++k) c[k] = c[k - 1] * d[k];
    if (__builtin_expect(batch_ok && c[K - 1] < 0x1p1000, 1)) {
        double R = rcp_batch(c[K - 1]);
#pragma unroll
        for (int k = K - 1; k > 0; --k) {
            r[k] = R * c[k - 1];
            R = R * d[k];
        }
        r[0] = R;
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) r[k] = rcp_nr2(d[k]);
    }
}

// How the hot loops apply the branch-A test to a term.  2: the compare
// itself writes the wave's execution mask (v_cmpx) around the term's
// accumulation; 1: the same mask through a compiler-generated branch (a
// compare, then a scalar mask update); in both, masked lanes add nothing
// and no select is spent.  0: through mask_keep on the reciprocal.
#ifndef GPP_EXEC_MASK
#define GPP_EXEC_MASK 2
#endif

// keep ? v : (a value of magnitude below 2^-1042) with one 32-bit select:
// only the high word (sign, exponent, top mantissa bits) is cleared, which
// leaves a denormal made of v's low word.  Added to any accumulator above
// 2^-990 in magnitude it changes nothing, so sums are the same as with an
// exact zero unless the whole sum is below ~2^-1000.
__device__ __forceinline__ double mask_keep(bool keep, double v) {
    const int lo = __double2loint(v);
    const int hi = keep ? __double2hiint(v) : 0;
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double next_up(double t) {
    return __longlong_as_double(__double_as_longlong(t) + 1);  // t > 0
}
__device__ __forceinline__ double next_down(double t) {
    return __longlong_as_double(__double_as_longlong(t) - 1);  // t > 0
}

// Per-(p,g) threshold thr with  A <=> wdiffr > thr,  bit-exact with the
// specification for every wdiffr >= 0.  fl(kLimitOne * d) is monotone in
// d, so {d : wtr < fl(kLimitOne * d)} = {d >= T}; A is then
// d > kLimitTwo && d >= T, i.e. d > max(kLimitTwo, pred(T)).
__device__ inline double branch_a_threshold(double wtr) {
#pragma clang fp contract(off)
    if (wtr < kFastWtr) return kLimitTwo;
    if (!(wtr <= 1.0e300)) return __builtin_inf();  // NaN/huge: never A
    double t = wtr * 4.0e-6;                          // ~ wtr / kLimitOne
    for (int i = 0; i < 64 && !(kLimitOne * t > wtr); ++i) t = next_up(t);
    for (int i = 0; i < 64 && (kLimitOne * next_down(t) > wtr); ++i) t = next_down(t);
    double p = next_down(t);
    return p > kLimitTwo ? p : kLimitTwo;
}

__device__ inline bool branch_b_holds(double wtr, double wdiffr) {
#pragma clang fp contract(off)
    return wtr > kTolZero * wdiffr;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Element at byte offset `off` of a complex row of `len` elements whose
// base is wave-uniform: a raw buffer load with the row in a scalar buffer
// descriptor (gfx9 descriptor word 3 = 0x00020000) and the offset in a
// vector register.  Offsets at or beyond the row length read as zero.
__device__ __forceinline__ cplx load_row_elem(gptr<double2> row, int len, uint32_t off) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(const double2 *)row, (short)0, len * (int)sizeof(double2), 0x00020000);
    const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    return {v.x, v.y};
}

// Mark a pointer read from memory as a global-memory pointer, so accesses
// through it compile to global/scalar loads instead of flat ones (pointers
// passed as kernel arguments get this from address-space inference).
// A wave-uniform value moved into scalar registers (the value of lane 0).
__device__ __forceinline__ double to_uniform(double t) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(t));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(t));
    return __hiloint2double(hi, lo);
}

// Wave total of v, returned as a wave-uniform (scalar-register) value.
__device__ __forceinline__ double wave_sum_uniform(double v) { return to_uniform(wave_sum(v)); }

// Map a hardware workgroup id to a logical one so that each of the 8 XCDs
// (which receive workgroups round-robin) walks a contiguous logical range
// and its private L2 sees neighbouring tiles.  A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
    const uint32_t kXcd = 8;
    uint32_t x = b % kXcd, i = b / kXcd, per = n / kXcd, rem = n % kXcd;
    return x * per + (x < rem ? x : rem) + i;
}

}  // namespace gpp
