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

constexpr int kWave = 64;

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmake(double re, double im) { return {re, im}; }
__device__ __forceinline__ cplx cload(const double2 *p) {
    double2 v = *p;
    return {v.x, v.y};
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
// a / b with an IEEE-rounded real division of the scaled numerator.
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    double den = fma(b.re, b.re, b.im * b.im);
    double inv = 1.0 / den;
    cplx num = cmul_conj(a, b);
    return {num.re * inv, num.im * inv};
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

// Map a hardware workgroup id to a logical one so that each of the 8 XCDs
// (which receive workgroups round-robin) walks a contiguous logical range
// and its private L2 sees neighbouring tiles.  A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
    const uint32_t kXcd = 8;
    uint32_t x = b % kXcd, i = b / kXcd, per = n / kXcd, rem = n % kXcd;
    return x * per + (x < rem ? x : rem) + i;
}

}  // namespace gpp
