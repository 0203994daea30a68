// Per-step arithmetic of the rollout shared by its two kernel layouts:
// precision-dispatched elementary operations, angle wrapping, Kahan sums.
#pragma once

#include "engine.h"

namespace smc {

template <typename R> struct V2;
template <> struct V2<float> { typedef float2 t; };
template <> struct V2<double> { typedef double2 t; };
template <typename R> struct V4;
template <> struct V4<float> { typedef float4 t; };
template <> struct V4<double> { typedef double4 t; };

// Occupancy target (waves per SIMD) of the world-per-lane rollout per
// aircraft bucket: the state takes about 8 VGPRs per aircraft.
template <typename R, int NMAX>
constexpr int wm_waves() { return sizeof(R) == 4 ? (NMAX <= 4 ? 4 : (NMAX <= 10 ? 3 : 2)) : 1; }

// An aircraft that has landed is parked at x = kGoneX + i kGoneDX: far from
// every other aircraft, parked or not, so pair tests need no presence check.
constexpr double kGoneX = 1.0e9, kGoneDX = 1.0e8;

__device__ __forceinline__ float m_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double m_fma(double a, double b, double c) { return fma(a, b, c); }

// A wave-uniform real moved to scalar registers.
__device__ __forceinline__ float uniform_real(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uniform_real(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}

constexpr double kG0 = 9.80665;
constexpr double kRho0 = 1.225, kT0 = 288.15, kLapse = 0.0065, kRair = 287.05287;

// Elementary operations of the rollout.  FP64 (the reference precision) uses
// correctly rounded division / square root and the ocml transcendentals.
// FP32 uses the hardware reciprocal, square root, exp2, log2, sin and cos
// (about 1 ulp, sin/cos ~1e-6 absolute for |x| < 256 turns) and a polynomial
// arctangent (see fast_atan2): all far below the 1e-5 relative budget of the
// FP32 path, which the parity tests check against the FP64 oracle.
template <typename R> struct Ops;
template <> struct Ops<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double pow_pos(double b, double e) { return ::exp(e * ::log(b)); }
    static __device__ __forceinline__ void sincos(double x, double* s, double* c) { ::sincos(x, s, c); }
    static __device__ __forceinline__ double sin(double x) { return ::sin(x); }
    static __device__ __forceinline__ double atan2(double y, double x) { return ::atan2(y, x); }
    // atan2 for x >= 0 (the right half-plane)
    static __device__ __forceinline__ double atan2_xpos(double y, double x) { return ::atan2(y, x); }
};

// atan(t) for t in [0, 1] as t P(t^2), P of degree 7 fitted by iteratively
// reweighted least squares toward minimax (max error 4e-8 in exact
// arithmetic, 1.4e-7 evaluated in FP32); the quadrant follows from the
// signs and the magnitude order of (x, y).  fast_atan2_abs: the angle of
// (|x|, |y|) in [0, pi/2].
__device__ __forceinline__ float fast_atan2_abs(float ay, float ax) {
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(fmaxf(mx, 1e-30f));
    const float q = t * t;
    float p = -0.004054339602589607f;
    p = fmaf(p, q, 0.02186211571097374f);
    p = fmaf(p, q, -0.05591108277440071f);
    p = fmaf(p, q, 0.09642104804515839f);
    p = fmaf(p, q, -0.13908593356609344f);
    p = fmaf(p, q, 0.1994655877351761f);
    p = fmaf(p, q, -0.33329859375953674f);
    p = fmaf(p, q, 0.9999993443489075f);
    const float a = t * p;
    return ay > ax ? 1.57079632679489662f - a : a;
}
__device__ __forceinline__ float fast_atan2(float y, float x) {
    const float a = fast_atan2_abs(fabsf(y), fabsf(x));
    return copysignf(x < 0.f ? 3.14159265358979324f - a : a, y);
}

template <> struct Ops<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float pow_pos(float b, float e) {
        return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(b));
    }
    static __device__ __forceinline__ void sincos(float x, float* s, float* c) {
        *s = __sinf(x);
        *c = __cosf(x);
    }
    static __device__ __forceinline__ float sin(float x) { return __sinf(x); }
    static __device__ __forceinline__ float atan2(float y, float x) { return fast_atan2(y, x); }
    // atan2 for x >= 0 (+0 included): fast_atan2 without the left half-plane
    static __device__ __forceinline__ float atan2_xpos(float y, float x) {
        return copysignf(fast_atan2_abs(fabsf(y), x), y);
    }
};

template <typename R>
__device__ __forceinline__ R wrap_angle(R a) {
    return a - Consts<R>::two_pi * m_floor((a + Consts<R>::pi) * Consts<R>::inv_two_pi);
}

// v clamped to [lo, hi] (lo <= hi).  FP32: one v_med3_f32, which needs no
// canonicalisation of loop-invariant bounds (min / max in IEEE mode do).
template <typename R>
__device__ __forceinline__ R clampr(R v, R lo, R hi) { return m_min(m_max(v, lo), hi); }
template <>
__device__ __forceinline__ float clampr<float>(float v, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}

// max(v, lo) for a loop-invariant bound: a median with +inf in FP32.
template <typename R>
__device__ __forceinline__ R maxr(R v, R lo) { return m_max(v, lo); }
template <>
__device__ __forceinline__ float maxr<float>(float v, float lo) {
    return __builtin_amdgcn_fmed3f(v, lo, __builtin_inff());
}

// Kahan-compensated accumulation.
template <typename R>
__device__ __forceinline__ void kahan_add(R& sum, R& comp, R x) {
    const R y = x - comp;
    const R t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

}  // namespace smc
