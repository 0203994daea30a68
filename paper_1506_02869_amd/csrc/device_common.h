// Device primitives shared by the HIP kernels of the SMC-MPC engine:
// Philox4x32-10, uniform / normal transforms, precision-overloaded math and
// wave-level synchronisation.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// Philox purposes: third counter word is purpose | scenario << 8.
enum Purpose : uint32_t {
    P_INIT = 1, P_WIND = 2, P_RESAMPLE = 3, P_MOVE = 4, P_ACCEPT = 5, P_MALA = 6
};

struct Words4 { uint32_t w0, w1, w2, w3; };

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
// takes the 32x32->64 products of counter words 0 and 2 with the two round
// multipliers, mixes the high halves with the other two counter words and
// the key, and the key is advanced by the Weyl increments between rounds.
__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                           uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return Words4{c0, c1, c2, c3};
}

// Counter (element, iteration, purpose | scenario << 8, mpc step),
// key (seed low, seed high).
struct Stream {
    uint32_t c1, c2, c3, k0, k1;
};

__host__ __device__ inline Stream make_stream(uint64_t seed, int64_t mpc_step,
                                              int32_t iter, uint32_t purpose,
                                              int32_t scenario) {
    Stream s;
    s.c1 = (uint32_t)iter;
    s.c2 = (purpose & 0xFFu) | ((uint32_t)scenario << 8);
    s.c3 = (uint32_t)(uint64_t)mpc_step;
    s.k0 = (uint32_t)(seed & 0xFFFFFFFFull);
    s.k1 = (uint32_t)(seed >> 32);
    return s;
}

__device__ __forceinline__ Words4 draw(const Stream& s, uint32_t elem) {
    return philox10(elem, s.c1, s.c2, s.c3, s.k0, s.k1);
}

// u = ((a >> 6) 2^26 + (b >> 6) + 1/2) 2^-52 in (0, 1); every step exact.
__device__ __forceinline__ double uniform01(uint32_t a, uint32_t b) {
    return ((double)(a >> 6) * 67108864.0 + (double)(b >> 6) + 0.5) *
           2.220446049250313e-16;
}

// Box-Muller pair from one counter (u1 from words 0,1; u2 from words 2,3),
// evaluated in FP64 for every precision of the consumer.
__device__ __forceinline__ void normal_pair(const Words4& w, double& z0, double& z1) {
    const double u1 = uniform01(w.w0, w.w1);
    const double u2 = uniform01(w.w2, w.w3);
    const double r = sqrt(-2.0 * log(u1));
    const double th = 6.283185307179586 * u2;
    double s, c;
    sincos(th, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// ---- precision-overloaded math ---------------------------------------------
__device__ __forceinline__ float  m_sqrt(float x)  { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float  m_abs(float x)   { return fabsf(x); }
__device__ __forceinline__ double m_abs(double x)  { return fabs(x); }
__device__ __forceinline__ float  m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_floor(double x){ return floor(x); }
__device__ __forceinline__ float  m_sin(float x)   { return sinf(x); }
__device__ __forceinline__ double m_sin(double x)  { return sin(x); }
__device__ __forceinline__ float  m_atan2(float y, float x)   { return atan2f(y, x); }
__device__ __forceinline__ double m_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ void m_sincos(float x, float* s, float* c)   { sincosf(x, s, c); }
__device__ __forceinline__ void m_sincos(double x, double* s, double* c){ sincos(x, s, c); }
__device__ __forceinline__ float  m_exp(float x)   { return expf(x); }
__device__ __forceinline__ double m_exp(double x)  { return exp(x); }
__device__ __forceinline__ float  m_log(float x)   { return logf(x); }
__device__ __forceinline__ double m_log(double x)  { return log(x); }
__device__ __forceinline__ float  m_min(float a, float b)   { return fminf(a, b); }
__device__ __forceinline__ double m_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float  m_max(float a, float b)   { return fmaxf(a, b); }
__device__ __forceinline__ double m_max(double a, double b) { return fmax(a, b); }

template <typename R> struct Consts;
template <> struct Consts<float> {
    static constexpr float pi = 3.14159265358979323846f;
    static constexpr float two_pi = 6.28318530717958647692f;
    static constexpr float inv_two_pi = 0.15915494309189533577f;
    static constexpr float half_pi = 1.57079632679489661923f;
};
template <> struct Consts<double> {
    static constexpr double pi = 3.14159265358979323846;
    static constexpr double two_pi = 6.28318530717958647692;
    static constexpr double inv_two_pi = 0.15915494309189533577;
    static constexpr double half_pi = 1.57079632679489661923;
};

// Wave-level ordering point for LDS exchanges confined to one wavefront:
// a compiler fence around an instruction-scheduling barrier (LDS operations
// of one wave complete in issue order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace smc
