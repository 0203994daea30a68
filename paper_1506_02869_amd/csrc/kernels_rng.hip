// Counter-based random draws of the SMC loop and the moves built on them:
// Philox words, particle initialisation, wind normals, resampling offsets,
// gather + jitter, random-walk proposals and Metropolis acceptance.
#include "engine.h"

namespace smc {

template <typename R>
__device__ __forceinline__ R to_real(double x) { return (R)x; }

__global__ void k_philox_words(Stream s, uint32_t e0, int64_t n, uint32_t* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const Words4 w = draw(s, e0 + (uint32_t)t);
    uint4* o = reinterpret_cast<uint4*>(out);
    o[t] = make_uint4(w.w0, w.w1, w.w2, w.w3);
}

// Alg. 1 initialisation: every normalised control ~ U(0, 1).
template <typename R>
__global__ void k_init_particles(Stream s, int64_t count, R* u) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const Words4 w = draw(s, (uint32_t)e);
    u[e] = to_real<R>(uniform01(w.w0, w.w1));
}

// Z[g][2m + c]: thread per (g, m) with m fastest so that the pair of
// components is one coalesced 2-element store; counter element m G + g.
template <typename R>
__global__ void k_wind_normals(Stream s, int G, int M, R* Z) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)G * M) return;
    const int m = (int)(t % M);
    const int g = (int)(t / M);
    const Words4 w = draw(s, (uint32_t)((int64_t)m * G + g));
    double z0, z1;
    normal_pair(w, z0, z1);
    R* dst = Z + (int64_t)g * (2 * M) + 2 * m;
    dst[0] = to_real<R>(z0);
    dst[1] = to_real<R>(z1);
}

__global__ void k_resample_offsets(Stream s, int N, uint32_t* U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    U[i] = draw(s, (uint32_t)i).w0;
}

// u_out[k][i][:] = u_in[anc[i][k]][i][:], then the paper's Gaussian
// white-noise perturbation (clamped to the control box) if jitter != 0.
// Thread per element (k, i, d), d over the D = 3 S controls of an aircraft.
template <typename R>
__global__ void k_gather_move(int P, int N, int D, const R* __restrict__ u_in,
                              const int32_t* __restrict__ anc,
                              R* __restrict__ u_out, Stream s, double sigma,
                              int jitter) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)P * N * D;
    if (e >= total) return;
    const int d = (int)(e % D);
    const int64_t ki = e / D;
    const int i = (int)(ki % N);
    const int k = (int)(ki / N);
    const int src = anc[(int64_t)i * P + k];
    double v = (double)u_in[((int64_t)src * N + i) * D + d];
    if (jitter) {
        double z0, z1;
        normal_pair(draw(s, (uint32_t)e), z0, z1);
        v = fmin(fmax(v + sigma * z0, 0.0), 1.0);
    }
    u_out[e] = to_real<R>(v);
}

// u' = reflect(u + sigma xi): reflection of the real line into [0, 1]
// (period 2), so the proposal density stays symmetric.
template <typename R>
__global__ void k_propose(int64_t count, const R* __restrict__ u,
                          R* __restrict__ up, Stream s, double sigma) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double z0, z1;
    normal_pair(draw(s, (uint32_t)e), z0, z1);
    const double v = (double)u[e] + sigma * z0;
    double r = v - 2.0 * floor(v * 0.5);
    if (r > 1.0) r = 2.0 - r;
    up[e] = to_real<R>(r);
}

// Metropolis decision per particle on the joint target prod_i W_i.
__global__ void k_accept_decide(int P, int N, const double* __restrict__ logw,
                                const double* __restrict__ logw_prop, Stream s,
                                int32_t* __restrict__ flags) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s_new = 0.0, s_old = 0.0;
    for (int i = 0; i < N; ++i) {
        s_new += logw_prop[(int64_t)p * N + i];
        s_old += logw[(int64_t)p * N + i];
    }
    int acc;
    if (s_new == -INFINITY) {
        acc = 0;
    } else if (s_old == -INFINITY) {
        acc = 1;
    } else {
        const Words4 w = draw(s, (uint32_t)p);
        acc = log(uniform01(w.w0, w.w1)) < (s_new - s_old) ? 1 : 0;
    }
    flags[p] = acc;
}

// Replace accepted particles' controls and per-aircraft rows.
template <typename R>
__global__ void k_accept_apply(int P, int N, int D, R* __restrict__ u,
                               const R* __restrict__ up,
                               double* __restrict__ chat,
                               const double* __restrict__ chat_prop,
                               uint8_t* __restrict__ feas,
                               const uint8_t* __restrict__ feas_prop,
                               double* __restrict__ logw,
                               const double* __restrict__ logw_prop,
                               const int32_t* __restrict__ flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)N * D;
    if (e >= (int64_t)P * per) return;
    const int p = (int)(e / per);
    if (!flags[p]) return;
    u[e] = up[e];
    const int64_t r = e - (int64_t)p * per;
    if (r < N) {
        const int64_t j = (int64_t)p * N + r;
        chat[j] = chat_prop[j];
        feas[j] = feas_prop[j];
        logw[j] = logw_prop[j];
    }
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_philox_words(Stream s, uint32_t e0, int64_t n, uint32_t* out,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_words, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       s, e0, n, out);
    return hipGetLastError();
}

hipError_t launch_init_particles(int prec, Stream s, int64_t count, void* u,
                                 hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_init_particles<double>, dim3(blocks_for(count, 256)),
                           dim3(256), 0, st, s, count, (double*)u);
    else
        hipLaunchKernelGGL(k_init_particles<float>, dim3(blocks_for(count, 256)),
                           dim3(256), 0, st, s, count, (float*)u);
    return hipGetLastError();
}

hipError_t launch_wind_normals(int prec, Stream s, int G, int M, void* Z,
                               hipStream_t st) {
    const int64_t n = (int64_t)G * M;
    if (prec == 0)
        hipLaunchKernelGGL(k_wind_normals<double>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, s, G, M, (double*)Z);
    else
        hipLaunchKernelGGL(k_wind_normals<float>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, s, G, M, (float*)Z);
    return hipGetLastError();
}

hipError_t launch_resample_offsets(Stream s, int N, uint32_t* U, hipStream_t st) {
    hipLaunchKernelGGL(k_resample_offsets, dim3(1), dim3(64), 0, st, s, N, U);
    return hipGetLastError();
}

hipError_t launch_gather_move(int prec, int P, int N, int D, const void* u_in,
                              const int32_t* anc, void* u_out, Stream s,
                              double sigma, int jitter, hipStream_t st) {
    const int64_t n = (int64_t)P * N * D;
    if (prec == 0)
        hipLaunchKernelGGL(k_gather_move<double>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, P, N, D, (const double*)u_in, anc, (double*)u_out,
                           s, sigma, jitter);
    else
        hipLaunchKernelGGL(k_gather_move<float>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, P, N, D, (const float*)u_in, anc, (float*)u_out,
                           s, sigma, jitter);
    return hipGetLastError();
}

hipError_t launch_propose(int prec, int64_t count, const void* u, void* u_prop,
                          Stream s, double sigma, hipStream_t st) {
    if (prec == 0)
        hipLaunchKernelGGL(k_propose<double>, dim3(blocks_for(count, 256)), dim3(256),
                           0, st, count, (const double*)u, (double*)u_prop, s, sigma);
    else
        hipLaunchKernelGGL(k_propose<float>, dim3(blocks_for(count, 256)), dim3(256),
                           0, st, count, (const float*)u, (float*)u_prop, s, sigma);
    return hipGetLastError();
}

hipError_t launch_accept_apply(int prec, int P, int N, int D, void* u, const void* u_prop,
                               double* chat, const double* chat_prop, uint8_t* feas_pn,
                               const uint8_t* feas_prop, double* logw, const double* logw_prop,
                               const int32_t* flags, hipStream_t st) {
    const int64_t n = (int64_t)P * N * D;
    if (prec == 0)
        hipLaunchKernelGGL(k_accept_apply<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, P,
                           N, D, (double*)u, (const double*)u_prop, chat, chat_prop, feas_pn,
                           feas_prop, logw, logw_prop, flags);
    else
        hipLaunchKernelGGL(k_accept_apply<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, P,
                           N, D, (float*)u, (const float*)u_prop, chat, chat_prop, feas_pn,
                           feas_prop, logw, logw_prop, flags);
    return hipGetLastError();
}

hipError_t launch_accept(int prec, int P, int N, int D, void* u,
                         const void* u_prop, double* chat,
                         const double* chat_prop, uint8_t* feas_pn,
                         const uint8_t* feas_prop, double* logw,
                         const double* logw_prop, Stream s, int32_t* accepted,
                         int32_t* flags, hipStream_t st) {
    int32_t* f = accepted ? accepted : flags;
    hipLaunchKernelGGL(k_accept_decide, dim3(blocks_for(P, 256)), dim3(256), 0, st,
                       P, N, logw, logw_prop, s, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)P * N * D;
    if (prec == 0)
        hipLaunchKernelGGL(k_accept_apply<double>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, P, N, D, (double*)u, (const double*)u_prop, chat,
                           chat_prop, feas_pn, feas_prop, logw, logw_prop, f);
    else
        hipLaunchKernelGGL(k_accept_apply<float>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, P, N, D, (float*)u, (const float*)u_prop, chat,
                           chat_prop, feas_pn, feas_prop, logw, logw_prop, f);
    return hipGetLastError();
}

}  // namespace smc
