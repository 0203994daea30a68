// Counter-based random draws of the SMC loop and the moves built on them:
// Philox words, particle initialisation, wind normals, resampling offsets,
// gather + jitter, random-walk proposals and Metropolis acceptance.
#include "smc_steps.h"

namespace smc {

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
    u[e] = to_real<R>(init_value(s, (uint32_t)e));
}

// Warm start of the receding-horizon loop (Sec. "Model Predictive Control",
// "Rolling Window": the window moved by the applied first control
// segment): element e = ((l N + i) S + s) 3 + c takes element e + 3 of the
// previous final population (segment s + 1) for s < S - 1; the last
// segment is the fresh initialisation's draw of element e.
template <typename R>
__global__ void k_warm_start(Stream s, int64_t count, int S, const R* __restrict__ prev,
                             R* __restrict__ u) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const int seg = (int)((e / 3) % S);
    u[e] = seg < S - 1 ? prev[e + 3] : to_real<R>(init_value(s, (uint32_t)e));
}

// Z[g][2m + c]: thread per (g, m) with m fastest so that the pair of
// components is one coalesced 2-element store; counter element m G + g.
template <typename R>
__global__ void k_wind_normals(Stream s, int G, int M, R* Z) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)G * M) return;
    const int m = (int)(t % M);
    const int g = (int)(t / M);
    normals_at<R>(s, G, g, m, Z + (int64_t)g * (2 * M) + 2 * m);
}

// Normals of the time-correlated wind model (Sec. "Wind Model", linear
// Gaussian model): thread per (g, m) runs u(0) = v(0), u(k) = a u(k-1) +
// b v(k) over the H steps in FP64 registers, v(k) the Box-Muller pair of
// counter (k M + m) G + g, and stores u(k) in column k M + m.  The factor
// applied afterwards is linear, so Qhat u(k) follows the paper's recursion
// W(k) = a W(k-1) + Q v(k) with Q = b Qhat.  Consecutive threads store
// consecutive pairs of one row.
template <typename R>
__global__ void k_wind_normals_ar1(Stream s, int G, int M, int H, double a, double b, R* Z) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)G * M) return;
    const int m = (int)(t % M);
    const int g = (int)(t / M);
    R* row = Z + (int64_t)g * 2 * ((int64_t)H * M);
    double u0 = 0.0, u1 = 0.0;
    for (int k = 0; k < H; ++k) {
        const int64_t col = (int64_t)k * M + m;
        double z0, z1;
        normal_pair(draw(s, (uint32_t)(col * G + g)), z0, z1);
        if (k == 0) {
            u0 = z0;
            u1 = z1;
        } else {
            const double p0 = a * u0, p1 = a * u1;
            u0 = p0 + b * z0;
            u1 = p1 + b * z1;
        }
        row[2 * col] = to_real<R>(u0);
        row[2 * col + 1] = to_real<R>(u1);
    }
}

// The same recursion with the vertical factor applied on the fly (nz
// divides 64): lane per (h, m, iz), the nz levels of a horizontal node in
// consecutive lanes of one wave, which exchange their u(k) by shuffles and
// store Y[h][col][iz] = sum_{j <= iz} Lz[iz][j] u_j(k) (FP64 sums), the
// input of the horizontal factor's product.  The normals are those of
// k_wind_normals_ar1 (counter (k M + m) G + g, g = h nz + iz).
template <typename R>
__global__ void k_wind_normals_ar1_levels(Stream s, int G, int M, int H, int nz, double a,
                                          double b, const double* __restrict__ Lz, R* Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // G M is a multiple of nz and nz divides 64: a level group is wholly in
    // or out of range, and wholly inside one wave
    if (t >= (int64_t)G * M) return;
    const int iz = (int)(t % nz);
    const int64_t r = t / nz;
    const int m = (int)(r % M);
    const int h = (int)(r / M);
    const int g = h * nz + iz;
    const int base = (int)(threadIdx.x & 63) - iz;
    const int64_t NC = 2 * (int64_t)H * M;
    R* yrow = Y + (int64_t)h * NC * nz + iz;
    double u0 = 0.0, u1 = 0.0;
    for (int k = 0; k < H; ++k) {
        const int64_t col = (int64_t)k * M + m;
        double z0, z1;
        normal_pair(draw(s, (uint32_t)(col * G + g)), z0, z1);
        if (k == 0) {
            u0 = z0;
            u1 = z1;
        } else {
            const double p0 = a * u0, p1 = a * u1;
            u0 = p0 + b * z0;
            u1 = p1 + b * z1;
        }
        double y0 = 0.0, y1 = 0.0;
        for (int j = 0; j < nz; ++j) {
            const double v0 = __shfl(u0, base + j, 64);
            const double v1 = __shfl(u1, base + j, 64);
            if (j <= iz) {
                const double l = Lz[iz * nz + j];
                y0 += l * v0;
                y1 += l * v1;
            }
        }
        yrow[(2 * col) * nz] = to_real<R>(y0);
        yrow[(2 * col + 1) * nz] = to_real<R>(y1);
    }
}

__global__ void k_resample_offsets(Stream s, int N, uint32_t* U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    U[i] = draw(s, (uint32_t)i).w0;
}

// Thread per element (k, i, d), d over the D = 3 S controls of an aircraft.
template <typename R>
__global__ void k_gather_move(int P, int N, int D, const R* __restrict__ u_in,
                              const int32_t* __restrict__ anc,
                              R* __restrict__ u_out, Stream s, double sigma,
                              int jitter) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)P * N * D) return;
    gather_move_at<R>(e, P, N, D, u_in, anc, u_out, s, sigma, jitter);
}

template <typename R>
__global__ void k_propose(int64_t count, const R* __restrict__ u,
                          R* __restrict__ up, Stream s, double sigma) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    propose_at<R>(e, u, up, s, sigma);
}

__global__ void k_accept_decide(int P, int N, const double* __restrict__ logw,
                                const double* __restrict__ logw_prop, Stream s,
                                int32_t* __restrict__ flags) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    flags[p] = accept_decide_at(p, N, logw, logw_prop, s);
}

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
    if (e >= (int64_t)P * N * D) return;
    accept_apply_at<R>(e, N, D, u, up, chat, chat_prop, feas, feas_prop, logw, logw_prop, flags);
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

hipError_t launch_warm_start(int prec, Stream s, int64_t count, int S, const void* prev,
                             void* u, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (prec == 0)
        hipLaunchKernelGGL(k_warm_start<double>, dim3(blocks_for(count, 256)), dim3(256), 0, st,
                           s, count, S, (const double*)prev, (double*)u);
    else
        hipLaunchKernelGGL(k_warm_start<float>, dim3(blocks_for(count, 256)), dim3(256), 0, st,
                           s, count, S, (const float*)prev, (float*)u);
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

hipError_t launch_wind_normals_ar1(int prec, Stream s, int G, int M, int H, double a, double b,
                                   void* Z, hipStream_t st) {
    const int64_t n = (int64_t)G * M;
    if (prec == 0)
        hipLaunchKernelGGL(k_wind_normals_ar1<double>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, s, G, M, H, a, b, (double*)Z);
    else
        hipLaunchKernelGGL(k_wind_normals_ar1<float>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, s, G, M, H, a, b, (float*)Z);
    return hipGetLastError();
}

hipError_t launch_wind_normals_ar1_levels(int prec, Stream s, int G, int M, int H, int nz,
                                          double a, double b, const double* Lz, void* Y,
                                          hipStream_t st) {
    if (nz < 1 || 64 % nz != 0 || G % nz != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)G * M;
    if (prec == 0)
        hipLaunchKernelGGL(k_wind_normals_ar1_levels<double>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, s, G, M, H, nz, a, b, Lz, (double*)Y);
    else
        hipLaunchKernelGGL(k_wind_normals_ar1_levels<float>, dim3(blocks_for(n, 256)), dim3(256),
                           0, st, s, G, M, H, nz, a, b, Lz, (float*)Y);
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
