// SMC weighting, resampling and selection kernels (Alg. 1; Sec. "Weight
// Scaling", "Particle Resampling and Perturbation", "Final Sample Selection").
#include <mutex>

#include "smc_steps.h"

namespace smc {

__global__ void k_reduce(int P, int M, int N, const double* __restrict__ cost,
                         const uint8_t* __restrict__ feas, double beta,
                         double* __restrict__ chat, uint8_t* __restrict__ feas_pn,
                         double* __restrict__ logw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t PN = (int64_t)P * N;
    if (t >= PN) return;
    reduce_at(t, PN, M, cost, feas, beta, chat, feas_pn, logw);
}

// The paper's literal weighting (Alg. 1 inner loop; Sec. "Weight Scaling"):
// every pass m multiplies the weight by the objective value 1 - cost_m and a
// violation zeroes it, so log W = sum_m log(1 - cost_m) (Kahan-compensated,
// pass order) or -inf; c_hat and feasibility as in k_reduce.
__global__ void k_reduce_product(int P, int M, int N, const double* __restrict__ cost,
                                 const uint8_t* __restrict__ feas, double* __restrict__ chat,
                                 uint8_t* __restrict__ feas_pn, double* __restrict__ logw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t PN = (int64_t)P * N;
    if (t >= PN) return;
    double sum = 0.0, comp = 0.0, ls = 0.0, lc = 0.0;
    int ok = 1, zero = 0;
    for (int m = 0; m < M; ++m) {
        const double x = cost[(int64_t)m * PN + t];
        const double y = x - comp;
        const double s = sum + y;
        comp = (s - sum) - y;
        sum = s;
        ok &= feas[(int64_t)m * PN + t];
        if (x >= 1.0) {
            zero = 1;
        } else {
            const double ly = log1p(-x) - lc;
            const double lt = ls + ly;
            lc = (lt - ls) - ly;
            ls = lt;
        }
    }
    chat[t] = sum / (double)M;
    feas_pn[t] = (uint8_t)ok;
    logw[t] = (ok && !zero) ? ls : -INFINITY;
}

// One workgroup per aircraft row i.
__global__ void __launch_bounds__(RS_THREADS) k_resample(int P, int N,
                                                         const double* __restrict__ logw,
                                                         const uint32_t* __restrict__ Uarr,
                                                         double* __restrict__ scan,
                                                         int32_t* __restrict__ anc,
                                                         double* __restrict__ ess) {
    __shared__ double red[RS_THREADS];
    __shared__ double red2[RS_THREADS];
    const int i = blockIdx.x;
    resample_row(P, N, i, logw, Uarr[i], scan + (int64_t)i * P, anc + (int64_t)i * P,
                 ess ? ess + i : nullptr, red, red2);
}

// Single workgroup.
__global__ void __launch_bounds__(1024) k_select(int P, int N, const double* __restrict__ logw,
                                                 const double* __restrict__ chat, double beta,
                                                 int32_t* __restrict__ best) {
    __shared__ int sb[1024];
    __shared__ double ss[1024];
    __shared__ int sl[1024];
    select_block(P, N, logw, chat, beta, best, sb, ss, sl);
}

template <typename R>
__global__ void k_write_result(int N, int S, const R* __restrict__ u,
                               const int32_t* __restrict__ best,
                               const double* __restrict__ chat, const Ctrl3 box,
                               double* __restrict__ controls, double* __restrict__ cost,
                               int32_t* __restrict__ status) {
    write_result_block<R>(N, S, u, best, chat, box, controls, cost, status);
}

hipError_t launch_reduce(int P, int M, int N, const double* cost, const uint8_t* feas,
                         double beta, double* chat, uint8_t* feas_pn, double* logw,
                         hipStream_t st) {
    const int64_t n = (int64_t)P * N;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, M, N,
                       cost, feas, beta, chat, feas_pn, logw);
    return hipGetLastError();
}

hipError_t launch_reduce_product(int P, int M, int N, const double* cost, const uint8_t* feas,
                                 double* chat, uint8_t* feas_pn, double* logw, hipStream_t st) {
    const int64_t n = (int64_t)P * N;
    hipLaunchKernelGGL(k_reduce_product, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, M,
                       N, cost, feas, chat, feas_pn, logw);
    return hipGetLastError();
}

hipError_t launch_resample(int P, int N, const double* logw, const uint32_t* U, double* scan,
                           int32_t* anc, double* ess, hipStream_t st) {
    hipLaunchKernelGGL(k_resample, dim3(N), dim3(RS_THREADS), 0, st, P, N, logw, U, scan, anc,
                       ess);
    return hipGetLastError();
}

// ---- resampling with a static workspace ------------------------------------
// The prefix-scan workspace of smc_k_resample_noalloc: a file-scope device
// array, so the call allocates nothing.  Each device holds its own copy
// (32 MiB) from the library's first use on it until the process ends.  Host
// code never passes the array's name to a kernel (in host code it is a
// host-side stand-in): the device address comes from hipGetSymbolAddress,
// once per device, with that device current.  The scan is written in full
// before it is read, so nothing needs clearing between calls; calls that
// overlap on one device share the array and race.
static __device__ __align__(256) double scratch[kStaticScanDoubles];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t launch_resample_static(int P, int N, const double* logw, const uint32_t* U,
                                  int32_t* anc, double* ess, hipStream_t st) {
    if (P < 1 || N < 1 || (int64_t)P * N > kStaticScanDoubles) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    double* scan = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            g_scratch_dev[dev] = static_cast<double*>(p);
        }
        scan = g_scratch_dev[dev];
    }
    return launch_resample(P, N, logw, U, scan, anc, ess, st);
}

hipError_t launch_select(int P, int N, const double* logw, const double* chat, double beta,
                         int32_t* best, hipStream_t st) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st, P, N, logw, chat, beta, best);
    return hipGetLastError();
}

hipError_t launch_write_result(int prec, int N, int S, const void* u, const int32_t* best,
                               const double* chat, const double* lo, const double* sp,
                               double* controls_out, double* cost_out, int32_t* status_out,
                               hipStream_t st) {
    Ctrl3 box;
    for (int c = 0; c < 3; ++c) { box.lo[c] = lo[c]; box.sp[c] = sp[c]; }
    if (prec == 0)
        hipLaunchKernelGGL(k_write_result<double>, dim3(1), dim3(256), 0, st, N, S,
                           (const double*)u, best, chat, box, controls_out, cost_out,
                           status_out);
    else
        hipLaunchKernelGGL(k_write_result<float>, dim3(1), dim3(256), 0, st, N, S,
                           (const float*)u, best, chat, box, controls_out, cost_out,
                           status_out);
    return hipGetLastError();
}

}  // namespace smc
