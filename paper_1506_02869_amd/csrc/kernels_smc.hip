// SMC weighting, resampling and selection kernels (Alg. 1; Sec. "Weight
// Scaling", "Particle Resampling and Perturbation", "Final Sample Selection").
#include "engine.h"

namespace smc {

// c_hat[p][i] = (1/M) sum_m cost[m][p][i] (Kahan-compensated FP64, sample
// order), feasible = all samples feasible, logw = -beta c_hat or -inf.
__global__ void k_reduce(int P, int M, int N, const double* __restrict__ cost,
                         const uint8_t* __restrict__ feas, double beta,
                         double* __restrict__ chat, uint8_t* __restrict__ feas_pn,
                         double* __restrict__ logw) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t PN = (int64_t)P * N;
    if (t >= PN) return;
    double sum = 0.0, comp = 0.0;
    int ok = 1;
    for (int m = 0; m < M; ++m) {
        const double x = cost[(int64_t)m * PN + t];
        const double y = x - comp;
        const double s = sum + y;
        comp = (s - sum) - y;
        sum = s;
        ok &= feas[(int64_t)m * PN + t];
    }
    const double c = sum / (double)M;
    chat[t] = c;
    feas_pn[t] = (uint8_t)ok;
    logw[t] = ok ? -beta * c : -INFINITY;
}

constexpr int RS_THREADS = 1024;

__device__ __forceinline__ void mul64x64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
    lo = a * b;
    hi = __umul64hi(a, b);
}

// C_l P 2^32 > (k 2^32 + U) Q, all operands exact integers, 128-bit compare.
__device__ __forceinline__ bool above_threshold(uint64_t C, uint64_t P, uint64_t k, uint64_t U,
                                                uint64_t Q) {
    uint64_t h1, l1, h2, l2;
    mul64x64(C, P, h1, l1);
    const uint64_t H1 = (h1 << 32) | (l1 >> 32);
    const uint64_t L1 = l1 << 32;
    mul64x64((k << 32) | U, Q, h2, l2);
    return (H1 > h2) || (H1 == h2 && L1 > l2);
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
    const int tid = threadIdx.x;
    double* C = scan + (int64_t)i * P;
    int32_t* A = anc + (int64_t)i * P;

    // 1) max log-weight of the row
    double mx = -INFINITY;
    for (int l = tid; l < P; l += RS_THREADS) mx = fmax(mx, logw[(int64_t)l * N + i]);
    red[tid] = mx;
    __syncthreads();
    for (int s = RS_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    if (mx == -INFINITY) {  // every particle violates: keep the population
        for (int l = tid; l < P; l += RS_THREADS) A[l] = l;
        if (ess && tid == 0) ess[i] = 0.0;
        return;
    }

    // 2) quantised weights, per-thread chunk sums (integers < 2^52: exact)
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    const double scale = ldexp(1.0, 52 - lg);
    const int chunk = (P + RS_THREADS - 1) / RS_THREADS;
    const int l0 = min(P, tid * chunk), l1 = min(P, l0 + chunk);
    double run = 0.0, sw = 0.0, sw2 = 0.0;
    for (int l = l0; l < l1; ++l) {
        const double w = exp(logw[(int64_t)l * N + i] - mx);
        run += floor(w * scale);
        C[l] = run;
        sw += w;
        sw2 += w * w;
    }
    red[tid] = run;
    __syncthreads();
    // inclusive scan of the chunk totals (Hillis-Steele; exact on integers)
    for (int off = 1; off < RS_THREADS; off <<= 1) {
        const double add = tid >= off ? red[tid - off] : 0.0;
        __syncthreads();
        red[tid] += add;
        __syncthreads();
    }
    const double offset = tid > 0 ? red[tid - 1] : 0.0;
    const double Qd = red[RS_THREADS - 1];
    for (int l = l0; l < l1; ++l) C[l] += offset;

    if (ess) {
        __syncthreads();
        red[tid] = sw;
        red2[tid] = sw2;
        __syncthreads();
        for (int s = RS_THREADS / 2; s > 0; s >>= 1) {
            if (tid < s) { red[tid] += red[tid + s]; red2[tid] += red2[tid + s]; }
            __syncthreads();
        }
        if (tid == 0) ess[i] = red[0] * red[0] / red2[0];
    }
    __threadfence_block();
    __syncthreads();

    // 3) systematic ancestors by binary search on the exact scan
    const uint64_t Q = (uint64_t)Qd;
    const uint64_t U = Uarr[i];
    const uint64_t PP = (uint64_t)P;
    for (int k = l0; k < l1; ++k) {
        int lo = 0, hi = P - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (above_threshold((uint64_t)C[mid], PP, (uint64_t)k, U, Q)) hi = mid;
            else lo = mid + 1;
        }
        A[k] = lo;
    }
}

// Final selection: lexicographic best of (fewest violating aircraft, largest
// sum of -beta c_hat, lowest index).  Single workgroup.
__global__ void __launch_bounds__(1024) k_select(int P, int N, const double* __restrict__ logw,
                                                 const double* __restrict__ chat, double beta,
                                                 int32_t* __restrict__ best) {
    __shared__ int sb[1024];
    __shared__ double ss[1024];
    __shared__ int sl[1024];
    const int tid = threadIdx.x;
    int bb = 1 << 30, bl = -1;
    double bs = -INFINITY;
    for (int l = tid; l < P; l += 1024) {
        int nbad = 0;
        double s = 0.0;
        for (int i = 0; i < N; ++i) {
            const double lw = logw[(int64_t)l * N + i];
            if (lw == -INFINITY) ++nbad;
            s += -beta * chat[(int64_t)l * N + i];
        }
        const bool better = (bl < 0) || (nbad < bb) || (nbad == bb && s > bs);
        if (better) { bb = nbad; bs = s; bl = l; }
    }
    sb[tid] = bb; ss[tid] = bs; sl[tid] = bl;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (tid < st) {
            const int ob = sb[tid + st], ol = sl[tid + st];
            const double os = ss[tid + st];
            bool take = false;
            if (ol >= 0) {
                if (sl[tid] < 0) take = true;
                else if (ob < sb[tid]) take = true;
                else if (ob == sb[tid] && os > ss[tid]) take = true;
                else if (ob == sb[tid] && os == ss[tid] && ol < sl[tid]) take = true;
            }
            if (take) { sb[tid] = ob; ss[tid] = os; sl[tid] = ol; }
        }
        __syncthreads();
    }
    if (tid == 0) {
        best[0] = sl[0];
        best[1] = sb[0] > 0 ? 1 : 0;
    }
}

template <typename R>
__global__ void k_write_result(int N, int S, const R* __restrict__ u,
                               const int32_t* __restrict__ best,
                               const double* __restrict__ chat, double lo0, double lo1,
                               double lo2, double sp0, double sp1, double sp2,
                               double* __restrict__ controls, double* __restrict__ cost,
                               int32_t* __restrict__ status) {
    const int t = threadIdx.x;
    const int l = best[0];
    const int D = N * S * 3;
    const R* ub = u + (int64_t)l * D;
    for (int e = t; e < D; e += blockDim.x) {
        const int c = e % 3;
        const double lo = c == 0 ? lo0 : (c == 1 ? lo1 : lo2);
        const double sp = c == 0 ? sp0 : (c == 1 ? sp1 : sp2);
        controls[e] = lo + (double)ub[e] * sp;
    }
    if (t == 0) {
        double tot = 0.0;
        for (int i = 0; i < N; ++i) {
            const double c = chat[(int64_t)l * N + i];
            cost[1 + i] = c;
            tot += c;
        }
        cost[0] = tot;
        if (status) status[0] = best[1] ? 1 : 0;
    }
}

hipError_t launch_reduce(int P, int M, int N, const double* cost, const uint8_t* feas,
                         double beta, double* chat, uint8_t* feas_pn, double* logw,
                         hipStream_t st) {
    const int64_t n = (int64_t)P * N;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, M, N,
                       cost, feas, beta, chat, feas_pn, logw);
    return hipGetLastError();
}

hipError_t launch_resample(int P, int N, const double* logw, const uint32_t* U, double* scan,
                           int32_t* anc, double* ess, hipStream_t st) {
    hipLaunchKernelGGL(k_resample, dim3(N), dim3(RS_THREADS), 0, st, P, N, logw, U, scan, anc,
                       ess);
    return hipGetLastError();
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
    if (prec == 0)
        hipLaunchKernelGGL(k_write_result<double>, dim3(1), dim3(256), 0, st, N, S,
                           (const double*)u, best, chat, lo[0], lo[1], lo[2], sp[0], sp[1],
                           sp[2], controls_out, cost_out, status_out);
    else
        hipLaunchKernelGGL(k_write_result<float>, dim3(1), dim3(256), 0, st, N, S,
                           (const float*)u, best, chat, lo[0], lo[1], lo[2], sp[0], sp[1],
                           sp[2], controls_out, cost_out, status_out);
    return hipGetLastError();
}

}  // namespace smc
