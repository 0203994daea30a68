// Per-element and per-workgroup bodies of the SMC kernels (Alg. 1), shared
// by the single-scenario launches and the batched launches so that both
// compute bit-identical results from the same inputs.
#pragma once

#include "engine.h"

namespace smc {

template <typename R>
__device__ __forceinline__ R to_real(double x) { return (R)x; }

// ---- particle initialisation: every normalised control ~ U(0, 1) ----------
__device__ __forceinline__ double init_value(const Stream& s, uint32_t e) {
    const Words4 w = draw(s, e);
    return uniform01(w.w0, w.w1);
}

// ---- wind normals: the pair (Z[g][2m], Z[g][2m + 1]) from counter m G + g -
template <typename R>
__device__ __forceinline__ void normals_at(const Stream& s, int G, int g, int m, R* dst) {
    const Words4 w = draw(s, (uint32_t)((int64_t)m * G + g));
    double z0, z1;
    normal_pair(w, z0, z1);
    dst[0] = to_real<R>(z0);
    dst[1] = to_real<R>(z1);
}

// ---- cost reduction (Sec. "Particle Costing", "Weight Scaling") ----------
// c_hat[t] = (1/M) sum_m cost[m PN + t] (Kahan-compensated FP64, sample
// order), feasible = all samples feasible, logw = -beta c_hat or -inf.
__device__ __forceinline__ void reduce_at(int64_t t, int64_t PN, int M,
                                          const double* __restrict__ cost,
                                          const uint8_t* __restrict__ feas, double beta,
                                          double* __restrict__ chat,
                                          uint8_t* __restrict__ feas_pn,
                                          double* __restrict__ logw) {
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

// ---- systematic resampling of one aircraft row (Sec. "Particle Resampling
// and Perturbation") -------------------------------------------------------
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

// One workgroup of RS_THREADS threads resamples row i of logw[P][N]:
// quantised weights floor(exp(lw - max) 2^(52 - ceil log2 P)), exact FP64
// inclusive scan into C[P], ancestors A[P] by searching the scan against the
// thresholds (k + U 2^-32) Q / P.  red, red2: RS_THREADS doubles of LDS.
__device__ __forceinline__ void resample_row(int P, int N, int i, const double* __restrict__ logw,
                                             uint32_t Uw, double* __restrict__ C,
                                             int32_t* __restrict__ A, double* ess_out,
                                             double* red, double* red2) {
    const int tid = threadIdx.x;
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
        if (ess_out && tid == 0) *ess_out = 0.0;
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

    if (ess_out) {
        __syncthreads();
        red[tid] = sw;
        red2[tid] = sw2;
        __syncthreads();
        for (int s = RS_THREADS / 2; s > 0; s >>= 1) {
            if (tid < s) { red[tid] += red[tid + s]; red2[tid] += red2[tid + s]; }
            __syncthreads();
        }
        if (tid == 0) *ess_out = red[0] * red[0] / red2[0];
    }
    __threadfence_block();
    __syncthreads();

    // 3) systematic ancestors on the exact scan: A[k] is the first index
    // whose C is above threshold k (P - 1 if none).  The thresholds grow
    // with k, so A is nondecreasing along the thread's run of k: each search
    // starts at the previous ancestor (every index below it is below the
    // new threshold too), walks up to 8 entries, then halves the rest.
    const uint64_t Q = (uint64_t)Qd;
    const uint64_t U = Uw;
    const uint64_t PP = (uint64_t)P;
    int lo = 0;
    for (int k = l0; k < l1; ++k) {
        int w = 0;
        while (lo < P - 1 && w < 8 && !above_threshold((uint64_t)C[lo], PP, (uint64_t)k, U, Q)) {
            ++lo;
            ++w;
        }
        if (w == 8 && lo < P - 1 && !above_threshold((uint64_t)C[lo], PP, (uint64_t)k, U, Q)) {
            int hi = P - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (above_threshold((uint64_t)C[mid], PP, (uint64_t)k, U, Q)) hi = mid;
                else lo = mid + 1;
            }
        }
        A[k] = lo;
    }
}

// ---- gather by ancestor + the paper's jitter move ------------------------
// u_out[k][i][d] = u_in[anc[i][k]][i][d], then Gaussian white noise clamped
// to the control box if jitter != 0; element e = (k N + i) D + d.
template <typename R>
__device__ __forceinline__ void gather_move_at(int64_t e, int P, int N, int D,
                                               const R* __restrict__ u_in,
                                               const int32_t* __restrict__ anc,
                                               R* __restrict__ u_out, const Stream& s,
                                               double sigma, int jitter) {
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

// ---- random-walk proposal: u' = reflect(u + sigma xi) into [0, 1] --------
// (reflection of the real line with period 2 keeps the density symmetric)
template <typename R>
__device__ __forceinline__ void propose_at(int64_t e, const R* __restrict__ u,
                                           R* __restrict__ up, const Stream& s, double sigma) {
    double z0, z1;
    normal_pair(draw(s, (uint32_t)e), z0, z1);
    const double v = (double)u[e] + sigma * z0;
    double r = v - 2.0 * floor(v * 0.5);
    if (r > 1.0) r = 2.0 - r;
    up[e] = to_real<R>(r);
}

// ---- the Langevin move in logit coordinates theta = logit(u) -------------
// The logit map takes the control box (0, 1)^D one-to-one onto R^D, so no
// proposal leaves the box.  Carried to theta, the tempered target gains the
// Jacobian prod u (1 - u) of u = logistic(theta), and its log-gradient in
// theta is g u (1 - u) + 1 - 2 u with g = coef * gsum the gradient in u
// (gsum: the adjoint's gradient summed over the wind samples; coef =
// -beta_J / M).  eps is a standard deviation in logit units.
__device__ __forceinline__ double logit_of(double u) { return log(u) - log1p(-u); }

__device__ __forceinline__ double logistic_of(double t) {
    const double e = exp(-fabs(t));
    return t >= 0.0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

// (eps^2 / 2) times that log-gradient at u
__device__ __forceinline__ double mala_drift_at(double u, double g, double eps) {
    return 0.5 * eps * eps * (g * u * (1.0 - u) + 1.0 - 2.0 * u);
}

// ---- Langevin proposal: u' = logistic(logit(u) + drift + eps xi) ----------
template <typename R>
__device__ __forceinline__ void mala_propose_at(int64_t e, const R* __restrict__ u,
                                                const double* __restrict__ gsum, double coef,
                                                double eps, const Stream& s, R* __restrict__ up) {
    double z0, z1;
    normal_pair(draw(s, (uint32_t)e), z0, z1);
    const double a = (double)u[e];
    up[e] = to_real<R>(logistic_of(logit_of(a) + mala_drift_at(a, coef * gsum[e], eps) + eps * z0));
}

// ---- Langevin decision of particle p: reject a proposal on a face of the
// box (u' rounded to 0 or 1 in the storage precision, where the carried
// target vanishes) or violating; accept one if the current particle
// violates; otherwise accept iff log U < sum_i logw' - sum_i logw
// + log q(theta | theta') - log q(theta' | theta) + log J(u') - log J(u),
// with theta, theta' the logits of the stored controls --------------------
template <typename R>
__device__ __forceinline__ int mala_decide_at(int p, int N, int D, const R* __restrict__ u,
                                              const R* __restrict__ up,
                                              const double* __restrict__ g,
                                              const double* __restrict__ gp_, double coef,
                                              double eps, const double* __restrict__ logw,
                                              const double* __restrict__ logw_prop,
                                              const Stream& s) {
    const int64_t base = (int64_t)p * N * D;
    const int64_t n = (int64_t)N * D;
    bool inside = true;
    double fwd = 0.0, bwd = 0.0, ljac = 0.0;
    for (int64_t e = 0; e < n; ++e) {
        const double a = (double)u[base + e], b = (double)up[base + e];
        if (!(b > 0.0 && b < 1.0)) {
            inside = false;
            break;
        }
        const double ta = logit_of(a), tb = logit_of(b);
        const double d1 = tb - ta - mala_drift_at(a, coef * g[base + e], eps);    // theta' | theta
        const double d2 = ta - tb - mala_drift_at(b, coef * gp_[base + e], eps);  // theta | theta'
        fwd += d1 * d1;
        bwd += d2 * d2;
        ljac += (log(b) + log1p(-b)) - (log(a) + log1p(-a));
    }
    double s_new = 0.0, s_old = 0.0;
    for (int i = 0; i < N; ++i) {
        s_new += logw_prop[(int64_t)p * N + i];
        s_old += logw[(int64_t)p * N + i];
    }
    if (!inside || s_new == -INFINITY) return 0;
    if (s_old == -INFINITY) return 1;
    const double lq = (fwd - bwd) / (2.0 * eps * eps) + ljac;
    const Words4 w = draw(s, (uint32_t)p);
    return log(uniform01(w.w0, w.w1)) < (s_new - s_old) + lq ? 1 : 0;
}

// ---- Metropolis decision of particle p on the joint target prod_i W_i ----
__device__ __forceinline__ int accept_decide_at(int p, int N, const double* __restrict__ logw,
                                                const double* __restrict__ logw_prop,
                                                const Stream& s) {
    double s_new = 0.0, s_old = 0.0;
    for (int i = 0; i < N; ++i) {
        s_new += logw_prop[(int64_t)p * N + i];
        s_old += logw[(int64_t)p * N + i];
    }
    if (s_new == -INFINITY) return 0;
    if (s_old == -INFINITY) return 1;
    const Words4 w = draw(s, (uint32_t)p);
    return log(uniform01(w.w0, w.w1)) < (s_new - s_old) ? 1 : 0;
}

// Replace an accepted particle's controls and per-aircraft rows (element e
// of the [P][N][D] controls; the first N elements of a particle carry its
// per-aircraft rows).
template <typename R>
__device__ __forceinline__ void accept_apply_at(int64_t e, int N, int D, R* __restrict__ u,
                                                const R* __restrict__ up,
                                                double* __restrict__ chat,
                                                const double* __restrict__ chat_prop,
                                                uint8_t* __restrict__ feas,
                                                const uint8_t* __restrict__ feas_prop,
                                                double* __restrict__ logw,
                                                const double* __restrict__ logw_prop,
                                                const int32_t* __restrict__ flags) {
    const int64_t per = (int64_t)N * D;
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

// ---- final selection (Sec. "Final Sample Selection") ---------------------
// Lexicographic best of (fewest violating aircraft, largest sum of
// -beta c_hat, lowest index) by one workgroup of 1024 threads; best[0] =
// index, best[1] = 1 if the best particle still violates.  sb, ss, sl: 1024
// entries of LDS each.
__device__ __forceinline__ void select_block(int P, int N, const double* __restrict__ logw,
                                             const double* __restrict__ chat, double beta,
                                             int32_t* __restrict__ best, int* sb, double* ss,
                                             int* sl) {
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

// Physical controls of the selected particle and its expected costs
// (cost[0] = sum over aircraft, cost[1 + i] = c_hat_i); one workgroup.
template <typename R>
__device__ __forceinline__ void write_result_block(int N, int S, const R* __restrict__ u,
                                                   const int32_t* __restrict__ best,
                                                   const double* __restrict__ chat,
                                                   const Ctrl3 box,
                                                   double* __restrict__ controls,
                                                   double* __restrict__ cost,
                                                   int32_t* __restrict__ status) {
    const int t = threadIdx.x;
    const int l = best[0];
    const int D = N * S * 3;
    const R* ub = u + (int64_t)l * D;
    for (int e = t; e < D; e += blockDim.x) {
        const int c = e % 3;
        const double lo = c == 0 ? box.lo[0] : (c == 1 ? box.lo[1] : box.lo[2]);
        const double sp = c == 0 ? box.sp[0] : (c == 1 ? box.sp[1] : box.sp[2]);
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

}  // namespace smc
