// Batched SMC kernels: the steps of Alg. 1 for every scenario of a batch in
// one launch each.  The grid's y index (or the row table) picks the
// scenario; the per-element arithmetic is the shared body of the
// single-scenario kernel, with that scenario's Philox streams, so each
// scenario's result is the one its own single-scenario run gives.  Every
// per-step input is read from device memory (table, step header), so a
// captured graph of these launches replays for any MPC step.
#include "smc_steps.h"

namespace smc {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_b_fill(uint32_t* __restrict__ p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}

template <typename R>
__global__ void k_b_init(const BatchScen* __restrict__ tab, const BatchStep* __restrict__ hdr,
                         R* __restrict__ u) {
    const BatchScen& sc = tab[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)sc.rp.P * sc.N * sc.D) return;
    const Stream s = make_stream(sc.seed, hdr->mpc_step, 0, P_INIT, sc.scen_id);
    u[sc.off_u + e] = to_real<R>(init_value(s, (uint32_t)e));
}

// Z[g][n 2M + 2m + c] for scenario n: the scenario's normals occupy a block
// of 2M columns of one matrix, so one GEMM with the shared factor serves
// the whole batch.
template <typename R>
__global__ void k_b_normals(const BatchScen* __restrict__ tab, const BatchStep* __restrict__ hdr,
                            int ns, int J, int G, int M, R* __restrict__ Z) {
    const int n = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)G * M) return;
    const BatchScen& sc = tab[n];
    const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_WIND, sc.scen_id);
    const int m = (int)(t % M);
    const int g = (int)(t / M);
    normals_at<R>(s, G, g, m, Z + (int64_t)g * ((int64_t)ns * 2 * M) + (int64_t)n * 2 * M + 2 * m);
}

__global__ void k_b_reduce(const BatchScen* __restrict__ tab, int J, double* __restrict__ chat,
                           uint8_t* __restrict__ feas_pn, double* __restrict__ logw) {
    const BatchScen& sc = tab[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t PN = (int64_t)sc.rp.P * sc.N;
    if (t >= PN) return;
    reduce_at(t, PN, sc.rp.M, sc.ra.cost, sc.ra.feas, sc.beta[J], chat + sc.off_pn,
              feas_pn + sc.off_pn, logw + sc.off_pn);
}

// Row r of the batch is aircraft r - off_n of scenario row_scen[r].
__global__ void k_b_resample_offsets(const BatchScen* __restrict__ tab,
                                     const BatchStep* __restrict__ hdr,
                                     const int32_t* __restrict__ row_scen, int rows, int J,
                                     uint32_t* __restrict__ U) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const BatchScen& sc = tab[row_scen[r]];
    const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_RESAMPLE, sc.scen_id);
    U[r] = draw(s, (uint32_t)(r - sc.off_n)).w0;
}

__global__ void __launch_bounds__(RS_THREADS) k_b_resample(const BatchScen* __restrict__ tab,
                                                           const int32_t* __restrict__ row_scen,
                                                           int P, const double* __restrict__ logw,
                                                           const uint32_t* __restrict__ U,
                                                           double* __restrict__ scan,
                                                           int32_t* __restrict__ anc) {
    __shared__ double red[RS_THREADS];
    __shared__ double red2[RS_THREADS];
    const int r = blockIdx.x;
    const BatchScen& sc = tab[row_scen[r]];
    resample_row(P, sc.N, r - sc.off_n, logw + sc.off_pn, U[r], scan + (int64_t)r * P,
                 anc + (int64_t)r * P, nullptr, red, red2);
}

template <typename R>
__global__ void k_b_gather_move(const BatchScen* __restrict__ tab,
                                const BatchStep* __restrict__ hdr, int J,
                                const R* __restrict__ u_in, const int32_t* __restrict__ anc,
                                R* __restrict__ u_out, int jitter) {
    const BatchScen& sc = tab[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P = sc.rp.P;
    if (e >= (int64_t)P * sc.N * sc.D) return;
    const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_MOVE, sc.scen_id);
    gather_move_at<R>(e, P, sc.N, sc.D, u_in + sc.off_u, anc + (int64_t)sc.off_n * P,
                      u_out + sc.off_u, s, sc.sigma_move, jitter);
}

template <typename R>
__global__ void k_b_propose(const BatchScen* __restrict__ tab, const BatchStep* __restrict__ hdr,
                            int J, const R* __restrict__ u, R* __restrict__ up) {
    const BatchScen& sc = tab[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)sc.rp.P * sc.N * sc.D) return;
    const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_MOVE, sc.scen_id);
    propose_at<R>(e, u + sc.off_u, up + sc.off_u, s, sc.sigma_move);
}

// Langevin proposal of every scenario (the adjoint's gradient g laid out
// like the particles).
template <typename R>
__global__ void k_b_mala_propose(const BatchScen* __restrict__ tab,
                                 const BatchStep* __restrict__ hdr, int J, const R* __restrict__ u,
                                 const double* __restrict__ g, R* __restrict__ up) {
    const BatchScen& sc = tab[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)sc.rp.P * sc.N * sc.D) return;
    const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_MALA, sc.scen_id);
    const double coef = -sc.beta[J] / (double)sc.rp.M;
    mala_propose_at<R>(e, u + sc.off_u, g + sc.off_u, coef, sc.mala_step, s, up + sc.off_u);
}

// Langevin decision per particle; accepted counts as for random-walk moves.
template <typename R>
__global__ void k_b_mala_decide(const BatchScen* __restrict__ tab,
                                const BatchStep* __restrict__ hdr, int J, const R* __restrict__ u,
                                const R* __restrict__ up, const double* __restrict__ g,
                                const double* __restrict__ g_prop, const double* __restrict__ logw,
                                const double* __restrict__ logw_prop, int32_t* __restrict__ flags,
                                uint32_t* __restrict__ accepted) {
    const int n = blockIdx.y;
    const BatchScen& sc = tab[n];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = sc.rp.P;
    int acc = 0;
    if (p < P) {
        const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_ACCEPT, sc.scen_id);
        const double coef = -sc.beta[J] / (double)sc.rp.M;
        acc = mala_decide_at<R>(p, sc.N, sc.D, u + sc.off_u, up + sc.off_u, g + sc.off_u,
                                g_prop + sc.off_u, coef, sc.mala_step, logw + sc.off_pn,
                                logw_prop + sc.off_pn, s);
        flags[(int64_t)n * P + p] = acc;
    }
    const int cnt = __popcll(__ballot(acc != 0));
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(accepted + n, (uint32_t)cnt);
}

// Decision per particle; accepted counts per scenario for the step's
// acceptance rate (one atomic per wave).
__global__ void k_b_accept_decide(const BatchScen* __restrict__ tab,
                                  const BatchStep* __restrict__ hdr, int J,
                                  const double* __restrict__ logw,
                                  const double* __restrict__ logw_prop,
                                  int32_t* __restrict__ flags, uint32_t* __restrict__ accepted) {
    const int n = blockIdx.y;
    const BatchScen& sc = tab[n];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = sc.rp.P;
    int acc = 0;
    if (p < P) {
        const Stream s = make_stream(sc.seed, hdr->mpc_step, J, P_ACCEPT, sc.scen_id);
        acc = accept_decide_at(p, sc.N, logw + sc.off_pn, logw_prop + sc.off_pn, s);
        flags[(int64_t)n * P + p] = acc;
    }
    const int cnt = __popcll(__ballot(acc != 0));
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(accepted + n, (uint32_t)cnt);
}

template <typename R>
__global__ void k_b_accept_apply(const BatchScen* __restrict__ tab, R* __restrict__ u,
                                 const R* __restrict__ up, double* __restrict__ chat,
                                 const double* __restrict__ chat_prop,
                                 uint8_t* __restrict__ feas, const uint8_t* __restrict__ feas_prop,
                                 double* __restrict__ logw, const double* __restrict__ logw_prop,
                                 const int32_t* __restrict__ flags) {
    const int n = blockIdx.y;
    const BatchScen& sc = tab[n];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int P = sc.rp.P;
    if (e >= (int64_t)P * sc.N * sc.D) return;
    const int64_t o = sc.off_pn;
    accept_apply_at<R>(e, sc.N, sc.D, u + sc.off_u, up + sc.off_u, chat + o, chat_prop + o,
                       feas + o, feas_prop + o, logw + o, logw_prop + o, flags + (int64_t)n * P);
}

__global__ void __launch_bounds__(1024) k_b_select(const BatchScen* __restrict__ tab, int J,
                                                   int P, const double* __restrict__ logw,
                                                   const double* __restrict__ chat,
                                                   int32_t* __restrict__ best) {
    __shared__ int sb[1024];
    __shared__ double ss[1024];
    __shared__ int sl[1024];
    const int n = blockIdx.x;
    const BatchScen& sc = tab[n];
    select_block(P, sc.N, logw + sc.off_pn, chat + sc.off_pn, sc.beta[J], best + 2 * n, sb, ss,
                 sl);
}

template <typename R>
__global__ void k_b_write_result(const BatchScen* __restrict__ tab, const R* __restrict__ u,
                                 const int32_t* __restrict__ best,
                                 const double* __restrict__ chat, double* __restrict__ controls,
                                 double* __restrict__ cost, int32_t* __restrict__ status) {
    const int n = blockIdx.x;
    const BatchScen& sc = tab[n];
    write_result_block<R>(sc.N, sc.S, u + sc.off_u, best + 2 * n, chat + sc.off_pn, sc.box,
                          controls + sc.off_ctrl, cost + sc.off_cost, status + n);
}

// ---- launchers ------------------------------------------------------------------

hipError_t launch_b_fill(uint32_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_fill, dim3(nblk(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_b_init(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                         int64_t max_count, void* u, hipStream_t st) {
    const dim3 grid(nblk(max_count, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_init<double>, grid, dim3(256), 0, st, tab, hdr, (double*)u);
    else
        hipLaunchKernelGGL(k_b_init<float>, grid, dim3(256), 0, st, tab, hdr, (float*)u);
    return hipGetLastError();
}

hipError_t launch_b_normals(int prec, const BatchScen* tab, const BatchStep* hdr, int ns, int J,
                            int G, int M, void* Z, hipStream_t st) {
    const dim3 grid(nblk((int64_t)G * M, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_normals<double>, grid, dim3(256), 0, st, tab, hdr, ns, J, G, M,
                           (double*)Z);
    else
        hipLaunchKernelGGL(k_b_normals<float>, grid, dim3(256), 0, st, tab, hdr, ns, J, G, M,
                           (float*)Z);
    return hipGetLastError();
}

hipError_t launch_b_reduce(const BatchScen* tab, int ns, int J, int64_t max_pn, double* chat,
                           uint8_t* feas_pn, double* logw, hipStream_t st) {
    hipLaunchKernelGGL(k_b_reduce, dim3(nblk(max_pn, 256), (unsigned)ns), dim3(256), 0, st, tab,
                       J, chat, feas_pn, logw);
    return hipGetLastError();
}

hipError_t launch_b_resample_offsets(const BatchScen* tab, const BatchStep* hdr,
                                     const int32_t* row_scen, int rows, int J, uint32_t* U,
                                     hipStream_t st) {
    hipLaunchKernelGGL(k_b_resample_offsets, dim3(nblk(rows, 256)), dim3(256), 0, st, tab, hdr,
                       row_scen, rows, J, U);
    return hipGetLastError();
}

hipError_t launch_b_resample(const BatchScen* tab, const int32_t* row_scen, int rows, int P,
                             const double* logw, const uint32_t* U, double* scan, int32_t* anc,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_b_resample, dim3((unsigned)rows), dim3(RS_THREADS), 0, st, tab,
                       row_scen, P, logw, U, scan, anc);
    return hipGetLastError();
}

hipError_t launch_b_gather_move(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                                int J, int64_t max_count, const void* u_in, const int32_t* anc,
                                void* u_out, int jitter, hipStream_t st) {
    const dim3 grid(nblk(max_count, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_gather_move<double>, grid, dim3(256), 0, st, tab, hdr, J,
                           (const double*)u_in, anc, (double*)u_out, jitter);
    else
        hipLaunchKernelGGL(k_b_gather_move<float>, grid, dim3(256), 0, st, tab, hdr, J,
                           (const float*)u_in, anc, (float*)u_out, jitter);
    return hipGetLastError();
}

hipError_t launch_b_propose(int prec, const BatchScen* tab, const BatchStep* hdr, int ns, int J,
                            int64_t max_count, const void* u, void* u_prop, hipStream_t st) {
    const dim3 grid(nblk(max_count, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_propose<double>, grid, dim3(256), 0, st, tab, hdr, J,
                           (const double*)u, (double*)u_prop);
    else
        hipLaunchKernelGGL(k_b_propose<float>, grid, dim3(256), 0, st, tab, hdr, J,
                           (const float*)u, (float*)u_prop);
    return hipGetLastError();
}

hipError_t launch_b_accept(int prec, const BatchScen* tab, const BatchStep* hdr, int ns, int J,
                           int P, int64_t max_count, void* u, const void* u_prop, double* chat,
                           const double* chat_prop, uint8_t* feas_pn, const uint8_t* feas_prop,
                           double* logw, const double* logw_prop, int32_t* flags,
                           uint32_t* accepted, hipStream_t st) {
    hipLaunchKernelGGL(k_b_accept_decide, dim3(nblk(P, 256), (unsigned)ns), dim3(256), 0, st,
                       tab, hdr, J, logw, logw_prop, flags, accepted);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(nblk(max_count, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_accept_apply<double>, grid, dim3(256), 0, st, tab, (double*)u,
                           (const double*)u_prop, chat, chat_prop, feas_pn, feas_prop, logw,
                           logw_prop, flags);
    else
        hipLaunchKernelGGL(k_b_accept_apply<float>, grid, dim3(256), 0, st, tab, (float*)u,
                           (const float*)u_prop, chat, chat_prop, feas_pn, feas_prop, logw,
                           logw_prop, flags);
    return hipGetLastError();
}

hipError_t launch_b_mala_propose(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                                int J, int64_t max_count, const void* u, const double* g,
                                void* u_prop, hipStream_t st) {
    const dim3 grid(nblk(max_count, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_mala_propose<double>, grid, dim3(256), 0, st, tab, hdr, J,
                           (const double*)u, g, (double*)u_prop);
    else
        hipLaunchKernelGGL(k_b_mala_propose<float>, grid, dim3(256), 0, st, tab, hdr, J,
                           (const float*)u, g, (float*)u_prop);
    return hipGetLastError();
}

hipError_t launch_b_mala_accept(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                                int J, int P, int64_t max_count, void* u, const void* u_prop,
                                const double* g, const double* g_prop, double* chat,
                                const double* chat_prop, uint8_t* feas_pn,
                                const uint8_t* feas_prop, double* logw, const double* logw_prop,
                                int32_t* flags, uint32_t* accepted, hipStream_t st) {
    const dim3 dgrid(nblk(P, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_mala_decide<double>, dgrid, dim3(256), 0, st, tab, hdr, J,
                           (const double*)u, (const double*)u_prop, g, g_prop, logw, logw_prop,
                           flags, accepted);
    else
        hipLaunchKernelGGL(k_b_mala_decide<float>, dgrid, dim3(256), 0, st, tab, hdr, J,
                           (const float*)u, (const float*)u_prop, g, g_prop, logw, logw_prop,
                           flags, accepted);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(nblk(max_count, 256), (unsigned)ns);
    if (prec == 0)
        hipLaunchKernelGGL(k_b_accept_apply<double>, grid, dim3(256), 0, st, tab, (double*)u,
                           (const double*)u_prop, chat, chat_prop, feas_pn, feas_prop, logw,
                           logw_prop, flags);
    else
        hipLaunchKernelGGL(k_b_accept_apply<float>, grid, dim3(256), 0, st, tab, (float*)u,
                           (const float*)u_prop, chat, chat_prop, feas_pn, feas_prop, logw,
                           logw_prop, flags);
    return hipGetLastError();
}

hipError_t launch_b_select(const BatchScen* tab, int ns, int J, int P, const double* logw,
                           const double* chat, int32_t* best, hipStream_t st) {
    hipLaunchKernelGGL(k_b_select, dim3((unsigned)ns), dim3(1024), 0, st, tab, J, P, logw, chat,
                       best);
    return hipGetLastError();
}

hipError_t launch_b_write_result(int prec, const BatchScen* tab, int ns, const void* u,
                                 const int32_t* best, const double* chat, double* controls_out,
                                 double* cost_out, int32_t* status_out, hipStream_t st) {
    if (prec == 0)
        hipLaunchKernelGGL(k_b_write_result<double>, dim3((unsigned)ns), dim3(256), 0, st, tab,
                           (const double*)u, best, chat, controls_out, cost_out, status_out);
    else
        hipLaunchKernelGGL(k_b_write_result<float>, dim3((unsigned)ns), dim3(256), 0, st, tab,
                           (const float*)u, best, chat, controls_out, cost_out, status_out);
    return hipGetLastError();
}

}  // namespace smc
