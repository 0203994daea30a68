/*
 * smc_kernels.h -- kernel-level entry points of the SMC-MPC engine.
 *
 * Each function runs exactly one step of the hot path on device buffers, so
 * that every step can be checked on its own against an independent
 * implementation fed with identical inputs.  smc_mpc_step() chains the same
 * kernels.
 *
 * Conventions (in addition to those of smc_mpc.h):
 *  - All array pointers are DEVICE pointers, caller-owned; `stream` is a
 *    hipStream_t passed as void*.  NULL is the null (legacy default) stream,
 *    which orders with every blocking stream (PyTorch's default stream is
 *    the null stream, handle 0), so inputs written there are complete before
 *    the library reads them and later work there waits for the outputs.
 *    Calls return after queueing the work; synchronise the stream (or queue
 *    later work on it) before reading outputs.
 *  - "real" arrays hold double for an SMC_FP64 context and float for an
 *    SMC_FP32 context.  Costs, log-weights and scans are double always.
 *  - Sizes are validated on the host before any launch (SMC_EINVAL).
 *  - Layouts (row-major):
 *      particles u      [P][N][S][3] real, normalised controls in [0, 1]
 *      wind normals Z   [G][2M]      real, column 2m+c = sample m, component c
 *      wind fields W    [M][G][2]    real
 *      rollout cost     [M][P][N]    double;  rollout feasibility same, uint8
 *      expected cost    [P][N]       double;  feasibility [P][N] uint8
 *      log-weights      [P][N]       double (-inf = violating aircraft)
 *      ancestors        [N][P]       int32
 *    with G = nx ny nz grid points, grid point g = (ix ny + iy) nz + iz.
 */
#ifndef SMC_KERNELS_H
#define SMC_KERNELS_H

#include <stdint.h>
#include "smc_mpc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 (Salmon et al., SC'11) words of n consecutive counters
 * (element e0 .. e0+n-1) of stream (seed, mpc_step, iter, purpose,
 * scenario).  out[4 n] uint32: the 4 words of each counter.  This replaces
 * the paper's stateful per-thread generator (Sec. "Kernel Design") by a
 * counter-based one, so any draw is reproducible from its coordinates. */
smc_status smc_k_philox(uint64_t seed, int64_t mpc_step, int32_t iter,
                        int32_t purpose, int32_t scenario, int64_t e0, int64_t n,
                        uint32_t* out, void* stream);

/* Alg. 1 initialisation (Sec. "Particles"): u[P][N][S][3] ~ U(0, 1) from the
 * INIT stream, element ((p N + i) S + s) 3 + c. */
smc_status smc_k_init_particles(smc_ctx* ctx, int64_t mpc_step, int32_t P,
                                void* u, void* stream);

/* Standard normals Z[G][2M] of iteration `iter` (WIND stream, element
 * m G + g, Box-Muller pair -> components x, y). */
smc_status smc_k_wind_normals(smc_ctx* ctx, int64_t mpc_step, int32_t iter,
                              void* Z, void* stream);

/* Wind fields W[m][g][c] = wind_mean[c] + sum_h Lchol[g][h] Z[h][2m+c]
 * (Sec. "Wind Model": Cholesky factor times Gaussian vector), with the
 * context's lower-triangular factor Lchol = sigma Lx (x) Ly (x) Lz.  Up to 16
 * grid levels the product is grouped by that structure: each horizontal
 * node's levels mixed by Lz, then sigma Lx (x) Ly applied by an MFMA GEMM
 * (the same product up to rounding order); above 16 levels, the dense
 * factor's MFMA GEMM.  Uses the context's scratch buffers: calls on one
 * context are ordered by their stream.  wind_mean: host [2]. */
smc_status smc_k_wind_gemm(smc_ctx* ctx, const void* Z, const double* wind_mean,
                           void* W, void* stream);

/* Copy of the context's dense factor Lchol[G][G] (real) into `out`. */
smc_status smc_k_wind_factor(smc_ctx* ctx, void* out, void* stream);

/* The wind fields of iteration `iter` under the context's wind model, as an
 * update draws them (Sec. "Wind Model").  SMC_WIND_SE: W[M][G][2], the
 * same as smc_k_wind_normals then smc_k_wind_gemm.  SMC_WIND_EXP_AR1:
 * W[H][M][G][2] for the H = horizon_max steps: the normals of every step
 * and sample (those of sample k M + m under the static numbering) go
 * through the time recursion u(k) = a u(k-1) + sqrt(1 - a^2) v(k), then
 * through the factor; the factor is linear, so step k's field is the
 * paper's W(k) plus wind_mean.  W: device, caller-allocated; the context's
 * normals buffer is the workspace (calls on one context run in stream
 * order).  wind_mean: host [2]. */
smc_status smc_k_wind_fields(smc_ctx* ctx, int64_t mpc_step, int32_t iter,
                             const double* wind_mean, void* W, void* stream);

/* Rollout of P particles under the fields W ([M][G][2], or [H][M][G][2]
 * for a context with the time-correlated wind: step k reads field k) (Sec. "Trajectory Planning",
 * eq. hor; Sec. "Constraint Handling"; eq. TO_init; Sec. "Particle Costing";
 * eq. avoidance): cost[M][P][N] (double), feas[M][P][N] (uint8).
 * states[N][6] double and k_active[N] int32 are device arrays.
 * steps (device uint64[128], may be NULL): simulated aircraft-steps are
 * added to slots 0..63 and separation tests with both aircraft present to
 * slots 64..127 (spread over the slots; sum each half). */
smc_status smc_k_rollout(smc_ctx* ctx, const void* u, int32_t P, const void* W,
                         const double* states, const int32_t* k_active,
                         int32_t horizon, double* cost, uint8_t* feas,
                         uint64_t* steps, void* stream);

/* Expected cost over the M wind samples (Kahan-compensated FP64 sum in
 * sample order), feasibility (all samples), log-weight -beta * c_hat or -inf
 * (Sec. "Weight Scaling").  chat, logw [P][N] double; feas_pn [P][N] uint8. */
smc_status smc_k_reduce(smc_ctx* ctx, int32_t P, const double* cost,
                        const uint8_t* feas, double beta, double* chat,
                        uint8_t* feas_pn, double* logw, void* stream);

/* The paper's literal weighting over M passes (Alg. 1 inner loop, Sec.
 * "Weight Scaling"): cost[M][P][N], feas[M][P][N] as smc_k_rollout writes
 * them for M samples (1 <= M <= the context's n_wind); c_hat and
 * feasibility as smc_k_reduce; logw = sum_m log(1 - cost_m)
 * (Kahan-compensated FP64, pass order), -inf if any pass violates or has
 * cost >= 1. */
smc_status smc_k_reduce_product(smc_ctx* ctx, int32_t P, int32_t M, const double* cost,
                                const uint8_t* feas, double* chat, uint8_t* feas_pn,
                                double* logw, void* stream);

/* First Philox word of the RESAMPLE stream for each aircraft row:
 * U[N] uint32. */
smc_status smc_k_resample_offsets(smc_ctx* ctx, int64_t mpc_step, int32_t iter,
                                  uint32_t* U, void* stream);

/* Per-aircraft systematic resampling (Sec. "Particle Resampling and
 * Perturbation"): for each row i, q_l = floor(exp(logw - max) 2^Kq) with
 * Kq = 52 - ceil(log2 P), exact FP64 inclusive scan C, ancestors
 * a_k = min{l : C_l P 2^32 > (k 2^32 + U_i) Q} in exact integer arithmetic;
 * identity for an all -inf row.  logw [P][N], U [N], anc [N][P] int32.
 * ess (device double[N], may be NULL): effective sample size per row. */
smc_status smc_k_resample(smc_ctx* ctx, int32_t P, const double* logw,
                          const uint32_t* U, int32_t* anc, double* ess,
                          void* stream);

/* The same resampling with no allocation and no context, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the prefix-scan workspace
 * is a static device array of 2^22 doubles (32 MiB) that each device holds
 * from the first call on it until the process ends; the call makes no
 * hipMalloc / hipFree and no allocating library call.  N in [1, 64], P >= 1,
 * N * P <= 2^22 (SMC_EINVAL otherwise, message in smc_last_error(NULL)).
 * Arguments and results as smc_k_resample (logw [P][N], U [N], anc [N][P],
 * ess [N] or NULL; device pointers; stream NULL = the null stream).  Every
 * call on a device shares its workspace: calls that may overlap on one
 * device (different streams, threads) race and must be serialised by the
 * caller. */
smc_status smc_k_resample_noalloc(int32_t N, int32_t P, const double* logw,
                                  const uint32_t* U, int32_t* anc, double* ess,
                                  void* stream);

/* Gather by ancestors, then (if jitter != 0) the paper's Gaussian white-noise
 * perturbation u += sigma_move xi (MOVE stream of `iter`), clamped to [0, 1]
 * (Alg. 1 resample / perturb).  u_in, u_out [P][N][S][3] real (distinct). */
smc_status smc_k_gather_move(smc_ctx* ctx, int32_t P, const void* u_in,
                             const int32_t* anc, void* u_out, int64_t mpc_step,
                             int32_t iter, int32_t jitter, void* stream);

/* Random-walk proposal u' = reflect(u + sigma_move xi) (MOVE stream),
 * reflection into [0, 1] keeps the proposal symmetric. */
smc_status smc_k_propose(smc_ctx* ctx, int32_t P, const void* u, void* u_prop,
                         int64_t mpc_step, int32_t iter, void* stream);

/* Metropolis acceptance on the joint particle (target prod_i W_i, final
 * selection rule of Sec. "Final Sample Selection"): reject a violating
 * proposal, accept a proposal if the current particle violates, otherwise
 * accept iff log U < sum_i logw' - sum_i logw (ACCEPT stream, element p).
 * Accepted rows of u, chat, feas_pn, logw are replaced by the proposal's.
 * accepted (device int32[P], may be NULL) receives the decisions. */
smc_status smc_k_accept(smc_ctx* ctx, int32_t P, void* u, const void* u_prop,
                        double* chat, const double* chat_prop,
                        uint8_t* feas_pn, const uint8_t* feas_prop,
                        double* logw, const double* logw_prop,
                        int64_t mpc_step, int32_t iter, int32_t* accepted,
                        void* stream);

/* Final selection (Sec. "Final Sample Selection"): the particle with the
 * largest sum of log-weights, lowest index on ties; if every particle has a
 * violating aircraft, the fewest violators first, then the largest sum of
 * -beta c_hat.  best[0] = index, best[1] = 1 if infeasible else 0. */
smc_status smc_k_select(smc_ctx* ctx, int32_t P, const double* logw,
                        const double* chat, double beta, int32_t* best,
                        void* stream);

/* Adjoint of the fuel + time part of the cost (build addition; the paper's
 * optimiser is derivative-free): grad[P][N][S][3] (double) =
 * d/du_norm sum_m cost_ft[m][p][i], the sum over the M wind samples of W of
 * the fuel element and the time-to-go element of each aircraft, by a
 * hand-written reverse sweep with state checkpoints every 25 steps.
 * Landing carries no derivative; clamps and max/min take the active branch.
 * Limits: S <= 16, horizon <= 400 (SMC_EINVAL). */
smc_status smc_k_rollout_grad(smc_ctx* ctx, const void* u, int32_t P, const void* W,
                              const double* states, const int32_t* k_active,
                              int32_t horizon, double* grad, void* stream);

/* Langevin proposal in logit coordinates theta = log(u / (1 - u)), which map
 * the control box (0, 1)^D one-to-one onto R^D:
 *   u' = logistic(theta + (eps^2/2) (g u (1 - u) + 1 - 2 u) + eps xi),
 * the drift being the log-gradient in theta of the tempered target carried
 * to logit coordinates (its Jacobian prod u (1 - u) included), with
 * g = -(beta/M) grad the gradient in u (grad as returned by
 * smc_k_rollout_grad), eps = the scenario's mala_step (a standard deviation
 * in logit units), xi from the MALA stream of `iter`.  u in (0, 1). */
smc_status smc_k_mala_propose(smc_ctx* ctx, int32_t P, const void* u,
                              const double* grad, double beta, void* u_prop,
                              int64_t mpc_step, int32_t iter, void* stream);

/* Metropolis-adjusted acceptance of the Langevin proposal with the full
 * target prod_i W_i: reject a proposal that rounds onto a face of the box
 * (u' = 0 or 1 in the context's precision) or violates, accept if the
 * current particle violates, otherwise accept iff
 * log U < sum_i logw' - sum_i logw + log q(theta|theta') - log q(theta'|theta)
 *         + sum log(u'(1 - u')) - sum log(u(1 - u))
 * (logits of the stored controls; ACCEPT stream, element p).  Accepted rows of u, chat, feas_pn, logw are replaced;
 * accepted[P] (device int32) receives the decisions. */
smc_status smc_k_mala_accept(smc_ctx* ctx, int32_t P, void* u, const void* u_prop,
                             const double* grad, const double* grad_prop, double beta,
                             double* chat, const double* chat_prop, uint8_t* feas_pn,
                             const uint8_t* feas_prop, double* logw,
                             const double* logw_prop, int64_t mpc_step, int32_t iter,
                             int32_t* accepted, void* stream);

/* Rollout kernel layout used by every pass of this context:
 *  0 automatic (world-per-lane for N <= 20; above, particle tile in FP32
 *    and aircraft-per-lane in FP64),
 *  1 aircraft-per-lane: one lane per (particle, sample, aircraft), the world's
 *    aircraft in consecutive lanes of a wavefront, positions exchanged in LDS;
 *  2 world-per-lane: one lane per (particle, sample) holding all N aircraft
 *    in registers (N <= 20);
 *  3 particle-per-wave (FP32, N <= 64): the lanes of a wavefront are 64 wind
 *    samples of one particle; each aircraft's wind-independent step (speed,
 *    thrust, fuel, mass, altitude, heading, unary checks) is computed once
 *    per particle and step, and only pairs within the vertical separation
 *    get the horizontal test (exact: the altitudes do not depend on the
 *    wind).  Uses the context's workspace for a sample-interleaved copy of
 *    the fields, so calls on one context must run in stream order.
 *  4 particle tile (FP32, N <= 64; the automatic choice above 20 aircraft
 *    in FP32): a wavefront holds 4 particles x 16 wind samples, a
 *    workgroup one block of 16 samples, so that the wind lookups of the
 *    workgroups on one XCD stay in one block of the fields; otherwise as 3.
 * All compute the same rollout; SMC_EINVAL for an unsupported choice. */
smc_status smc_set_rollout_layout(smc_ctx* ctx, int32_t layout);

#ifdef __cplusplus
}
#endif
#endif /* SMC_KERNELS_H */
