/*
 * smc_batch.h -- C ABI of the batched SMC-MPC engine: many independent MPC
 * scenarios (terminal areas, or one area under several traffic hypotheses)
 * solved by one sequence of launches per MPC update.
 *
 * Each scenario runs the SMC loop of Alg. 1 (Sec. "Sequential Monte Carlo
 * Optimisation") exactly as smc_mpc_step() runs it for that scenario alone:
 * same Philox streams (seed, scenario_id), same arithmetic, so a scenario's
 * returned controls and costs are bit-identical to its single-scenario run.
 * What batching changes is the launch structure:
 *  - the rollout is one persistent launch per aircraft bucket (N <= 2, 4, 6,
 *    8, 10, 12, 16, 20) whose waves take work items (64 worlds of one
 *    scenario) from an atomic queue ordered by decreasing N^2 H;
 *  - the wind fields of all scenarios come from one GEMM with the shared
 *    Cholesky factor (all scenarios share the grid, box and covariance);
 *  - every other step is one launch over all scenarios;
 *  - the whole update can be captured once in a HIP graph and replayed for
 *    every later update (per-update inputs are read from device memory).
 * The paper runs one scenario per solve; the batched form is an addition.
 *
 * Conventions are those of smc_mpc.h (caller-owned arrays, negative status
 * codes leave outputs untouched, host validation before device work, one
 * batch per host thread / stream).  Per-scenario arrays are concatenated in
 * scenario order: states [sum N_s][6], k_active [sum N_s], wind_mean
 * [n_scen][2], horizons [n_scen], controls [sum N_s S_s 3] (scenario s's
 * N_s x S_s x 3 block after those of scenarios 0..s-1), expected costs
 * [sum (1 + N_s)] (total, then per aircraft, per scenario), status [n_scen].
 */
#ifndef SMC_BATCH_H
#define SMC_BATCH_H

#include <stdint.h>

#include "smc_mpc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smc_batch smc_batch;

#define SMC_BATCH_BUCKETS 8      /* aircraft buckets N <= 2,4,6,8,10,12,16,20 */
#define SMC_BATCH_MAX_AIRCRAFT 20
#define SMC_BATCH_MAX_SCENARIOS 4096

/* Launch shape of the persistent rollout, per aircraft bucket.  Any value
 * gives the same results; only the speed differs.
 *  block[b]: lanes per workgroup, 64, 128 or 256 (0 = default: 256 in FP32,
 *     128 in FP64); the segment's staged controls, NMAX x 3 x block reals,
 *     must fit 64 KB of LDS (smc_batch_set_tuning rejects shapes that do not).
 *  grid_mult[b]: workgroups = resident capacity of the chip x grid_mult
 *     (1..4; 0 = default 1).
 *  order: 0 = items by decreasing N^2 H (default), 1 = scenario order. */
typedef struct {
    int32_t block[SMC_BATCH_BUCKETS];
    int32_t grid_mult[SMC_BATCH_BUCKETS];
    int32_t order;
} smc_batch_tuning;

/* Diagnostics of one batched update (optional output). */
typedef struct {
    int32_t n_scenarios;
    int32_t iterations;        /* weighting passes per scenario (= n_iters)     */
    int64_t aircraft_steps;    /* simulated aircraft-steps, all scenarios       */
    int64_t pair_tests;        /* separation tests with both aircraft present   */
    double ms_total;           /* device time of the update (events)            */
    double accept_rate;        /* mean MH acceptance (0 for jitter)             */
    double feasible_frac;      /* feasible (particle, aircraft) rows, last pass */
    int32_t graph;             /* 1 if the update replayed the captured graph   */
    int32_t rollout_launches;  /* persistent rollout launches in the update     */
    int32_t rollout_passes;    /* rollout passes (all buckets) in the update    */
    double ms_rollout;         /* summed duration of the rollout passes (device
                                  events; 0 when the update replayed a graph)  */
} smc_batch_info;

/* Create a batch of n_scen (1..SMC_BATCH_MAX_SCENARIOS) scenarios.  Each
 * scenario is validated as by smc_mpc_init(); across the batch they must
 * share n_particles, n_wind, n_iters, precision, move (any of SMC_MOVE_*),
 * grid_n, box, wind_sigma, wind_ell and wind_nugget, and have at most
 * SMC_BATCH_MAX_AIRCRAFT aircraft.  Everything else (aircraft, N, S,
 * horizon_max, costs, limits, kappa, sigma_move, mala_step, seed,
 * scenario_id) may differ.  With SMC_MOVE_MALA every iteration adds two
 * adjoint launches per scenario (gradients of the particles and of the
 * proposals), and a captured graph is re-captured when the horizons change.
 * Errors: SMC_EINVAL (message names the scenario), SMC_ENOTSPD, SMC_ENOMEM,
 * SMC_EDEVICE; *out is NULL on error. */
smc_status smc_batch_init(const smc_scenario* scenarios, int32_t n_scen, smc_batch** out);

/* One MPC update of every scenario (host arrays, synchronous).  horizons[s]
 * in [S_s, horizon_max_s]; status_out[s] = SMC_OK or SMC_INFEASIBLE.  The
 * return value is SMC_INFEASIBLE if any scenario is, else SMC_OK.
 * info may be NULL. */
smc_status smc_batch_step(smc_batch* b, int64_t mpc_step, const double* states,
                          const int32_t* k_active, const double* wind_mean,
                          const int32_t* horizons, double* controls_out,
                          double* exp_cost_out, int32_t* status_out, smc_batch_info* info);

/* Device-pointer form: states, k_active, controls_out, exp_cost_out and
 * status_out are device pointers (status_out may be NULL); wind_mean and
 * horizons are host arrays.  Work is queued on `stream` (hipStream_t; NULL =
 * the null stream, ordered with every blocking stream such as PyTorch's
 * default stream); without info the call does not wait for the device
 * and returns SMC_OK (per-scenario status in status_out). */
smc_status smc_batch_step_dev(smc_batch* b, int64_t mpc_step, const double* d_states,
                              const int32_t* d_k_active, const double* wind_mean,
                              const int32_t* horizons, double* d_controls_out,
                              double* d_exp_cost_out, int32_t* d_status_out,
                              smc_batch_info* info, void* stream);

/* Capture the update in a HIP graph on its next call and replay it on later
 * calls (enable = 1), or launch kernel by kernel (0, default).  A change of
 * tuning drops the captured graph. */
smc_status smc_batch_set_graph(smc_batch* b, int32_t enable);

smc_status smc_batch_get_tuning(const smc_batch* b, smc_batch_tuning* out);
/* Validates every field; zero fields take the defaults. */
smc_status smc_batch_set_tuning(smc_batch* b, const smc_batch_tuning* t);

/* Time the persistent rollout of each bucket present in the batch for every
 * candidate launch shape (block 64 / 128 / 256 x grid_mult 1 / 2) on the
 * update's first wind fields and particles (inputs as for smc_batch_step),
 * keep the fastest (median of `reps` >= 1 timings), install it and copy it
 * to *out (may be NULL).  Synchronous. */
smc_status smc_batch_autotune(smc_batch* b, int64_t mpc_step, const double* states,
                              const int32_t* k_active, const double* wind_mean,
                              const int32_t* horizons, int32_t reps, smc_batch_tuning* out);

/* Work plan of the persistent rollout (host only, no device needed): for
 * scenario sizes n_aircraft[n_scen] and horizons[n_scen] with L particles
 * and M wind samples, the items of bucket b are item_scen / item_world0
 * [bucket_start[b] .. bucket_start[b] + bucket_count[b]), each 64 worlds
 * (world = l + L m) of one scenario.  order as in smc_batch_tuning.
 * Returns SMC_EINVAL if capacity is below the item count, which is
 * sum_s ceil(L M / 64) (also returned in *n_items, which may be NULL). */
smc_status smc_batch_plan(int32_t n_scen, const int32_t* n_aircraft, const int32_t* horizons,
                          int32_t n_particles, int32_t n_wind, int32_t order,
                          int32_t* bucket_start, int32_t* bucket_count, int32_t* item_scen,
                          int32_t* item_world0, int64_t capacity, int64_t* n_items);

/* Message of the last failing call on b (or of the last failing
 * smc_batch_init / smc_batch_plan when b is NULL). */
const char* smc_batch_last_error(const smc_batch* b);

/* Release the batch and its device memory.  NULL is a no-op. */
void smc_batch_destroy(smc_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* SMC_BATCH_H */
