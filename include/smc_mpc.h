/*
 * smc_mpc.h -- C ABI of the MI355X SMC-MPC rollout engine.
 *
 * One call of smc_mpc_step() solves one MPC update of a terminal-area traffic
 * scenario with Sequential Monte Carlo optimisation (Alg. 1 of Eele &
 * Maciejowski, "Sequential Monte Carlo Optimisation for Air Traffic
 * Management", CUED/F-INFENG/TR.693): particles of per-segment control
 * sequences for all aircraft are rolled out under sampled wind fields, scored,
 * weighted per aircraft, resampled per aircraft and moved, over annealed
 * iterations; the best particle's controls and expected cost are returned
 * (Sec. "Model Predictive Control": the whole sequence over the horizon is
 * returned, only its first part is applied by the caller).
 *
 * Conventions
 *  - Every array argument is caller-owned; the library copies what it needs.
 *    Functions with the _dev suffix take device pointers and a hipStream_t
 *    (passed as void*; NULL = the null stream, which orders with every
 *    blocking stream, e.g. PyTorch's default stream), never free caller
 *    memory and may return before the work completes (outputs are valid
 *    after the stream is synchronised or to later work on that stream).
 *  - Host-pointer functions are synchronous.
 *  - Errors are negative smc_status codes; outputs are then left untouched.
 *    Argument validation happens on the host before any device work.
 *    smc_last_error() returns a message for the last failing call on a ctx.
 *  - SMC_INFEASIBLE (positive) is a warning: outputs are valid and hold the
 *    particle with the fewest violating aircraft.
 *  - One context per host thread / stream; a context is not thread-safe.
 *  - Units are SI, angles in radians. Arrays are row-major (C order).
 */
#ifndef SMC_MPC_H
#define SMC_MPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smc_ctx smc_ctx;

typedef enum {
    SMC_OK = 0,
    SMC_INFEASIBLE = 1, /* warning: no particle without a violating aircraft */
    SMC_EINVAL = -1,    /* invalid argument or scenario                      */
    SMC_ENOMEM = -2,    /* device allocation failed                          */
    SMC_EDEVICE = -3,   /* HIP runtime or kernel error                       */
    SMC_ENOTSPD = -4    /* wind covariance factorisation failed              */
} smc_status;

enum { SMC_ARRIVAL = 0, SMC_DEPARTURE = 1 };
enum { SMC_FP64 = 0, SMC_FP32 = 1 };
/* moves after weighting: the paper's clamped Gaussian jitter after
 * resampling; random-walk Metropolis; Metropolis-adjusted Langevin with the
 * gradient of the fuel + time cost (both Metropolis forms act before
 * resampling, with the joint target prod_i W_i) */
enum { SMC_MOVE_JITTER = 0, SMC_MOVE_RWMH = 1, SMC_MOVE_MALA = 2 };
/* Wind models: a static squared-exponential field per sample, or the paper's
 * exponential covariance with its time recursion (one field per step). */
enum { SMC_WIND_SE = 0, SMC_WIND_EXP_AR1 = 1 };
/* Weighting: tempered (log W = -kappa SampleSchedule(J) mean cost over the
 * n_wind samples) or the paper's literal product over SampleSchedule(J) + 1
 * passes. */
enum { SMC_WEIGHT_TEMPERED = 0, SMC_WEIGHT_PRODUCT = 1 };
/* Control parametrisation: the kinematic segment controls (heading rate,
 * airspeed reached at the segment's end, climb rate), or the paper's own
 * per-step thrust, flight-path angle and bank (Sec. "Trajectory Planning and
 * Disturbance Realisations", eq. hor; Sec. "Particles"). */
enum { SMC_CONTROLS_KINEMATIC = 0, SMC_CONTROLS_PAPER = 1 };

#define SMC_AC_NPAR 9   /* aircraft parameters per aircraft, see smc_scenario */
#define SMC_COST_NW 9   /* cost weights, see smc_scenario */
#define SMC_MAX_AIRCRAFT 64

/*
 * Scenario: copied at smc_mpc_init(); pointers need only live for that call.
 *
 *  n_aircraft N (1..64), n_segments S (per aircraft), horizon_max H (steps),
 *  n_particles L, n_wind M (wind samples per SMC iteration), n_iters K
 *  (weighting passes; K-1 resample/move rounds), dt step length [s].
 *  box = (W_x, W_y, Z_top): the area [-W_x/2, W_x/2] x [-W_y/2, W_y/2] x
 *  [0, Z_top]; the wind grid has grid_n = (nx, ny, nz) >= 2 nodes per axis
 *  spanning it (Sec. "Wind Model": Gaussian field on a grid, trilinear
 *  interpolation). wind_sigma, wind_ell, wind_nugget: squared-exponential
 *  covariance sigma^2 prod_a exp(-d_a^2 / 2 ell^2) factored per axis with
 *  the nugget added to each 1-D Gram matrix.
 *  sep_h, sep_v: required horizontal / vertical separation (= 2 P_r, 2 P_h of
 *  eq. (avoidance)); a pair closer than both violates.
 *  kind[N]: SMC_ARRIVAL / SMC_DEPARTURE.
 *  aircraft[N x 9]: wing area, C_D0, C_D2 (parabolic drag polar), C_f1, C_f2
 *  (fuel flow eta = C_f1 (1 + v / C_f2), Sec. "Fuel Estimate 1"), T_max,
 *  empty mass, bank limit phi_max, climb-angle limit gamma_max
 *  (Sec. "Constraint Handling").
 *  ctrl_lo/ctrl_hi: bounds of the three per-segment controls (heading rate
 *  [rad/s], airspeed reached at segment end [m/s], climb rate [m/s]).
 *  env: z_min, z_max, v_min, v_max.  landing: P_runway, P_beta, P_chi, P_vs
 *  (eq. TO_init) and the nominal glide angle beta_f.
 *  targets[N x 4] (departures): bearing theta_F, altitude Z, speed v_D,
 *  exit radius D_TMA (Sec. "Departure").
 *  cost_w: arrival heading, arrival glide, arrival fuel, departure bearing,
 *  departure fuel, departure altitude, departure speed (Tab. coeff),
 *  alpha_time, alpha_noise; the table part is scaled by
 *  (1 - alpha_time - alpha_noise).  time_norm [s] normalises time-to-go.
 *  noise_alt: altitude A_c above which noise is neglected; popdense[ny_p x
 *  nx_p] in [0, 1] spanning the box horizontally (Sec. "Noise Pollution
 *  Reduction"), or NULL.
 *  precision SMC_FP64 / SMC_FP32 (dynamics and wind; weights, scans and the
 *  accumulation over wind samples are FP64 in both), move SMC_MOVE_*,
 *  kappa (tempering scale: beta_J = kappa floor(3 + 5 e^{0.05 J}),
 *  Sec. "Simulation Setup"), sigma_move (move step in normalised control
 *  units), mala_step (standard deviation of the Langevin proposal in logit
 *  coordinates of the normalised controls), seed (Philox key), scenario_id
 *  (Philox stream tag).
 *  wind_model SMC_WIND_SE: the squared-exponential field above, one static
 *  field per wind sample and SMC iteration.  SMC_WIND_EXP_AR1 (Sec. "Wind
 *  Model", eq. cov and the linear Gaussian model after it): covariance
 *  wind_sigma^2 exp(-wind_beta |dxy|) exp(-wind_gamma |dz|) [1/m], Euclidean
 *  horizontal distance, the nugget added to the horizontal (nx ny points)
 *  and vertical (nz levels) Gram matrices, factor Qhat = sigma L_h (x) L_z;
 *  per sample one field per step k < horizon_max: W(0) = Qhat v(0),
 *  W(k+1) = a W(k) + sqrt(1 - a^2) Qhat v(k+1), a = exp(-dt / wind_tcorr)
 *  (wind_tcorr = G_t [s], > 0; infinity freezes the field), v(k) of sample m
 *  being the normals of sample k M + m; wind_ell is not used.  Limits of
 *  SMC_WIND_EXP_AR1: n_aircraft <= 20, move not SMC_MOVE_MALA, not in
 *  the batched form; horizon_max * n_wind * G * 2
 *  reals below 2^31 bytes; at most 16 levels (nz); init factors the
 *  (nx ny)^2 horizontal Gram matrix on the host.
 *  weighting SMC_WEIGHT_TEMPERED: every iteration J rolls out all n_wind
 *  samples and log W = -kappa SampleSchedule(J) c_hat.  SMC_WEIGHT_PRODUCT
 *  (Alg. 1 inner loop, Sec. "Weight Scaling"): iteration J makes
 *  SampleSchedule(J) + 1 passes, pass j under wind sample j (the first
 *  samples of the iteration's fields), and each multiplies the weight by
 *  the objective value 1 - cost: log W = sum_j log(1 - cost_j), -inf after
 *  a violation; c_hat is the mean over the passes.  Needs n_wind >=
 *  SampleSchedule(n_iters - 1) + 1, the static wind model and a move other
 *  than SMC_MOVE_MALA; not in the batched form.
 *  control_model SMC_CONTROLS_KINEMATIC: segment s of n_segments holds
 *  (heading rate [rad/s], airspeed [m/s], climb rate [m/s]) for the steps
 *  floor(k n_segments / horizon) = s.  SMC_CONTROLS_PAPER: step k has its own
 *  control set k (n_segments >= horizon_max, so D = 3 N horizon per
 *  particle), (thrust as a fraction of the aircraft's T_max, flight-path
 *  angle gamma [rad], bank phi [rad]) with ctrl_lo/ctrl_hi bounding those
 *  three (thrust fraction >= 0, |angles| < pi/2); v' = v + dt ((T - D)/m
 *  - g sin gamma), chi' = chi + dt L sin(phi) / (m v), L = m g cos(gamma) /
 *  cos(phi), z' = z + dt v sin(gamma), fuel dt eta(v) T; the departure
 *  altitude band grows at v_max sin(max |gamma bound|).  Limits:
 *  n_aircraft <= 20 (world-per-lane rollout), static wind model, move not
 *  SMC_MOVE_MALA, no smc_plant_step, not in the batched form.
 *  warm_start 1 (Sec. "Model Predictive Control", "Rolling Window": the
 *  window moves by the applied first control segment): every update after
 *  the context's first starts from the previous update's final population
 *  (the particles of its last weighting pass), particle l's segment s taken
 *  from the previous particle l's segment s + 1 and the last segment drawn
 *  U(0, 1) as a fresh initialisation draws that element; 0: every update
 *  draws fresh particles (Alg. 1).  Kinematic controls only; not in the
 *  batched form.
 */
typedef struct {
    int32_t n_aircraft, n_segments, horizon_max, n_particles, n_wind, n_iters;
    double dt;
    double box[3];
    int32_t grid_n[3];
    double wind_sigma, wind_ell, wind_nugget;
    double sep_h, sep_v;
    const int8_t* kind;
    const double* aircraft;
    double ctrl_lo[3], ctrl_hi[3];
    double env[4];
    double landing[5];
    const double* targets;
    double cost_w[SMC_COST_NW];
    double time_norm, noise_alt;
    const float* popdense;
    int32_t pop_n[2]; /* nx_p, ny_p */
    int32_t precision, move;
    double kappa, sigma_move, mala_step;
    uint64_t seed;
    int32_t scenario_id;
    int32_t wind_model;                         /* SMC_WIND_* */
    double wind_beta, wind_gamma, wind_tcorr;   /* SMC_WIND_EXP_AR1 only */
    int32_t weighting;                          /* SMC_WEIGHT_* */
    int32_t control_model;                      /* SMC_CONTROLS_* */
    int32_t warm_start;                         /* 0 or 1 */
} smc_scenario;

/* Diagnostics of one MPC update (optional output).  When requested, device
 * events bracket the rollout and wind GEMM launches on the update's stream. */
typedef struct {
    int32_t iterations;       /* weighting passes run (= n_iters)               */
    int32_t best_particle;    /* index of the returned particle                 */
    double feasible_frac;     /* (particle, aircraft) pairs feasible, last pass */
    double accept_rate;       /* mean MH acceptance (0 for jitter)              */
    double ess_min;           /* smallest per-aircraft ESS at the last pass     */
    int64_t aircraft_steps;   /* simulated aircraft-steps over all passes       */
    int64_t pair_tests;       /* separation tests with both aircraft present    */
    double ms_total;          /* wall time of the update, device events         */
    double ms_rollout;        /* summed duration of the rollout launches        */
    double ms_wind;           /* summed duration of the wind GEMM launches      */
    int32_t rollout_launches; /* rollout launches in the update                 */
    int32_t wind_launches;    /* wind GEMM launches in the update               */
    double ms_grad;           /* summed duration of the adjoint launches (MALA) */
    int32_t grad_launches;    /* adjoint launches in the update (MALA: 2 K)     */
    int64_t pair_tests_h;     /* pair tests that reached the horizontal distance
                               * comparison (= pair_tests except in the
                               * particle-per-wave rollout, which compares only
                               * pairs within the vertical separation)          */
} smc_step_info;

/* Create a context: validates the scenario, factors the wind covariance
 * (per-axis Cholesky, FP64) and expands it to the dense lower-triangular
 * G x G factor on the device, allocates all device buffers.
 * Errors: SMC_EINVAL (bad sizes / parameters), SMC_ENOTSPD, SMC_ENOMEM,
 * SMC_EDEVICE.  *out is NULL on error. */
smc_status smc_mpc_init(const smc_scenario* scenario, smc_ctx** out);

/* One MPC update (Alg. 1).
 *  mpc_step: Philox counter word (the update index).
 *  states[N x 6]: (x, y, z, v, chi, m) of each aircraft at its activation.
 *  k_active[N]: step at which the aircraft enters the horizon (0 = now);
 *     < 0 or >= horizon: not in the problem.
 *  wind_mean[2]: nominal wind (east, north) added to every field sample.
 *  horizon: 1..horizon_max steps, at least n_segments with the kinematic
 *     controls (no empty segment); any with the paper's per-step controls.
 *  controls_out[N x S x 3]: physical controls of the chosen particle.
 *  exp_cost_out[1 + N]: its total and per-aircraft expected cost (mean over
 *     the wind samples of the last pass; 0 best, 1 worst per aircraft).
 *  info: may be NULL. */
smc_status smc_mpc_step(smc_ctx* ctx, int64_t mpc_step, const double* states,
                        const int32_t* k_active, const double* wind_mean,
                        int32_t horizon, double* controls_out,
                        double* exp_cost_out, smc_step_info* info);

/* Device-pointer form of smc_mpc_step: states, k_active, controls_out and
 * exp_cost_out are device pointers; wind_mean is a host array of 2.
 * Work is queued on `stream` (hipStream_t, NULL = the context's stream).
 * When info is NULL the call does not synchronise; status_out (device int32,
 * may be NULL) receives 0 or SMC_INFEASIBLE. */
smc_status smc_mpc_step_dev(smc_ctx* ctx, int64_t mpc_step,
                            const double* d_states, const int32_t* d_k_active,
                            const double* wind_mean, int32_t horizon,
                            double* d_controls_out, double* d_exp_cost_out,
                            int32_t* d_status_out, smc_step_info* info,
                            void* stream);

/* Expected cost and feasibility of P given particles under the wind fields
 * of SMC iteration `iter` of update `mpc_step` (same Philox streams as
 * smc_mpc_step).  particles[P x N x S x 3] normalised controls in [0, 1];
 * cost_out[P x N]: mean cost over the wind samples; feasible_out[P x N]:
 * 1 if no sample violates.  Host pointers, synchronous. */
smc_status smc_eval_cost(smc_ctx* ctx, int64_t mpc_step, int32_t iter,
                         const double* states, const int32_t* k_active,
                         const double* wind_mean, int32_t horizon,
                         const double* particles, int32_t P,
                         double* cost_out, uint8_t* feasible_out);

/* The plant of the receding-horizon loop (Sec. "Model Predictive Control":
 * only the first part of the returned control sequence is applied, and the
 * plant's disturbance differs from the optimiser's predictions; Sec.
 * "Rolling Window": aircraft join at a pre-determined step and leave the
 * problem when they finish).  Every aircraft that has joined flies the first
 * n_steps steps of the plan `controls` [N x S x 3] (physical units, as
 * returned by smc_mpc_step for `horizon`; segment s(k) = floor(k S /
 * horizon)) from `states` with the rollout's arithmetic (the context's
 * precision), through one wind sample: sample 0 of the fields of iteration
 * word `plant_iter` of update `mpc_step` (an iteration word >= n_iters is
 * never drawn by the optimiser), with mean wind_mean; one static field, or
 * under SMC_WIND_EXP_AR1 that sample's field of each step (Sec. "Wind
 * Model").  An arrival stops when it meets the landing sector.
 *  states_out[N x 6]: states after the steps (an aircraft that has not
 *     joined keeps its state; a landed one its landing state).
 *  k_active_out[N]: activation steps for the next update: k_active -
 *     n_steps, at least 0, or -1 for an aircraft that was inactive, landed,
 *     or is a departure outside its exit radius D_TMA after the steps.
 *  event_out[N]: 1 landed, 2 left through the exit radius, 0 otherwise.
 * n_steps in [1, horizon], plant_iter >= 0.  Host pointers, synchronous.
 * Errors: SMC_EINVAL (nothing written), SMC_EDEVICE. */
smc_status smc_plant_step(smc_ctx* ctx, int64_t mpc_step, int32_t plant_iter,
                          const double* states, const int32_t* k_active,
                          const double* wind_mean, const double* controls,
                          int32_t horizon, int32_t n_steps, double* states_out,
                          int32_t* k_active_out, int32_t* event_out);

/* Message of the last failing call on ctx (or of the last failing init when
 * ctx is NULL).  Owned by the library, valid until the next call. */
const char* smc_last_error(const smc_ctx* ctx);

/* Release the context and its device memory.  NULL is a no-op. */
void smc_destroy(smc_ctx* ctx);

/* Library version string. */
const char* smc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SMC_MPC_H */
