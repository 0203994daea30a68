// Internal interface between the host orchestrator and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace smc {

constexpr int kMaxAircraft = 64;
constexpr int kStepSlots = 64;   // striped counters of simulated aircraft-steps
constexpr int kWorldLaneMaxN = 20;  // largest N of the world-per-lane rollout
// Largest workgroup of the aircraft-per-lane rollout (FP32 / FP64 lanes).
constexpr int kRolloutMaxBlock32 = 1024;
constexpr int kRolloutMaxBlock64 = 256;
constexpr int kAcR = 16;            // per-aircraft parameters in the rollout's precision

// Constants of the world-per-lane rollout in its own precision, derived on
// the host from the scalars of RolloutParams (so the kernel's step loop
// converts and combines nothing).  o* = offset of the grid map
// f = x inv_h + o; fn*1 / fn*2 = nodes - 1 / nodes - 2; c_* = cost weights
// with the normalisations folded in.
template <typename R>
struct RollConst {
    R ox, oy, inv_hx, inv_hy, inv_hz, fnx1, fny1, fnz1, fnx2, fny2, fnz2, fny, fnz;
    R inv_dt, g0, inv_g, sep_h2, sep_v, zmin, zmax, vmin, vmax;
    R p_run, p_beta, p_chi, p_vs, beta_f;
    R c_hdg, c_gl, c_brg, c_alt, a_time, a_noise, inv_tnorm, zdm_dt, inv_Ac;
    R isa_c, isa_e, rho0, dt, lo[3], span[3];
    R pop_ox, pop_oy, pop_inv_hx, pop_inv_hy, fpnx1, fpny1;
};

// Scalars of one rollout launch (uniform over the grid; kernel argument).
struct RolloutParams {
    int N, S, H, P, M, G;
    int nx, ny, nz;
    int use_noise, pop_nx, pop_ny;
    int control_model;      // 0 kinematic segment controls, 1 the paper's per-step (T, gamma, phi)
    double half_wx, half_wy, inv_hx, inv_hy, inv_hz;
    double pop_inv_hx, pop_inv_hy;
    double dt, sep_h2, sep_v;
    double ctrl_lo[3], ctrl_span[3];
    double zmin, zmax, vmin, vmax;
    double p_run, p_beta, p_chi, p_vs, beta_f;
    double w[9];
    double time_norm, noise_alt, zdot_max;
    int64_t w_kstride;      // reals between the fields of consecutive steps (0: one static field)
    RollConst<float> cf;    // world-per-lane constants, FP32
    RollConst<double> cd;   // world-per-lane constants, FP64
};

// Device arrays of one rollout launch.
struct RolloutArrays {
    const void* u;            // [P][N][S][3] real
    const void* W;            // [M][G][2] real, or [H][M][G][2] when w_kstride != 0
    const double* states;     // [N][6]
    const int32_t* k_active;  // [N]
    const double* acpar;      // [N][9]
    const double* targets;    // [N][4]
    const int8_t* kind;       // [N]
    const float* pop;         // [pop_ny][pop_nx] or null
    double* cost;             // [M][P][N]
    uint8_t* feas;            // [M][P][N]
    unsigned long long* steps;  // [2 kStepSlots] or null: aircraft-steps, pair tests
    // [kStepSlots] or null: pair tests that reached the horizontal comparison
    // (particle-per-wave layout: pairs within the vertical separation)
    unsigned long long* steps_h = nullptr;
};

// Control box: physical control c = lo[c] + normalised * sp[c].
struct Ctrl3 {
    double lo[3], sp[3];
};

// ---- batched form: many scenarios per launch ---------------------------------
// Buckets of the world-per-lane rollout (compile-time aircraft capacity).
constexpr int kNumBuckets = 8;
__host__ __device__ constexpr int bucket_nmax(int b) {
    return b == 0 ? 2 : b == 1 ? 4 : b == 2 ? 6 : b == 3 ? 8 : b == 4 ? 10 : b == 5 ? 12
         : b == 6 ? 16 : 20;
}
inline int bucket_of(int N) {
    for (int b = 0; b < kNumBuckets; ++b)
        if (N <= bucket_nmax(b)) return b;
    return -1;
}
constexpr int kItemWorlds = 64;   // worlds (particle, wind sample) per work item: one wave

// One scenario of a batch (device table).  The rollout's scalars and arrays
// (ra.u unused: each launch passes the control base pointer, and the
// scenario's controls start off_u elements after it), its per-aircraft rows,
// the tempering of every iteration and the offsets of its slices in the
// concatenated buffers of the batch.
struct BatchScen {
    RolloutParams rp;      // P = particles, H = this step's horizon
    RolloutArrays ra;      // cost / feas: this scenario's [M][P][N] slices
    const void* acR;       // [N][kAcR] real
    const double* beta;    // [K] beta_J = kappa floor(3 + 5 exp(0.05 J))
    uint64_t seed;
    int scen_id, N, S, D;  // D = 3 S controls per aircraft
    int off_n;             // first aircraft row of the scenario (states, k_active, resampling)
    int64_t off_u;         // controls [P][N][D]
    int64_t off_pn;        // per-particle rows [P][N] (c_hat, log-weights, feasibility)
    int64_t off_ctrl;      // returned controls [N][D]
    int64_t off_cost;      // returned expected costs [1 + N]
    double sigma_move;
    double mala_step;      // Langevin step (MALA moves)
    Ctrl3 box;
};

struct BatchItem {
    int scen;              // scenario of the item
    int world0;            // first world (l + P m) of the item's kItemWorlds
};

struct BatchStep {
    int64_t mpc_step;      // Philox counter word 3 of every draw of the step
};

// precision: 0 = double, 1 = float
hipError_t launch_philox_words(Stream s, uint32_t e0, int64_t n, uint32_t* out,
                               hipStream_t st);
// Warm start: u = the previous final population moved one control segment
// earlier, the last segment drawn as launch_init_particles draws it
// (count = P N S 3 elements; prev and u distinct).
hipError_t launch_warm_start(int prec, Stream s, int64_t count, int S, const void* prev,
                             void* u, hipStream_t st);
hipError_t launch_init_particles(int prec, Stream s, int64_t count, void* u,
                                 hipStream_t st);
hipError_t launch_wind_normals(int prec, Stream s, int G, int M, void* Z,
                               hipStream_t st);
// Normals of the time-correlated wind model: Z[G][2 H M], column (k M + m, c)
// holds u(k) = a u(k-1) + b v(k), u(0) = v(0), v(k) the pair of counter
// (k M + m) G + g; b = sqrt(1 - a^2).
hipError_t launch_wind_normals_ar1(int prec, Stream s, int G, int M, int H, double a, double b,
                                   void* Z, hipStream_t st);
// The recursion and the vertical factor in one pass (nz divides 64): writes
// Y[h][col][iz] as launch_wind_levels does from Z.
hipError_t launch_wind_normals_ar1_levels(int prec, Stream s, int G, int M, int H, int nz,
                                          double a, double b, const double* Lz, void* Y,
                                          hipStream_t st);
// Time-correlated wind with Qhat = sigma L_h (x) L_z: Y[h][col][iz] =
// sum_j Lz[iz][j] U[h nz + j][col] over the 2 M columns (nz <= 16), then
// W[m][h nz + iz][c] = w_c + sum_h' (sigma L_h)[h][h'] Y[h'][2 m + c][iz]
// (the triangular MFMA GEMM with nh rows and 2 M nz columns).
hipError_t launch_wind_levels(int prec, const void* U, const double* Lz, int nh, int nz, int M,
                              void* Y, hipStream_t st);
hipError_t launch_wind_gemm_levels(int prec, const void* Lh, const void* Y, double wm0,
                                   double wm1, int nh, int nz, int M, void* W, void* part,
                                   hipStream_t st);
hipError_t launch_kron_expand(int prec, const double* Lx, const double* Ly,
                              const double* Lz, int nx, int ny, int nz,
                              double sigma, void* Lfac, hipStream_t st);
// Wind GEMM.  When few output tiles would leave the chip idle (fewer than
// kWindGemmSplitBelow workgroups of whole row blocks), each K chunk runs in
// its own workgroup and `part` (wind_gemm_part_elems(G, M) reals, else
// unused) holds the chunk products.
constexpr int kWindGemmSplitBelow = 1024;
size_t wind_gemm_part_elems(int G, int M);
// Most grid levels of the vertical-factor pass (k_wind_levels).
constexpr int kMaxWindLevels = 16;
hipError_t launch_wind_gemm(int prec, const void* Lfac, const void* Z,
                            double wm0, double wm1, int G, int M, void* W, void* part,
                            hipStream_t st);
hipError_t launch_rollout(int prec, const RolloutParams& p,
                          const RolloutArrays& a, hipStream_t st);
bool rollout_wm_supported(int N);
// Sample-blocked fields for the rollouts whose lanes are wind samples: the
// samples split into blocks of B, block b holds Wt[b][g][B][2] (pairs of
// reals), so the samples of one grid point inside a block are contiguous
// and one block's fields are one contiguous range (the last block is
// padded to B samples).  B = M gives the plain sample-interleaved
// [G][M][2] layout.
constexpr int kWtBlockPw = 64;   // particle-per-wave rollout
constexpr int kWtBlockPt = 16;   // particle tile
__host__ __device__ inline int64_t wt_elems(int M, int G, int B) {
    return (int64_t)((M + B - 1) / B) * B * G;
}
// Particle-per-wave rollout (FP32, N <= 64): the 64 lanes of a wave are 64
// wind samples of one particle; Wt: the fields in blocks of kWtBlockPw.
bool rollout_pw_supported(int N, int prec);
hipError_t launch_rollout_pw(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                             const void* Wt, hipStream_t st);
// Particle-tile rollout (FP32, N <= 64): a wave holds 4 particles x 16 wind
// samples; Wt: the fields in blocks of kWtBlockPt.
bool rollout_pt_supported(int N, int prec);
hipError_t launch_rollout_pt(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                             const void* Wt, hipStream_t st);
// W[M][G][2] -> the sample-blocked Wt with blocks of B samples (pairs of
// reals), coalesced through LDS tiles.
hipError_t launch_wind_transpose(int prec, const void* W, int M, int G, int B, void* Wt,
                                 hipStream_t st);
// acR: [N][kAcR] real: wing area, C_D0, C_D2, dt C_f1, dt C_f1 / C_f2,
// T_max, empty mass, tan(phi_max), sin(gamma_max), theta_F, Z, v_D, D_TMA,
// (1 - alpha_time - alpha_noise) w_speed / speed span, kind (0 arrival,
// 1 departure), 0
hipError_t launch_rollout_wm(int prec, const RolloutParams& p, const RolloutArrays& a,
                             const void* acR, hipStream_t st);
// The same under one wind field per step (p.w_kstride reals apart).
hipError_t launch_rollout_wm_tv(int prec, const RolloutParams& p, const RolloutArrays& a,
                                const void* acR, hipStream_t st);
// adjoint of the fuel + time cost (sum over wind samples) w.r.t. the
// normalised controls; partial: chunk partials when M > 64
bool grad_supported(int H, int S);
size_t grad_partial_elems(int P, int N, int S, int M);
// W [M][G] pairs; Wt: workspace of the same size (the sample-interleaved
// copy the adjoint reads).
hipError_t launch_rollout_grad(int prec, const RolloutParams& rp, const void* u, const void* W,
                               const double* states, const int32_t* k_active, const double* acpar,
                               const double* targets, const int8_t* kind, void* Wt, double* partial,
                               double* grad_out, hipStream_t st);
// The receding-horizon plant: one lane per aircraft (N <= 64), one wind field.
hipError_t launch_plant(int prec, const RolloutParams& p, const double* ctrl, const void* W,
                        const double* states, const int32_t* k_active, const double* acpar,
                        const double* targets, const int8_t* kind, int n_steps,
                        double* states_out, int32_t* k_active_out, int32_t* event_out,
                        hipStream_t st);
hipError_t launch_mala_propose(int prec, int64_t count, const void* u, const double* gsum,
                               double coef, double eps, Stream s, void* up, hipStream_t st);
hipError_t launch_mala_decide(int prec, int P, int N, int D, const void* u, const void* up,
                              const double* g, const double* gprop, double coef, double eps,
                              const double* logw, const double* logw_prop, Stream s,
                              int32_t* flags, hipStream_t st);
hipError_t launch_accept_apply(int prec, int P, int N, int D, void* u, const void* u_prop,
                               double* chat, const double* chat_prop, uint8_t* feas_pn,
                               const uint8_t* feas_prop, double* logw, const double* logw_prop,
                               const int32_t* flags, hipStream_t st);
// The paper's literal weighting over M passes: log W = sum_m log(1 - cost_m).
hipError_t launch_reduce_product(int P, int M, int N, const double* cost, const uint8_t* feas,
                                 double* chat, uint8_t* feas_pn, double* logw, hipStream_t st);
hipError_t launch_reduce(int P, int M, int N, const double* cost,
                         const uint8_t* feas, double beta, double* chat,
                         uint8_t* feas_pn, double* logw, hipStream_t st);
hipError_t launch_resample_offsets(Stream s, int N, uint32_t* U, hipStream_t st);
hipError_t launch_resample(int P, int N, const double* logw, const uint32_t* U,
                           double* scan, int32_t* anc, double* ess,
                           hipStream_t st);
// The same with the scan workspace in a static device array (no
// allocation): P N <= kStaticScanDoubles, else hipErrorInvalidValue.
constexpr int64_t kStaticScanDoubles = int64_t(1) << 22;
constexpr int kMaxDevices = 64;
hipError_t launch_resample_static(int P, int N, const double* logw, const uint32_t* U,
                                  int32_t* anc, double* ess, hipStream_t st);
hipError_t launch_gather_move(int prec, int P, int N, int D, const void* u_in,
                              const int32_t* anc, void* u_out, Stream s,
                              double sigma, int jitter, hipStream_t st);
hipError_t launch_propose(int prec, int64_t count, const void* u, void* u_prop,
                          Stream s, double sigma, hipStream_t st);
hipError_t launch_accept(int prec, int P, int N, int D, void* u,
                         const void* u_prop, double* chat,
                         const double* chat_prop, uint8_t* feas_pn,
                         const uint8_t* feas_prop, double* logw,
                         const double* logw_prop, Stream s, int32_t* accepted,
                         int32_t* flags, hipStream_t st);
hipError_t launch_select(int P, int N, const double* logw, const double* chat,
                         double beta, int32_t* best, hipStream_t st);
hipError_t launch_wind_gemm_grouped(int prec, const void* Lfac, const void* Z,
                                    const double* wmean, int mper, int G, int M, void* W,
                                    void* part, hipStream_t st);
// The horizontal factor's product over level-mixed columns (as
// launch_wind_gemm_levels) with a mean per group of mper fields.
hipError_t launch_wind_gemm_levels_grouped(int prec, const void* Lh, const void* Y,
                                           const double* wmean, int mper, int nh, int nz, int M,
                                           void* W, void* part, hipStream_t st);

// batched launches: grids span every scenario of the table (ns entries)
hipError_t launch_b_fill(uint32_t* p, int64_t n, hipStream_t st);
hipError_t launch_b_init(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                         int64_t max_count, void* u, hipStream_t st);
hipError_t launch_b_normals(int prec, const BatchScen* tab, const BatchStep* hdr, int ns, int J,
                            int G, int M, void* Z, hipStream_t st);
// persistent world-per-lane rollout over the items of one bucket
hipError_t launch_b_rollout(int prec, int bucket, const BatchScen* tab, const BatchItem* items,
                            int n_items, uint32_t* queue, const void* u,
                            unsigned long long* steps, int block, int grid, hipStream_t st);
int b_rollout_resident(int prec, int bucket, int block);   // workgroups per CU
hipError_t launch_b_reduce(const BatchScen* tab, int ns, int J, int64_t max_pn, double* chat,
                           uint8_t* feas_pn, double* logw, hipStream_t st);
hipError_t launch_b_resample_offsets(const BatchScen* tab, const BatchStep* hdr,
                                     const int32_t* row_scen, int rows, int J, uint32_t* U,
                                     hipStream_t st);
hipError_t launch_b_resample(const BatchScen* tab, const int32_t* row_scen, int rows, int P,
                             const double* logw, const uint32_t* U, double* scan, int32_t* anc,
                             hipStream_t st);
hipError_t launch_b_gather_move(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                                int J, int64_t max_count, const void* u_in, const int32_t* anc,
                                void* u_out, int jitter, hipStream_t st);
hipError_t launch_b_propose(int prec, const BatchScen* tab, const BatchStep* hdr, int ns, int J,
                            int64_t max_count, const void* u, void* u_prop, hipStream_t st);
hipError_t launch_b_accept(int prec, const BatchScen* tab, const BatchStep* hdr, int ns, int J,
                           int P, int64_t max_count, void* u, const void* u_prop, double* chat,
                           const double* chat_prop, uint8_t* feas_pn, const uint8_t* feas_prop,
                           double* logw, const double* logw_prop, int32_t* flags,
                           uint32_t* accepted, hipStream_t st);
hipError_t launch_b_mala_propose(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                                int J, int64_t max_count, const void* u, const double* g,
                                void* u_prop, hipStream_t st);
hipError_t launch_b_mala_accept(int prec, const BatchScen* tab, const BatchStep* hdr, int ns,
                                int J, int P, int64_t max_count, void* u, const void* u_prop,
                                const double* g, const double* g_prop, double* chat,
                                const double* chat_prop, uint8_t* feas_pn,
                                const uint8_t* feas_prop, double* logw, const double* logw_prop,
                                int32_t* flags, uint32_t* accepted, hipStream_t st);
hipError_t launch_b_select(const BatchScen* tab, int ns, int J, int P, const double* logw,
                           const double* chat, int32_t* best, hipStream_t st);
hipError_t launch_b_write_result(int prec, const BatchScen* tab, int ns, const void* u,
                                 const int32_t* best, const double* chat, double* controls_out,
                                 double* cost_out, int32_t* status_out, hipStream_t st);

hipError_t launch_write_result(int prec, int N, int S, const void* u,
                               const int32_t* best, const double* chat,
                               const double* ctrl_lo, const double* ctrl_span,
                               double* controls_out, double* cost_out,
                               int32_t* status_out, hipStream_t st);

}  // namespace smc
