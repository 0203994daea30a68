// Host orchestrator and C ABI of the SMC-MPC engine: scenario validation,
// wind-covariance factorisation, device buffers, the SMC iteration loop of
// one MPC update (Alg. 1) and the kernel-level entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "engine.h"
#include "host_common.h"
#include "smc_kernels.h"
#include "smc_mpc.h"

using namespace smc;

namespace {

std::string g_init_error;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct smc_ctx {
    // scenario
    int N, S, Hmax, L, M, K, G, prec, move, scen_id;
    int nx, ny, nz;
    double dt, box[3], sigma, ell, nugget, sep_h, sep_v;
    double ctrl_lo[3], ctrl_hi[3], ctrl_span[3], env[4], landing[5], cost_w[9];
    double time_norm, noise_alt, kappa, sigma_move, mala_step;
    uint64_t seed;
    int pop_nx, pop_ny, use_noise;
    int wind_model;         // SMC_WIND_*
    double war1, bar1;      // time recursion: a = exp(-dt / G_t), b = sqrt(1 - a^2)
    int Mf;                 // fields per iteration: M (static) or H M (one per step)
    int weighting;          // SMC_WEIGHT_*
    size_t rsz;  // sizeof(real)
    RolloutParams rp;

    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> ev_roll, ev_wind, ev_grad;  // pairs bracketing launches
    std::vector<DevBuf> bufs;
    std::string err;

    // device buffers
    double *d_acpar = nullptr, *d_targets = nullptr;
    void* d_acR = nullptr;       // [N][kAcR] per-aircraft parameters, real
    int layout = 0;              // rollout layout: 0 auto, 1 aircraft/lane, 2 world/lane,
                                 // 3 particle/wave, 4 particle tile
    int8_t* d_kind = nullptr;
    float* d_pop = nullptr;
    void* d_Lfac = nullptr;
    void *d_Z = nullptr, *d_W = nullptr, *d_Wt = nullptr;
    int warm_start = 0;          // start from the previous update's population
    void* u_last = nullptr;      // the buffer holding the last update's final population
    void* d_wpart = nullptr;   // wind GEMM chunk products (few-tile shapes)
    // time-correlated wind, and the static wind's grouped product: sigma L_h
    // [nh][nh] real (L_h = Lx (x) Ly for the static wind), L_z [nz][nz]
    // double, the level-mixed normals Y [nh][2 Mf][nz] real
    void* d_Lh = nullptr;
    double* d_Lzd = nullptr;
    void* d_Y = nullptr;
    bool wind_grouped = false;   // static wind through (L_h (x) I) (I (x) L_z) Z
    double* d_one = nullptr;     // the 1 x 1 factor 1 (static wind's L_h expansion)
    void *d_u = nullptr, *d_u2 = nullptr, *d_up = nullptr;
    double* d_cost = nullptr;
    uint8_t* d_feas = nullptr;
    double *d_chat = nullptr, *d_logw = nullptr, *d_chat2 = nullptr, *d_logw2 = nullptr;
    uint8_t *d_feaspn = nullptr, *d_feaspn2 = nullptr;
    int32_t* d_anc = nullptr;
    uint32_t* d_U = nullptr;
    double* d_scan = nullptr;
    double* d_ess = nullptr;
    int32_t* d_flags = nullptr;
    double *d_g = nullptr, *d_g2 = nullptr, *d_gpart = nullptr;   // gradients (sum over samples)
    int32_t* d_best = nullptr;
    int32_t* d_status = nullptr;
    unsigned long long* d_steps = nullptr;
    double *d_states = nullptr, *d_ctrl_out = nullptr, *d_cost_out = nullptr;
    double* d_plant_states = nullptr;   // plant step: states after the steps
    int32_t* d_plant_i32 = nullptr;     // plant step: activation steps, events
    int32_t* d_kact = nullptr;
    int64_t eval_cap = 0;  // particles the eval buffers hold
    void* d_ueval = nullptr;
    double* d_ecost = nullptr;
    uint8_t* d_efeas = nullptr;
    double *d_echat = nullptr, *d_elogw = nullptr;
    uint8_t* d_efeaspn = nullptr;
};

namespace {

smc_status fail(smc_ctx* c, smc_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_init_error = buf;
    return code;
}

#define HIP_OK(ctx, expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((ctx), SMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

smc_status dalloc(smc_ctx* c, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, SMC_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    c->bufs.push_back(DevBuf{*p, bytes});
    return SMC_OK;
}

template <typename T>
smc_status dalloc_t(smc_ctx* c, T** p, size_t count) {
    void* v = nullptr;
    smc_status s = dalloc(c, &v, count * sizeof(T));
    *p = (T*)v;
    return s;
}

// Stream of a device-form call: the caller's handle as given.  NULL is the
// null (legacy default) stream, which every blocking stream orders with, so a
// caller that queues its inputs on its default stream (PyTorch's default
// stream has the handle 0) sees them written before the library reads them,
// and its later work waits for the library's outputs.
hipStream_t pick(smc_ctx*, void* stream) { return (hipStream_t)stream; }

double beta_of(const smc_ctx* c, int J) { return c->kappa * host::sample_schedule(J); }

smc_status validate(const smc_scenario* s) {
    if (!s) return fail(nullptr, SMC_EINVAL, "scenario is NULL");
    if (s->n_aircraft < 1 || s->n_aircraft > SMC_MAX_AIRCRAFT)
        return fail(nullptr, SMC_EINVAL, "n_aircraft must be in [1, %d]", SMC_MAX_AIRCRAFT);
    if (s->n_segments < 1) return fail(nullptr, SMC_EINVAL, "n_segments must be >= 1");
    if (s->horizon_max < 1 || s->horizon_max > 100000)
        return fail(nullptr, SMC_EINVAL, "horizon_max must be in [1, 100000]");
    if (s->n_segments > s->horizon_max)
        return fail(nullptr, SMC_EINVAL, "n_segments must not exceed horizon_max");
    if (s->n_particles < 1 || s->n_particles > (1 << 24))
        return fail(nullptr, SMC_EINVAL, "n_particles must be in [1, 2^24]");
    if (s->n_wind < 1 || s->n_wind > 4096) return fail(nullptr, SMC_EINVAL, "n_wind must be in [1, 4096]");
    if (s->n_iters < 1) return fail(nullptr, SMC_EINVAL, "n_iters must be >= 1");
    if (!(s->dt > 0)) return fail(nullptr, SMC_EINVAL, "dt must be > 0");
    for (int a = 0; a < 3; ++a) {
        if (!(s->box[a] > 0)) return fail(nullptr, SMC_EINVAL, "box dimensions must be > 0");
        if (s->grid_n[a] < 2 || s->grid_n[a] > 4096)
            return fail(nullptr, SMC_EINVAL, "grid_n must be in [2, 4096] per axis");
        if (!(s->ctrl_hi[a] >= s->ctrl_lo[a])) return fail(nullptr, SMC_EINVAL, "ctrl_hi < ctrl_lo");
    }
    const int64_t G = (int64_t)s->grid_n[0] * s->grid_n[1] * s->grid_n[2];
    if (G > 65536) return fail(nullptr, SMC_EINVAL, "grid has more than 65536 points");
    if (s->wind_model != SMC_WIND_SE && s->wind_model != SMC_WIND_EXP_AR1)
        return fail(nullptr, SMC_EINVAL, "wind_model must be SMC_WIND_SE or SMC_WIND_EXP_AR1");
    if (!(s->wind_sigma >= 0) || !(s->wind_nugget >= 0) ||
        (s->wind_model == SMC_WIND_SE && !(s->wind_ell > 0)))
        return fail(nullptr, SMC_EINVAL, "wind parameters out of range");
    if (s->weighting != SMC_WEIGHT_TEMPERED && s->weighting != SMC_WEIGHT_PRODUCT)
        return fail(nullptr, SMC_EINVAL, "weighting must be SMC_WEIGHT_TEMPERED or SMC_WEIGHT_PRODUCT");
    if (s->weighting == SMC_WEIGHT_PRODUCT) {
        const int need = (int)host::sample_schedule(s->n_iters - 1) + 1;
        if (s->n_wind < need)
            return fail(nullptr, SMC_EINVAL, "product weighting needs n_wind >= SampleSchedule(n_iters - 1) + 1 = %d",
                        need);
        if (s->move == SMC_MOVE_MALA)
            return fail(nullptr, SMC_EINVAL, "product weighting does not support the gradient move");
        if (s->wind_model != SMC_WIND_SE)
            return fail(nullptr, SMC_EINVAL, "product weighting takes the static wind model");
    }
    if (s->wind_model == SMC_WIND_EXP_AR1) {
        if (!(s->wind_beta > 0) || !(s->wind_gamma > 0) || !(s->wind_tcorr > 0))
            return fail(nullptr, SMC_EINVAL, "wind_beta, wind_gamma and wind_tcorr must be > 0");
        if (s->n_aircraft > kWorldLaneMaxN)
            return fail(nullptr, SMC_EINVAL, "time-correlated wind supports at most %d aircraft",
                        kWorldLaneMaxN);
        if (s->move == SMC_MOVE_MALA)
            return fail(nullptr, SMC_EINVAL, "time-correlated wind does not support the gradient move");
        if ((int64_t)s->grid_n[0] * s->grid_n[1] > 4096)
            return fail(nullptr, SMC_EINVAL, "time-correlated wind: at most 4096 horizontal nodes");
        if (s->grid_n[2] > 16)
            return fail(nullptr, SMC_EINVAL, "time-correlated wind: at most 16 levels");
        const double rbytes = s->precision == SMC_FP64 ? 8.0 : 4.0;
        if ((double)s->horizon_max * s->n_wind * G * 2 * rbytes >= 2147483648.0)
            return fail(nullptr, SMC_EINVAL, "time-correlated wind: the fields of all steps must take below 2^31 bytes");
    }
    if (s->control_model != SMC_CONTROLS_KINEMATIC && s->control_model != SMC_CONTROLS_PAPER)
        return fail(nullptr, SMC_EINVAL, "control_model must be SMC_CONTROLS_KINEMATIC or SMC_CONTROLS_PAPER");
    if (s->warm_start != 0 && s->warm_start != 1)
        return fail(nullptr, SMC_EINVAL, "warm_start must be 0 or 1");
    if (s->warm_start && s->control_model != SMC_CONTROLS_KINEMATIC)
        return fail(nullptr, SMC_EINVAL, "warm_start: kinematic segment controls only");
    if (s->control_model == SMC_CONTROLS_PAPER) {
        if (s->n_segments < s->horizon_max)
            return fail(nullptr, SMC_EINVAL, "the paper's controls need n_segments >= horizon_max (one control set per step)");
        if (s->n_aircraft > kWorldLaneMaxN)
            return fail(nullptr, SMC_EINVAL, "the paper's controls support at most %d aircraft", kWorldLaneMaxN);
        if (s->wind_model != SMC_WIND_SE)
            return fail(nullptr, SMC_EINVAL, "the paper's controls take the static wind model");
        if (s->move == SMC_MOVE_MALA)
            return fail(nullptr, SMC_EINVAL, "the paper's controls do not support the gradient move");
        if (!(s->ctrl_lo[0] >= 0) || !(s->ctrl_lo[1] > -1.5707963267948966) ||
            !(s->ctrl_hi[1] < 1.5707963267948966) || !(s->ctrl_lo[2] > -1.5707963267948966) ||
            !(s->ctrl_hi[2] < 1.5707963267948966))
            return fail(nullptr, SMC_EINVAL, "the paper's controls: thrust fraction >= 0 and |angles| < pi/2");
    } else if (!(s->ctrl_lo[1] > 0)) {
        return fail(nullptr, SMC_EINVAL, "airspeed control must be > 0");
    }
    if (!(s->sep_h >= 0) || !(s->sep_v >= 0)) return fail(nullptr, SMC_EINVAL, "separations must be >= 0");
    if (!s->kind || !s->aircraft || !s->targets)
        return fail(nullptr, SMC_EINVAL, "kind, aircraft and targets are required");
    for (int i = 0; i < s->n_aircraft; ++i) {
        if (s->kind[i] != SMC_ARRIVAL && s->kind[i] != SMC_DEPARTURE)
            return fail(nullptr, SMC_EINVAL, "kind[%d] must be 0 or 1", i);
        const double* a = s->aircraft + (size_t)i * SMC_AC_NPAR;
        if (!(a[0] > 0) || !(a[3] > 0) || !(a[4] > 0) || !(a[5] > 0))
            return fail(nullptr, SMC_EINVAL, "aircraft[%d]: wing area, C_f1, C_f2, T_max must be > 0", i);
        if (!(a[7] > 0) || !(a[7] < 1.5707963267948966) || !(a[8] > 0) || !(a[8] < 1.5707963267948966))
            return fail(nullptr, SMC_EINVAL, "aircraft[%d]: angle limits must be in (0, pi/2)", i);
        if (!(s->env[2] > 0)) return fail(nullptr, SMC_EINVAL, "v_min must be > 0");
    }
    if (!(s->time_norm > 0) || !(s->noise_alt > 0))
        return fail(nullptr, SMC_EINVAL, "time_norm and noise_alt must be > 0");
    if (s->popdense && (s->pop_n[0] < 2 || s->pop_n[1] < 2))
        return fail(nullptr, SMC_EINVAL, "population grid needs >= 2 nodes per axis");
    if (s->precision != SMC_FP64 && s->precision != SMC_FP32)
        return fail(nullptr, SMC_EINVAL, "precision must be SMC_FP64 or SMC_FP32");
    if (s->move != SMC_MOVE_JITTER && s->move != SMC_MOVE_RWMH && s->move != SMC_MOVE_MALA)
        return fail(nullptr, SMC_EINVAL, "move must be SMC_MOVE_JITTER, SMC_MOVE_RWMH or SMC_MOVE_MALA");
    if (s->move == SMC_MOVE_MALA && !grad_supported(s->horizon_max, s->n_segments))
        return fail(nullptr, SMC_EINVAL, "gradient move supports at most 16 segments and 400 steps");
    if (s->move == SMC_MOVE_MALA && !(s->mala_step > 0))
        return fail(nullptr, SMC_EINVAL, "mala_step must be > 0");
    if (!(s->kappa >= 0) || !(s->sigma_move >= 0))
        return fail(nullptr, SMC_EINVAL, "kappa and sigma_move must be >= 0");
    const double D = (double)s->n_particles * s->n_aircraft * s->n_segments * 3;
    if (D >= 4294967295.0)
        return fail(nullptr, SMC_EINVAL, "particle array exceeds 2^32 elements (Philox element index)");
    if ((double)G * s->n_wind >= 4294967295.0)
        return fail(nullptr, SMC_EINVAL, "wind normals exceed 2^32 elements");
    return SMC_OK;
}

// Chunk-product workspace of the wind GEMM for every sample count an update
// may use (each count up to M under the literal weighting).
size_t part_elems_upto(const smc_ctx* c) {
    size_t e = wind_gemm_part_elems(c->G, c->M);
    if (c->weighting == SMC_WEIGHT_PRODUCT)
        for (int m = 1; m < c->M; ++m) e = std::max(e, wind_gemm_part_elems(c->G, m));
    return e;
}

smc_status ensure_eval(smc_ctx* c, int64_t P) {
    if (P <= c->eval_cap) return SMC_OK;
    for (void* p : {c->d_ueval, (void*)c->d_ecost, (void*)c->d_efeas, (void*)c->d_echat,
                    (void*)c->d_elogw, (void*)c->d_efeaspn}) {
        if (!p) continue;
        for (auto it = c->bufs.begin(); it != c->bufs.end(); ++it)
            if (it->p == p) { (void)hipFree(p); c->bufs.erase(it); break; }
    }
    const size_t D = (size_t)c->N * c->S * 3;
    smc_status s;
    if ((s = dalloc(c, &c->d_ueval, (size_t)P * D * c->rsz))) return s;
    if ((s = dalloc_t(c, &c->d_ecost, (size_t)P * c->M * c->N))) return s;
    if ((s = dalloc_t(c, &c->d_efeas, (size_t)P * c->M * c->N))) return s;
    if ((s = dalloc_t(c, &c->d_echat, (size_t)P * c->N))) return s;
    if ((s = dalloc_t(c, &c->d_elogw, (size_t)P * c->N))) return s;
    if ((s = dalloc_t(c, &c->d_efeaspn, (size_t)P * c->N))) return s;
    c->eval_cap = P;
    return SMC_OK;
}

RolloutArrays rollout_arrays(smc_ctx* c, const void* u, const void* W, const double* states,
                             const int32_t* kact, double* cost, uint8_t* feas,
                             unsigned long long* steps) {
    RolloutArrays a;
    a.u = u;
    a.W = W;
    a.states = states;
    a.k_active = kact;
    a.acpar = c->d_acpar;
    a.targets = c->d_targets;
    a.kind = c->d_kind;
    a.pop = c->d_pop;
    a.cost = cost;
    a.feas = feas;
    a.steps = steps;
    // the context's own counters carry a third region for the horizontal
    // pair tests; a caller's counter buffer (kernel-level entry) does not
    a.steps_h = (steps && steps == c->d_steps) ? steps + 2 * kStepSlots : nullptr;
    return a;
}

// The rollout launch behind every pass: world-per-lane when N allows it,
// particle-per-wave above that in FP32 (after a copy of the fields into the
// sample-interleaved layout the wave's lanes read), aircraft-per-lane
// otherwise; or the layout asked for.
int rollout_layout(const smc_ctx* c) {
    if (c->rp.control_model == SMC_CONTROLS_PAPER) return 2;
    if (c->layout != 0) return c->layout;
    if (rollout_wm_supported(c->N)) return 2;
    return rollout_pt_supported(c->N, c->prec) ? 4 : 1;
}

hipError_t do_rollout(smc_ctx* c, const RolloutParams& rp, const RolloutArrays& a,
                      hipStream_t st) {
    if (rp.w_kstride != 0) return launch_rollout_wm_tv(c->prec, rp, a, c->d_acR, st);
    switch (rollout_layout(c)) {
    case 2: return launch_rollout_wm(c->prec, rp, a, c->d_acR, st);
    case 3:
    case 4: {
        const hipError_t e =
            launch_wind_transpose(c->prec, a.W, rp.M, rp.G,
                                  rollout_layout(c) == 3 ? kWtBlockPw : kWtBlockPt, c->d_Wt, st);
        if (e != hipSuccess) return e;
        return rollout_layout(c) == 3 ? launch_rollout_pw(rp, a, c->d_acR, c->d_Wt, st)
                                      : launch_rollout_pt(rp, a, c->d_acR, c->d_Wt, st);
    }
    default: return launch_rollout(c->prec, rp, a, st);
    }
}

smc_status check_horizon(smc_ctx* c, int32_t horizon) {
    if (horizon < 1 || horizon > c->Hmax)
        return fail(c, SMC_EINVAL, "horizon %d outside [1, %d]", horizon, c->Hmax);
    // kinematic segments must not be empty; the paper's per-step controls
    // take control set k at step k whatever the horizon
    if (c->rp.control_model == SMC_CONTROLS_KINEMATIC && horizon < c->S)
        return fail(c, SMC_EINVAL, "horizon %d shorter than n_segments %d", horizon, c->S);
    return SMC_OK;
}

// Normals of iteration J for the context's wind model (Sec. "Wind Model"):
// G x 2 M reals in d_Z (static); for the time-correlated model the time
// recursion over the H steps (d_Z, G x 2 H M), then the vertical factor
// along the levels (d_Y).
hipError_t wind_normals(smc_ctx* c, int64_t mpc_step, int J, hipStream_t st, int Ms = 0) {
    const Stream s = make_stream(c->seed, mpc_step, J, P_WIND, c->scen_id);
    if (c->wind_model != SMC_WIND_EXP_AR1)
        return launch_wind_normals(c->prec, s, c->G, Ms ? Ms : c->M, c->d_Z, st);
    if (64 % c->nz == 0)   // the levels of a node fit the lanes of one wave
        return launch_wind_normals_ar1_levels(c->prec, s, c->G, c->M, c->Hmax, c->nz, c->war1,
                                              c->bar1, c->d_Lzd, c->d_Y, st);
    hipError_t e = launch_wind_normals_ar1(c->prec, s, c->G, c->M, c->Hmax, c->war1, c->bar1,
                                           c->d_Z, st);
    if (e != hipSuccess) return e;
    return launch_wind_levels(c->prec, c->d_Z, c->d_Lzd, c->nx * c->ny, c->nz, c->Mf, c->d_Y, st);
}

// The fields from the normals: the dense factor's product (static), or the
// horizontal factor's product over the level-mixed normals.
// The static factor L = sigma Lx (x) Ly (x) Lz is applied in two groups:
// the levels' factor along z for every horizontal node, then the horizontal
// factor sigma Lx (x) Ly (an MFMA GEMM with nh rows over the level-mixed
// columns): the same product, nh (nh + 1) nz 2M flops instead of
// G (G + 1) 2M.
hipError_t wind_fields_grouped(smc_ctx* c, const void* Z, const double* wind_mean, int Mc,
                               void* W, hipStream_t st) {
    const int nh = c->nx * c->ny;
    const hipError_t e = launch_wind_levels(c->prec, Z, c->d_Lzd, nh, c->nz, Mc, c->d_Y, st);
    if (e != hipSuccess) return e;
    return launch_wind_gemm_levels(c->prec, c->d_Lh, c->d_Y, wind_mean[0], wind_mean[1], nh,
                                   c->nz, Mc, W, c->d_wpart, st);
}

hipError_t wind_fields_gemm(smc_ctx* c, const double* wind_mean, void* W, hipStream_t st,
                            int Ms = 0) {
    if (c->wind_model == SMC_WIND_EXP_AR1)
        return launch_wind_gemm_levels(c->prec, c->d_Lh, c->d_Y, wind_mean[0], wind_mean[1],
                                       c->nx * c->ny, c->nz, c->Mf, W, c->d_wpart, st);
    if (c->wind_grouped) return wind_fields_grouped(c, c->d_Z, wind_mean, Ms ? Ms : c->M, W, st);
    return launch_wind_gemm(c->prec, c->d_Lfac, c->d_Z, wind_mean[0], wind_mean[1], c->G,
                            Ms ? Ms : c->M, W, c->d_wpart, st);
}

// Samples (passes) of iteration J: all of them for the tempered weighting,
// SampleSchedule(J) + 1 for the paper's literal product (the first ones of
// the iteration's draw: the normals of sample m are counter m G + g).
int samples_of(const smc_ctx* c, int J) {
    return c->weighting == SMC_WEIGHT_PRODUCT ? (int)host::sample_schedule(J) + 1 : c->M;
}

// Weights of one pass set: tempered mean or the literal product.
hipError_t weigh(smc_ctx* c, int P, int Ms, double beta, double* chat, uint8_t* feaspn,
                 double* logw, hipStream_t st) {
    if (c->weighting == SMC_WEIGHT_PRODUCT)
        return launch_reduce_product(P, Ms, c->N, c->d_cost, c->d_feas, chat, feaspn, logw, st);
    return launch_reduce(P, Ms, c->N, c->d_cost, c->d_feas, beta, chat, feaspn, logw, st);
}

// The SMC loop of one MPC update on device buffers (Alg. 1).
smc_status run_step(smc_ctx* c, int64_t mpc_step, const double* d_states, const int32_t* d_kact,
                    const double* wind_mean, int32_t horizon, double* d_ctrl, double* d_cost_out,
                    int32_t* d_status, smc_step_info* info, hipStream_t st) {
    smc_status vs = check_horizon(c, horizon);
    if (vs) return vs;
    if (!wind_mean) return fail(c, SMC_EINVAL, "wind_mean is NULL");
    const int N = c->N, L = c->L, D = c->S * 3;
    const int64_t count = (int64_t)L * N * D;
    RolloutParams rp = c->rp;
    rp.H = horizon;
    rp.P = L;
    unsigned long long* steps = info ? c->d_steps : nullptr;
    if (info) {
        HIP_OK(c, hipMemsetAsync(c->d_steps, 0, sizeof(unsigned long long) * 3 * kStepSlots, st));
        HIP_OK(c, hipEventRecord(c->ev0, st));
    }
    void* u = c->d_u;
    void* u2 = c->d_u2;
    const Stream s_init = make_stream(c->seed, mpc_step, 0, P_INIT, c->scen_id);
    if (c->warm_start && c->u_last) {
        // the previous final population, moved one segment earlier, into
        // the other buffer
        if (c->u_last == u) std::swap(u, u2);
        HIP_OK(c, launch_warm_start(c->prec, s_init, count, c->S, c->u_last, u, st));
    } else {
        HIP_OK(c, launch_init_particles(c->prec, s_init, count, u, st));
    }
    double acc_sum = 0.0;
    int acc_n = 0, n_roll = 0, n_roll2 = 0;
    std::vector<int32_t> hflags;
    for (int J = 0; J < c->K; ++J) {
        const double beta = beta_of(c, J);
        const int Ms = samples_of(c, J);
        rp.M = Ms;
        HIP_OK(c, wind_normals(c, mpc_step, J, st, Ms));
        if (info) HIP_OK(c, hipEventRecord(c->ev_wind[2 * J], st));
        HIP_OK(c, wind_fields_gemm(c, wind_mean, c->d_W, st, Ms));
        if (info) HIP_OK(c, hipEventRecord(c->ev_wind[2 * J + 1], st));
        if (info) HIP_OK(c, hipEventRecord(c->ev_roll[4 * J], st));
        HIP_OK(c, do_rollout(c, rp,
                                 rollout_arrays(c, u, c->d_W, d_states, d_kact, c->d_cost,
                                                c->d_feas, steps),
                                 st));
        if (info) HIP_OK(c, hipEventRecord(c->ev_roll[4 * J + 1], st));
        ++n_roll;
        HIP_OK(c, weigh(c, L, Ms, beta, c->d_chat, c->d_feaspn, c->d_logw, st));
        if (c->move == SMC_MOVE_RWMH) {
            const Stream sm = make_stream(c->seed, mpc_step, J, P_MOVE, c->scen_id);
            HIP_OK(c, launch_propose(c->prec, count, u, c->d_up, sm, c->sigma_move, st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_roll[4 * J + 2], st));
            HIP_OK(c, do_rollout(c, rp,
                                     rollout_arrays(c, c->d_up, c->d_W, d_states, d_kact,
                                                    c->d_cost, c->d_feas, steps),
                                     st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_roll[4 * J + 3], st));
            ++n_roll2;
            HIP_OK(c, weigh(c, L, Ms, beta, c->d_chat2, c->d_feaspn2, c->d_logw2, st));
            HIP_OK(c, launch_accept(c->prec, L, N, D, u, c->d_up, c->d_chat, c->d_chat2,
                                    c->d_feaspn, c->d_feaspn2, c->d_logw, c->d_logw2,
                                    make_stream(c->seed, mpc_step, J, P_ACCEPT, c->scen_id),
                                    nullptr, c->d_flags, st));
            if (info) {
                hflags.resize(L);
                HIP_OK(c, hipMemcpyAsync(hflags.data(), c->d_flags, sizeof(int32_t) * L,
                                         hipMemcpyDeviceToHost, st));
                HIP_OK(c, hipStreamSynchronize(st));
                long a = 0;
                for (int l = 0; l < L; ++l) a += hflags[l];
                acc_sum += (double)a / L;
                ++acc_n;
            }
        }
        if (c->move == SMC_MOVE_MALA) {
            // Langevin proposal with the drift of the tempered fuel + time
            // cost; acceptance with the full target and the q ratio
            const double coef = -beta / (double)c->M;
            const double eps = c->mala_step;
            if (info) HIP_OK(c, hipEventRecord(c->ev_grad[4 * J], st));
            HIP_OK(c, launch_rollout_grad(c->prec, rp, u, c->d_W, d_states, d_kact, c->d_acpar,
                                          c->d_targets, c->d_kind, c->d_Wt, c->d_gpart, c->d_g, st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_grad[4 * J + 1], st));
            HIP_OK(c, launch_mala_propose(c->prec, count, u, c->d_g, coef, eps,
                                          make_stream(c->seed, mpc_step, J, P_MALA, c->scen_id),
                                          c->d_up, st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_roll[4 * J + 2], st));
            HIP_OK(c, do_rollout(c, rp,
                                 rollout_arrays(c, c->d_up, c->d_W, d_states, d_kact, c->d_cost,
                                                c->d_feas, steps),
                                 st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_roll[4 * J + 3], st));
            ++n_roll2;
            HIP_OK(c, launch_reduce(L, c->M, N, c->d_cost, c->d_feas, beta, c->d_chat2,
                                    c->d_feaspn2, c->d_logw2, st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_grad[4 * J + 2], st));
            HIP_OK(c, launch_rollout_grad(c->prec, rp, c->d_up, c->d_W, d_states, d_kact, c->d_acpar,
                                          c->d_targets, c->d_kind, c->d_Wt, c->d_gpart, c->d_g2, st));
            if (info) HIP_OK(c, hipEventRecord(c->ev_grad[4 * J + 3], st));
            HIP_OK(c, launch_mala_decide(c->prec, L, N, D, u, c->d_up, c->d_g, c->d_g2, coef, eps,
                                         c->d_logw, c->d_logw2,
                                         make_stream(c->seed, mpc_step, J, P_ACCEPT, c->scen_id),
                                         c->d_flags, st));
            HIP_OK(c, launch_accept_apply(c->prec, L, N, D, u, c->d_up, c->d_chat, c->d_chat2,
                                          c->d_feaspn, c->d_feaspn2, c->d_logw, c->d_logw2,
                                          c->d_flags, st));
            if (info) {
                hflags.resize(L);
                HIP_OK(c, hipMemcpyAsync(hflags.data(), c->d_flags, sizeof(int32_t) * L,
                                         hipMemcpyDeviceToHost, st));
                HIP_OK(c, hipStreamSynchronize(st));
                long a = 0;
                for (int l = 0; l < L; ++l) a += hflags[l];
                acc_sum += (double)a / L;
                ++acc_n;
            }
        }
        if (J == c->K - 1) break;
        HIP_OK(c, launch_resample_offsets(make_stream(c->seed, mpc_step, J, P_RESAMPLE, c->scen_id),
                                          N, c->d_U, st));
        HIP_OK(c, launch_resample(L, N, c->d_logw, c->d_U, c->d_scan, c->d_anc, nullptr, st));
        HIP_OK(c, launch_gather_move(c->prec, L, N, D, u, c->d_anc, u2,
                                     make_stream(c->seed, mpc_step, J, P_MOVE, c->scen_id),
                                     c->sigma_move, c->move == SMC_MOVE_JITTER ? 1 : 0, st));
        std::swap(u, u2);
    }
    c->u_last = u;   // this update's final population (a warm start's source)
    const double beta_last = beta_of(c, c->K - 1);
    HIP_OK(c, launch_select(L, N, c->d_logw, c->d_chat, beta_last, c->d_best, st));
    HIP_OK(c, launch_write_result(c->prec, N, c->S, u, c->d_best, c->d_chat, c->ctrl_lo,
                                  c->ctrl_span, d_ctrl, d_cost_out,
                                  d_status ? d_status : c->d_status, st));
    if (!info) return SMC_OK;

    HIP_OK(c, hipEventRecord(c->ev1, st));
    HIP_OK(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIP_OK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    int32_t best[2];
    HIP_OK(c, hipMemcpy(best, c->d_best, sizeof best, hipMemcpyDeviceToHost));
    std::vector<unsigned long long> cnt(3 * kStepSlots);
    HIP_OK(c, hipMemcpy(cnt.data(), c->d_steps, sizeof(unsigned long long) * 3 * kStepSlots,
                        hipMemcpyDeviceToHost));
    std::vector<uint8_t> fe((size_t)L * N);
    HIP_OK(c, hipMemcpy(fe.data(), c->d_feaspn, fe.size(), hipMemcpyDeviceToHost));
    // ESS of the final weights (diagnostic)
    HIP_OK(c, launch_resample_offsets(make_stream(c->seed, mpc_step, c->K - 1, P_RESAMPLE, c->scen_id),
                                      N, c->d_U, st));
    HIP_OK(c, launch_resample(L, N, c->d_logw, c->d_U, c->d_scan, c->d_anc, c->d_ess, st));
    std::vector<double> ess(N);
    HIP_OK(c, hipMemcpyAsync(ess.data(), c->d_ess, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
    long nf = 0;
    for (uint8_t f : fe) nf += f;
    unsigned long long tot = 0, totp = 0, toth = 0;
    for (int q = 0; q < kStepSlots; ++q) {
        tot += cnt[q];
        totp += cnt[kStepSlots + q];
        toth += cnt[2 * kStepSlots + q];
    }
    info->iterations = c->K;
    info->best_particle = best[0];
    info->feasible_frac = (double)nf / (double)fe.size();
    info->accept_rate = acc_n ? acc_sum / acc_n : 0.0;
    info->ess_min = *std::min_element(ess.begin(), ess.end());
    info->aircraft_steps = (int64_t)tot;
    info->pair_tests = (int64_t)totp;
    // the layouts whose lanes are the samples of particles test only pairs
    // within the vertical separation horizontally, the others all pairs
    const int lay = rollout_layout(c);
    info->pair_tests_h = (lay == 3 || lay == 4) && c->wind_model == SMC_WIND_SE ? (int64_t)toth
                                                                                 : (int64_t)totp;
    info->ms_total = ms;
    double ms_r = 0.0, ms_w = 0.0, ms_g = 0.0;
    const bool grad = c->move == SMC_MOVE_MALA;
    for (int J = 0; J < c->K; ++J) {
        if (grad) {
            for (int h = 0; h < 2; ++h) {
                float t = 0.f;
                HIP_OK(c, hipEventElapsedTime(&t, c->ev_grad[4 * J + 2 * h], c->ev_grad[4 * J + 2 * h + 1]));
                ms_g += t;
            }
        }
        float t = 0.f;
        HIP_OK(c, hipEventElapsedTime(&t, c->ev_wind[2 * J], c->ev_wind[2 * J + 1]));
        ms_w += t;
        HIP_OK(c, hipEventElapsedTime(&t, c->ev_roll[4 * J], c->ev_roll[4 * J + 1]));
        ms_r += t;
        if (J < n_roll2) {
            HIP_OK(c, hipEventElapsedTime(&t, c->ev_roll[4 * J + 2], c->ev_roll[4 * J + 3]));
            ms_r += t;
        }
    }
    info->ms_rollout = ms_r;
    info->ms_wind = ms_w;
    info->rollout_launches = n_roll + n_roll2;
    info->wind_launches = c->K;
    info->ms_grad = ms_g;
    info->grad_launches = grad ? 2 * c->K : 0;
    return best[1] ? SMC_INFEASIBLE : SMC_OK;
}

}  // namespace

namespace smc {
namespace host {

double sample_schedule(int J) { return std::floor(3.0 + 5.0 * std::exp(0.05 * J)); }

bool axis_factor(int n, double lo, double hi, double ell, double nugget, std::vector<double>& Lo) {
    std::vector<double> nodes(n), K((size_t)n * n);
    for (int a = 0; a < n; ++a) nodes[a] = (n == 1) ? lo : lo + (hi - lo) * a / (n - 1);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            const double d = nodes[a] - nodes[b];
            K[(size_t)a * n + b] = std::exp(-d * d / (2.0 * ell * ell)) + (a == b ? nugget : 0.0);
        }
    Lo.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = K[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= Lo[(size_t)j * n + k] * Lo[(size_t)j * n + k];
        if (!(s > 0.0)) return false;
        const double d = std::sqrt(s);
        Lo[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = K[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= Lo[(size_t)i * n + k] * Lo[(size_t)j * n + k];
            Lo[(size_t)i * n + j] = t / d;
        }
    }
    return true;
}

// Lower Cholesky factor of the n x n matrix K (row-major, FP64), row by row.
static bool cholesky_rows(int n, const std::vector<double>& K, std::vector<double>& Lo) {
    Lo.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        const double* Lj = Lo.data() + (size_t)j * n;
        double s = K[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= Lj[k] * Lj[k];
        if (!(s > 0.0)) return false;
        const double d = std::sqrt(s);
        Lo[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            const double* Li = Lo.data() + (size_t)i * n;
            double t = K[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= Li[k] * Lj[k];
            Lo[(size_t)i * n + j] = t / d;
        }
    }
    return true;
}

bool exp_factors(int nx, int ny, int nz, const double box[3], double beta, double gamma,
                 double nugget, std::vector<double>& Lh, std::vector<double>& Lz) {
    auto node = [](int n, double lo, double hi, int a) { return lo + (hi - lo) * a / (n - 1); };
    const int nh = nx * ny;
    std::vector<double> K((size_t)nh * nh);
    for (int p = 0; p < nh; ++p) {
        const double xp = node(nx, -0.5 * box[0], 0.5 * box[0], p / ny);
        const double yp = node(ny, -0.5 * box[1], 0.5 * box[1], p % ny);
        for (int q = 0; q < nh; ++q) {
            const double dx = xp - node(nx, -0.5 * box[0], 0.5 * box[0], q / ny);
            const double dy = yp - node(ny, -0.5 * box[1], 0.5 * box[1], q % ny);
            K[(size_t)p * nh + q] = std::exp(-beta * std::sqrt(dx * dx + dy * dy)) + (p == q ? nugget : 0.0);
        }
    }
    if (!cholesky_rows(nh, K, Lh)) return false;
    std::vector<double> Kz((size_t)nz * nz);
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < nz; ++b)
            Kz[(size_t)a * nz + b] =
                std::exp(-gamma * std::fabs(node(nz, 0.0, box[2], a) - node(nz, 0.0, box[2], b))) +
                (a == b ? nugget : 0.0);
    return cholesky_rows(nz, Kz, Lz);
}

smc_status validate_scenario(const smc_scenario* s, std::string& msg) {
    const smc_status r = validate(s);
    if (r) msg = g_init_error;
    return r;
}

void fill_rollout_params(const smc_scenario* s, RolloutParams& rp) {
    std::memset(&rp, 0, sizeof rp);
    const int nx = s->grid_n[0], ny = s->grid_n[1], nz = s->grid_n[2];
    const int use_noise = (s->popdense != nullptr && s->cost_w[8] != 0.0) ? 1 : 0;
    const int pop_nx = s->popdense ? s->pop_n[0] : 0, pop_ny = s->popdense ? s->pop_n[1] : 0;
    rp.N = s->n_aircraft; rp.S = s->n_segments; rp.H = s->horizon_max; rp.P = s->n_particles;
    rp.M = s->n_wind; rp.G = nx * ny * nz;
    rp.nx = nx; rp.ny = ny; rp.nz = nz;
    rp.use_noise = use_noise; rp.pop_nx = pop_nx; rp.pop_ny = pop_ny;
    rp.half_wx = 0.5 * s->box[0]; rp.half_wy = 0.5 * s->box[1];
    rp.inv_hx = (nx - 1) / s->box[0]; rp.inv_hy = (ny - 1) / s->box[1];
    rp.inv_hz = (nz - 1) / s->box[2];
    rp.pop_inv_hx = pop_nx > 1 ? (pop_nx - 1) / s->box[0] : 0.0;
    rp.pop_inv_hy = pop_ny > 1 ? (pop_ny - 1) / s->box[1] : 0.0;
    rp.dt = s->dt; rp.sep_h2 = s->sep_h * s->sep_h; rp.sep_v = s->sep_v;
    for (int a = 0; a < 3; ++a) {
        rp.ctrl_lo[a] = s->ctrl_lo[a];
        rp.ctrl_span[a] = s->ctrl_hi[a] - s->ctrl_lo[a];
    }
    rp.zmin = s->env[0]; rp.zmax = s->env[1]; rp.vmin = s->env[2]; rp.vmax = s->env[3];
    rp.p_run = s->landing[0]; rp.p_beta = s->landing[1]; rp.p_chi = s->landing[2];
    rp.p_vs = s->landing[3]; rp.beta_f = s->landing[4];
    for (int a = 0; a < 9; ++a) rp.w[a] = s->cost_w[a];
    rp.time_norm = s->time_norm; rp.noise_alt = s->noise_alt;
    rp.control_model = s->control_model;
    // bound of the climb rate (departure altitude band): the climb-rate
    // control's, or v_max sin(gamma bound) for the flight-path angle
    rp.zdot_max = s->control_model == SMC_CONTROLS_PAPER
                      ? s->env[3] * std::sin(std::max(std::fabs(s->ctrl_lo[1]), std::fabs(s->ctrl_hi[1])))
                      : std::max(std::fabs(s->ctrl_lo[2]), std::fabs(s->ctrl_hi[2]));
    fill_rollout_consts(rp);
}

namespace {
template <typename R>
void fill_consts(const RolloutParams& p, RollConst<R>& c) {
    const double pi = 3.14159265358979323846;
    const double mix = 1.0 - p.w[7] - p.w[8];
    c.ox = (R)(p.half_wx * p.inv_hx); c.oy = (R)(p.half_wy * p.inv_hy);
    c.inv_hx = (R)p.inv_hx; c.inv_hy = (R)p.inv_hy; c.inv_hz = (R)p.inv_hz;
    c.fnx1 = (R)(p.nx - 1); c.fny1 = (R)(p.ny - 1); c.fnz1 = (R)(p.nz - 1);
    c.fnx2 = (R)(p.nx - 2); c.fny2 = (R)(p.ny - 2); c.fnz2 = (R)(p.nz - 2);
    c.fny = (R)p.ny; c.fnz = (R)p.nz;
    c.inv_dt = (R)(1.0 / p.dt); c.g0 = (R)9.80665; c.inv_g = (R)(1.0 / 9.80665);
    c.sep_h2 = (R)p.sep_h2; c.sep_v = (R)p.sep_v;
    c.zmin = (R)p.zmin; c.zmax = (R)p.zmax; c.vmin = (R)p.vmin; c.vmax = (R)p.vmax;
    c.p_run = (R)p.p_run; c.p_beta = (R)p.p_beta; c.p_chi = (R)p.p_chi; c.p_vs = (R)p.p_vs;
    c.beta_f = (R)p.beta_f;
    c.c_hdg = (R)(mix * p.w[0] / pi);
    c.c_gl = (R)(mix * p.w[1] * 2.0 / pi);
    c.c_brg = (R)(mix * p.w[3] / pi);
    c.c_alt = (R)(mix * p.w[5]);
    c.a_time = (R)p.w[7]; c.a_noise = (R)p.w[8];
    c.inv_tnorm = (R)(1.0 / p.time_norm);
    c.zdm_dt = (R)(p.zdot_max * p.dt);
    c.inv_Ac = (R)(1.0 / p.noise_alt);
    c.isa_c = (R)(0.0065 / 288.15);
    c.isa_e = (R)(9.80665 / (287.05287 * 0.0065) - 1.0);
    c.rho0 = (R)1.225;
    c.dt = (R)p.dt;
    for (int a = 0; a < 3; ++a) { c.lo[a] = (R)p.ctrl_lo[a]; c.span[a] = (R)p.ctrl_span[a]; }
    c.pop_ox = (R)(p.half_wx * p.pop_inv_hx); c.pop_oy = (R)(p.half_wy * p.pop_inv_hy);
    c.pop_inv_hx = (R)p.pop_inv_hx; c.pop_inv_hy = (R)p.pop_inv_hy;
    c.fpnx1 = (R)(p.pop_nx - 1); c.fpny1 = (R)(p.pop_ny - 1);
}
}  // namespace

void fill_rollout_consts(RolloutParams& rp) {
    fill_consts<float>(rp, rp.cf);
    fill_consts<double>(rp, rp.cd);
}

void fill_acR(const smc_scenario* s, std::vector<double>& t) {
    const size_t N = (size_t)s->n_aircraft;
    t.assign(N * kAcR, 0.0);
    for (size_t i = 0; i < N; ++i) {
        const double* a = s->aircraft + i * SMC_AC_NPAR;
        const double* g = s->targets + i * 4;
        double* o = t.data() + i * kAcR;
        const double mix = 1.0 - s->cost_w[7] - s->cost_w[8];
        o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; o[3] = s->dt * a[3]; o[4] = s->dt * a[3] / a[4];
        o[5] = a[5]; o[6] = a[6]; o[7] = std::tan(a[7]); o[8] = std::sin(a[8]);
        o[9] = g[0]; o[10] = g[1]; o[11] = g[2]; o[12] = g[3];
        o[13] = mix * s->cost_w[6] / std::max(s->env[3] - g[2], g[2] - s->env[2]);
        o[14] = s->kind[i] == SMC_ARRIVAL ? 0.0 : 1.0;
    }
}

}  // namespace host
}  // namespace smc

extern "C" {

const char* smc_version(void) { return "smc-mpc-gfx950 0.1"; }

const char* smc_last_error(const smc_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

void smc_destroy(smc_ctx* c) {
    if (!c) return;
    // device-form calls queue on the caller's streams: wait for all of them
    // before the buffers go
    (void)hipDeviceSynchronize();
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& b : c->bufs) (void)hipFree(b.p);
    for (hipEvent_t e : c->ev_roll) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_wind) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_grad) (void)hipEventDestroy(e);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// No single device holds more (2^44 bytes = 16 TiB).
constexpr double kMaxDeviceBytes = 17592186044416.0;

// Bytes of the context's largest device buffers (a lower bound of what the
// initialisation allocates), in floating point so that no size overflows:
// per-world costs and feasibility, two particle control sets, the
// expanded wind factor, the normals, fields and their transposed copy.
double device_bytes_lower_bound(const smc_ctx* c) {
    const double L = c->L, N = c->N, M = c->M, G = c->G, Mf = c->Mf, D = 3.0 * c->S;
    const double r = (double)c->rsz;
    return M * L * N * (8.0 + 1.0) + 2.0 * L * N * D * r + G * G * r + G * 2.0 * Mf * r * 2.0 +
           M * G * 2.0 * r;
}

smc_status smc_mpc_init(const smc_scenario* s, smc_ctx** out) {
    if (!out) return fail(nullptr, SMC_EINVAL, "out is NULL");
    *out = nullptr;
    smc_status vs = validate(s);
    if (vs) return vs;
    smc_ctx* c = new (std::nothrow) smc_ctx();
    if (!c) return fail(nullptr, SMC_ENOMEM, "host allocation failed");
    c->N = s->n_aircraft; c->S = s->n_segments; c->Hmax = s->horizon_max;
    c->L = s->n_particles; c->M = s->n_wind; c->K = s->n_iters;
    c->nx = s->grid_n[0]; c->ny = s->grid_n[1]; c->nz = s->grid_n[2];
    c->G = c->nx * c->ny * c->nz;
    c->prec = s->precision; c->move = s->move; c->scen_id = s->scenario_id;
    c->dt = s->dt;
    for (int a = 0; a < 3; ++a) {
        c->box[a] = s->box[a];
        c->ctrl_lo[a] = s->ctrl_lo[a];
        c->ctrl_hi[a] = s->ctrl_hi[a];
        c->ctrl_span[a] = s->ctrl_hi[a] - s->ctrl_lo[a];
    }
    c->sigma = s->wind_sigma; c->ell = s->wind_ell; c->nugget = s->wind_nugget;
    c->sep_h = s->sep_h; c->sep_v = s->sep_v;
    std::memcpy(c->env, s->env, sizeof c->env);
    std::memcpy(c->landing, s->landing, sizeof c->landing);
    std::memcpy(c->cost_w, s->cost_w, sizeof c->cost_w);
    c->time_norm = s->time_norm; c->noise_alt = s->noise_alt;
    c->kappa = s->kappa; c->sigma_move = s->sigma_move; c->mala_step = s->mala_step;
    c->seed = s->seed;
    c->use_noise = (s->popdense != nullptr && s->cost_w[8] != 0.0) ? 1 : 0;
    c->pop_nx = s->popdense ? s->pop_n[0] : 0;
    c->pop_ny = s->popdense ? s->pop_n[1] : 0;
    c->rsz = c->prec == SMC_FP64 ? sizeof(double) : sizeof(float);
    c->wind_model = s->wind_model;
    c->war1 = c->wind_model == SMC_WIND_EXP_AR1 ? std::exp(-s->dt / s->wind_tcorr) : 0.0;
    c->bar1 = std::sqrt(std::max(0.0, 1.0 - c->war1 * c->war1));
    c->Mf = c->wind_model == SMC_WIND_EXP_AR1 ? c->Hmax * c->M : c->M;
    c->weighting = s->weighting;
    c->warm_start = s->warm_start;

    host::fill_rollout_params(s, c->rp);
    c->rp.w_kstride = c->wind_model == SMC_WIND_EXP_AR1 ? (int64_t)c->M * c->G * 2 : 0;

    // wind factor (FP64, host): per axis (squared-exponential), or the
    // horizontal and vertical factors of the exponential covariance, handed
    // to the Kronecker expansion as (nx ny, 1, nz) axes
    std::vector<double> Lx, Ly, Lz;
    int fx = c->nx, fy = c->ny;
    bool pd;
    c->wind_grouped = c->wind_model != SMC_WIND_EXP_AR1 && c->nz <= kMaxWindLevels;
    if (c->wind_model == SMC_WIND_EXP_AR1) {
        fx = c->nx * c->ny;
        fy = 1;
        Ly.assign(1, 1.0);
        pd = host::exp_factors(c->nx, c->ny, c->nz, c->box, s->wind_beta, s->wind_gamma, c->nugget,
                               Lx, Lz);
    } else {
        pd = host::axis_factor(c->nx, -0.5 * c->box[0], 0.5 * c->box[0], c->ell, c->nugget, Lx) &&
             host::axis_factor(c->ny, -0.5 * c->box[1], 0.5 * c->box[1], c->ell, c->nugget, Ly) &&
             host::axis_factor(c->nz, 0.0, c->box[2], c->ell, c->nugget, Lz);
    }
    if (!pd) {
        g_init_error = "wind covariance not positive definite (raise wind_nugget)";
        delete c;
        return SMC_ENOTSPD;
    }

    smc_status st;
    auto bail = [&](smc_status code) {
        g_init_error = c->err;
        smc_destroy(c);
        return code;
    };
    // the context's device memory, from its largest buffers (a lower bound
    // of the total): refused before any device work when no device could
    // hold it, and before the first allocation when this device's free
    // memory cannot
    const double need = device_bytes_lower_bound(c);
    if (need > kMaxDeviceBytes) {
        fail(c, SMC_ENOMEM, "the context needs at least %.4g bytes of device memory", need);
        return bail(SMC_ENOMEM);
    }
    hipError_t he = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (he != hipSuccess) {
        fail(c, SMC_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(he));
        return bail(SMC_EDEVICE);
    }
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need > (double)free_b) {
            fail(c, SMC_ENOMEM, "the context needs at least %.4g bytes of device memory, %zu free",
                 need, free_b);
            return bail(SMC_ENOMEM);
        }
        (void)hipGetLastError();
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        fail(c, SMC_EDEVICE, "hipEventCreate failed");
        return bail(SMC_EDEVICE);
    }
    c->ev_roll.assign((size_t)4 * c->K, nullptr);
    c->ev_wind.assign((size_t)2 * c->K, nullptr);
    c->ev_grad.assign(c->move == SMC_MOVE_MALA ? (size_t)4 * c->K : 0, nullptr);
    for (auto* v : {&c->ev_roll, &c->ev_wind, &c->ev_grad})
        for (auto& e : *v)
            if (hipEventCreate(&e) != hipSuccess) {
                fail(c, SMC_EDEVICE, "hipEventCreate failed");
                return bail(SMC_EDEVICE);
            }
    const size_t N = c->N, L = c->L, M = c->M, G = c->G, D = (size_t)c->S * 3, Mf = c->Mf;
    double *d_Lx = nullptr, *d_Ly = nullptr, *d_Lz = nullptr;
    if ((st = dalloc_t(c, &c->d_acpar, N * SMC_AC_NPAR)) || (st = dalloc_t(c, &c->d_targets, N * 4)) ||
        (st = dalloc_t(c, &c->d_kind, N)) ||
        (st = dalloc(c, &c->d_Lfac, G * G * c->rsz)) || (st = dalloc(c, &c->d_Z, G * 2 * Mf * c->rsz)) ||
        (st = dalloc(c, &c->d_W, Mf * G * 2 * c->rsz)) || (st = dalloc(c, &c->d_Wt, wt_elems(M, G, kWtBlockPw) * 2 * c->rsz)) ||
        (st = dalloc(c, &c->d_wpart, std::max<size_t>({part_elems_upto(c),
                                                       c->wind_model == SMC_WIND_EXP_AR1 ? wind_gemm_part_elems(fx, (int)Mf * c->nz) : 0,
                                                       c->wind_grouped ? wind_gemm_part_elems(c->nx * c->ny, (int)Mf * c->nz) : 0,
                                                       (size_t)1}) *
                                         c->rsz)) ||
        (st = dalloc(c, &c->d_u, L * N * D * c->rsz)) ||
        (st = dalloc(c, &c->d_u2, L * N * D * c->rsz)) ||
        (st = dalloc(c, &c->d_up, (c->move != SMC_MOVE_JITTER ? L : 1) * N * D * c->rsz)) ||
        (st = dalloc_t(c, &c->d_cost, M * L * N)) || (st = dalloc_t(c, &c->d_feas, M * L * N)) ||
        (st = dalloc_t(c, &c->d_chat, L * N)) || (st = dalloc_t(c, &c->d_logw, L * N)) ||
        (st = dalloc_t(c, &c->d_chat2, L * N)) || (st = dalloc_t(c, &c->d_logw2, L * N)) ||
        (st = dalloc_t(c, &c->d_feaspn, L * N)) || (st = dalloc_t(c, &c->d_feaspn2, L * N)) ||
        (st = dalloc_t(c, &c->d_anc, N * L)) || (st = dalloc_t(c, &c->d_U, N)) ||
        (st = dalloc_t(c, &c->d_scan, N * L)) || (st = dalloc_t(c, &c->d_ess, N)) ||
        (st = dalloc_t(c, &c->d_flags, L)) || (st = dalloc_t(c, &c->d_best, 2)) ||
        (st = dalloc_t(c, &c->d_status, 1)) || (st = dalloc_t(c, &c->d_steps, 3 * kStepSlots)) ||
        (st = dalloc_t(c, &c->d_states, N * 6)) || (st = dalloc_t(c, &c->d_kact, N)) ||
        (st = dalloc_t(c, &c->d_ctrl_out, N * D)) || (st = dalloc_t(c, &c->d_cost_out, 1 + N)) ||
        (st = dalloc_t(c, &c->d_plant_states, N * 6)) || (st = dalloc_t(c, &c->d_plant_i32, 2 * N)) ||
        (st = dalloc_t(c, &d_Lx, (size_t)fx * fx)) || (st = dalloc_t(c, &d_Ly, (size_t)fy * fy)) ||
        (st = dalloc_t(c, &d_Lz, (size_t)c->nz * c->nz)))
        return bail(st);
    if ((st = dalloc(c, &c->d_acR, N * kAcR * c->rsz))) return bail(st);
    if (c->wind_model == SMC_WIND_EXP_AR1 &&
        ((st = dalloc(c, &c->d_Lh, (size_t)fx * fx * c->rsz)) ||
         (st = dalloc_t(c, &c->d_Lzd, (size_t)c->nz * c->nz)) ||
         (st = dalloc(c, &c->d_Y, G * 2 * Mf * c->rsz))))
        return bail(st);
    if (c->wind_grouped &&
        ((st = dalloc(c, &c->d_Lh, (size_t)c->nx * c->ny * c->nx * c->ny * c->rsz)) ||
         (st = dalloc_t(c, &c->d_Lzd, (size_t)c->nz * c->nz)) ||
         (st = dalloc(c, &c->d_Y, G * 2 * Mf * c->rsz)) || (st = dalloc_t(c, &c->d_one, 1))))
        return bail(st);
    {
        const size_t gl = (c->move == SMC_MOVE_MALA ? L : 1) * N * D;
        if ((st = dalloc_t(c, &c->d_g, gl)) || (st = dalloc_t(c, &c->d_g2, gl)) ||
            (st = dalloc_t(c, &c->d_gpart, c->M > 64 ? grad_partial_elems((int)L, (int)N, c->S, (int)M) : 1)))
            return bail(st);
    }
    if (c->use_noise || s->popdense) {
        if ((st = dalloc_t(c, &c->d_pop, (size_t)c->pop_nx * c->pop_ny))) return bail(st);
    }
#define INIT_HIP(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            fail(c, SMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
            return bail(SMC_EDEVICE);                                                    \
        }                                                                                \
    } while (0)
    INIT_HIP(hipMemcpy(c->d_acpar, s->aircraft, N * SMC_AC_NPAR * sizeof(double), hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(c->d_targets, s->targets, N * 4 * sizeof(double), hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(c->d_kind, s->kind, N, hipMemcpyHostToDevice));
    {
        std::vector<double> t;
        host::fill_acR(s, t);
        if (c->prec == SMC_FP64) {
            INIT_HIP(hipMemcpy(c->d_acR, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
        } else {
            std::vector<float> f(t.begin(), t.end());
            INIT_HIP(hipMemcpy(c->d_acR, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    }
    if (c->d_pop)
        INIT_HIP(hipMemcpy(c->d_pop, s->popdense, (size_t)c->pop_nx * c->pop_ny * sizeof(float),
                           hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(d_Lx, Lx.data(), Lx.size() * sizeof(double), hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(d_Ly, Ly.data(), Ly.size() * sizeof(double), hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(d_Lz, Lz.data(), Lz.size() * sizeof(double), hipMemcpyHostToDevice));
    INIT_HIP(launch_kron_expand(c->prec, d_Lx, d_Ly, d_Lz, fx, fy, c->nz, c->sigma, c->d_Lfac,
                                c->stream));
    if (c->wind_grouped) {   // sigma Lx (x) Ly (d_one: the 1 x 1 factor 1), and L_z
        const double one = 1.0;
        INIT_HIP(hipMemcpy(c->d_one, &one, sizeof(double), hipMemcpyHostToDevice));
        INIT_HIP(launch_kron_expand(c->prec, d_Lx, d_Ly, c->d_one, fx, fy, 1, c->sigma, c->d_Lh,
                                    c->stream));
        INIT_HIP(hipMemcpy(c->d_Lzd, Lz.data(), Lz.size() * sizeof(double), hipMemcpyHostToDevice));
    } else if (c->d_Lh) {   // sigma L_h alone (d_Ly holds the 1 x 1 factor 1), and L_z
        INIT_HIP(launch_kron_expand(c->prec, d_Lx, d_Ly, d_Ly, fx, 1, 1, c->sigma, c->d_Lh,
                                    c->stream));
        INIT_HIP(hipMemcpy(c->d_Lzd, Lz.data(), Lz.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    INIT_HIP(hipStreamSynchronize(c->stream));
#undef INIT_HIP
    *out = c;
    return SMC_OK;
}

smc_status smc_mpc_step_dev(smc_ctx* c, int64_t mpc_step, const double* d_states,
                            const int32_t* d_kact, const double* wind_mean, int32_t horizon,
                            double* d_ctrl, double* d_cost_out, int32_t* d_status,
                            smc_step_info* info, void* stream) {
    if (!c) return fail(nullptr, SMC_EINVAL, "ctx is NULL");
    if (!d_states || !d_kact || !d_ctrl || !d_cost_out)
        return fail(c, SMC_EINVAL, "NULL device pointer");
    return run_step(c, mpc_step, d_states, d_kact, wind_mean, horizon, d_ctrl, d_cost_out,
                    d_status, info, pick(c, stream));
}

smc_status smc_mpc_step(smc_ctx* c, int64_t mpc_step, const double* states,
                        const int32_t* k_active, const double* wind_mean, int32_t horizon,
                        double* controls_out, double* exp_cost_out, smc_step_info* info) {
    if (!c) return fail(nullptr, SMC_EINVAL, "ctx is NULL");
    if (!states || !k_active || !wind_mean || !controls_out || !exp_cost_out)
        return fail(c, SMC_EINVAL, "NULL argument");
    smc_status vs = check_horizon(c, horizon);
    if (vs) return vs;
    hipStream_t st = c->stream;
    HIP_OK(c, hipMemcpyAsync(c->d_states, states, sizeof(double) * c->N * 6, hipMemcpyHostToDevice, st));
    HIP_OK(c, hipMemcpyAsync(c->d_kact, k_active, sizeof(int32_t) * c->N, hipMemcpyHostToDevice, st));
    smc_step_info local;
    smc_status r = run_step(c, mpc_step, c->d_states, c->d_kact, wind_mean, horizon, c->d_ctrl_out,
                            c->d_cost_out, c->d_status, info ? info : &local, st);
    if (r < 0) return r;
    HIP_OK(c, hipMemcpyAsync(controls_out, c->d_ctrl_out, sizeof(double) * c->N * c->S * 3,
                             hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(exp_cost_out, c->d_cost_out, sizeof(double) * (1 + c->N),
                             hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
    return r;
}

smc_status smc_plant_step(smc_ctx* c, int64_t mpc_step, int32_t plant_iter, const double* states,
                          const int32_t* k_active, const double* wind_mean, const double* controls,
                          int32_t horizon, int32_t n_steps, double* states_out,
                          int32_t* k_active_out, int32_t* event_out) {
    if (!c) return fail(nullptr, SMC_EINVAL, "ctx is NULL");
    if (!states || !k_active || !wind_mean || !controls || !states_out || !k_active_out || !event_out)
        return fail(c, SMC_EINVAL, "NULL argument");
    smc_status vs = check_horizon(c, horizon);
    if (vs) return vs;
    if (n_steps < 1 || n_steps > horizon) return fail(c, SMC_EINVAL, "n_steps must be in [1, horizon]");
    if (plant_iter < 0) return fail(c, SMC_EINVAL, "plant_iter must be >= 0");
    if (c->rp.control_model != SMC_CONTROLS_KINEMATIC)
        return fail(c, SMC_EINVAL, "smc_plant_step: kinematic controls only");
    hipStream_t st = c->stream;
    const int N = c->N;
    HIP_OK(c, hipMemcpyAsync(c->d_states, states, sizeof(double) * N * 6, hipMemcpyHostToDevice, st));
    HIP_OK(c, hipMemcpyAsync(c->d_kact, k_active, sizeof(int32_t) * N, hipMemcpyHostToDevice, st));
    HIP_OK(c, hipMemcpyAsync(c->d_ctrl_out, controls, sizeof(double) * N * c->S * 3,
                             hipMemcpyHostToDevice, st));
    // the fields of iteration word plant_iter (every step's under the
    // time-correlated model, rp.w_kstride apart); the plant flies sample 0
    HIP_OK(c, wind_normals(c, mpc_step, plant_iter, st));
    HIP_OK(c, wind_fields_gemm(c, wind_mean, c->d_W, st));
    RolloutParams rp = c->rp;
    rp.H = horizon;
    HIP_OK(c, launch_plant(c->prec, rp, c->d_ctrl_out, c->d_W, c->d_states, c->d_kact, c->d_acpar,
                           c->d_targets, c->d_kind, n_steps, c->d_plant_states, c->d_plant_i32,
                           c->d_plant_i32 + N, st));
    HIP_OK(c, hipMemcpyAsync(states_out, c->d_plant_states, sizeof(double) * N * 6,
                             hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(k_active_out, c->d_plant_i32, sizeof(int32_t) * N, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(event_out, c->d_plant_i32 + N, sizeof(int32_t) * N, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
    return SMC_OK;
}

smc_status smc_eval_cost(smc_ctx* c, int64_t mpc_step, int32_t iter, const double* states,
                         const int32_t* k_active, const double* wind_mean, int32_t horizon,
                         const double* particles, int32_t P, double* cost_out,
                         uint8_t* feasible_out) {
    if (!c) return fail(nullptr, SMC_EINVAL, "ctx is NULL");
    if (!states || !k_active || !wind_mean || !particles || !cost_out || !feasible_out)
        return fail(c, SMC_EINVAL, "NULL argument");
    if (P < 1) return fail(c, SMC_EINVAL, "P must be >= 1");
    if (iter < 0) return fail(c, SMC_EINVAL, "iter must be >= 0");
    smc_status vs = check_horizon(c, horizon);
    if (vs) return vs;
    if ((double)P * c->N * c->S * 3 >= 4294967295.0) return fail(c, SMC_EINVAL, "too many particles");
    if ((vs = ensure_eval(c, P))) return vs;
    hipStream_t st = c->stream;
    const size_t D = (size_t)c->N * c->S * 3;
    const size_t n = (size_t)P * D;
    if (c->prec == SMC_FP64) {
        HIP_OK(c, hipMemcpyAsync(c->d_ueval, particles, n * sizeof(double), hipMemcpyHostToDevice, st));
    } else {
        std::vector<float> tmp(n);
        for (size_t e = 0; e < n; ++e) tmp[e] = (float)particles[e];
        HIP_OK(c, hipMemcpyAsync(c->d_ueval, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_OK(c, hipStreamSynchronize(st));
    }
    HIP_OK(c, hipMemcpyAsync(c->d_states, states, sizeof(double) * c->N * 6, hipMemcpyHostToDevice, st));
    HIP_OK(c, hipMemcpyAsync(c->d_kact, k_active, sizeof(int32_t) * c->N, hipMemcpyHostToDevice, st));
    HIP_OK(c, wind_normals(c, mpc_step, iter, st));
    HIP_OK(c, wind_fields_gemm(c, wind_mean, c->d_W, st));
    RolloutParams rp = c->rp;
    rp.H = horizon;
    rp.P = P;
    HIP_OK(c, do_rollout(c, rp,
                             rollout_arrays(c, c->d_ueval, c->d_W, c->d_states, c->d_kact, c->d_ecost,
                                            c->d_efeas, nullptr),
                             st));
    HIP_OK(c, launch_reduce(P, c->M, c->N, c->d_ecost, c->d_efeas, 1.0, c->d_echat, c->d_efeaspn,
                            c->d_elogw, st));
    HIP_OK(c, hipMemcpyAsync(cost_out, c->d_echat, sizeof(double) * P * c->N, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipMemcpyAsync(feasible_out, c->d_efeaspn, (size_t)P * c->N, hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
    return SMC_OK;
}

// ---- kernel-level entry points -------------------------------------------------------

smc_status smc_k_philox(uint64_t seed, int64_t mpc_step, int32_t iter, int32_t purpose,
                        int32_t scenario, int64_t e0, int64_t n, uint32_t* out, void* stream) {
    if (!out || n < 0 || e0 < 0 || e0 + n > 4294967296LL)
        return fail(nullptr, SMC_EINVAL, "smc_k_philox: bad arguments");
    hipError_t e = launch_philox_words(make_stream(seed, mpc_step, iter, (uint32_t)purpose, scenario),
                                       (uint32_t)e0, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, SMC_EDEVICE, "philox launch: %s", hipGetErrorString(e));
    return SMC_OK;
}

smc_status smc_k_init_particles(smc_ctx* c, int64_t mpc_step, int32_t P, void* u, void* stream) {
    if (!c || !u || P < 1) return fail(c, SMC_EINVAL, "smc_k_init_particles: bad arguments");
    const int64_t count = (int64_t)P * c->N * c->S * 3;
    if (count >= 4294967296LL) return fail(c, SMC_EINVAL, "too many particles");
    HIP_OK(c, launch_init_particles(c->prec, make_stream(c->seed, mpc_step, 0, P_INIT, c->scen_id),
                                    count, u, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_wind_normals(smc_ctx* c, int64_t mpc_step, int32_t iter, void* Z, void* stream) {
    if (!c || !Z || iter < 0) return fail(c, SMC_EINVAL, "smc_k_wind_normals: bad arguments");
    HIP_OK(c, launch_wind_normals(c->prec, make_stream(c->seed, mpc_step, iter, P_WIND, c->scen_id),
                                  c->G, c->M, Z, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_wind_gemm(smc_ctx* c, const void* Z, const double* wind_mean, void* W, void* stream) {
    if (!c || !Z || !W || !wind_mean) return fail(c, SMC_EINVAL, "smc_k_wind_gemm: bad arguments");
    if (c->wind_grouped) {
        HIP_OK(c, wind_fields_grouped(c, Z, wind_mean, c->M, W, pick(c, stream)));
        return SMC_OK;
    }
    HIP_OK(c, launch_wind_gemm(c->prec, c->d_Lfac, Z, wind_mean[0], wind_mean[1], c->G, c->M, W,
                               c->d_wpart, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_wind_factor(smc_ctx* c, void* out, void* stream) {
    if (!c || !out) return fail(c, SMC_EINVAL, "smc_k_wind_factor: bad arguments");
    HIP_OK(c, hipMemcpyAsync(out, c->d_Lfac, (size_t)c->G * c->G * c->rsz, hipMemcpyDeviceToDevice,
                             pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_wind_fields(smc_ctx* c, int64_t mpc_step, int32_t iter, const double* wind_mean,
                             void* W, void* stream) {
    if (!c || !W || !wind_mean || iter < 0) return fail(c, SMC_EINVAL, "smc_k_wind_fields: bad arguments");
    hipStream_t st = pick(c, stream);
    HIP_OK(c, wind_normals(c, mpc_step, iter, st));
    HIP_OK(c, wind_fields_gemm(c, wind_mean, W, st));
    return SMC_OK;
}

smc_status smc_k_rollout(smc_ctx* c, const void* u, int32_t P, const void* W, const double* states,
                         const int32_t* k_active, int32_t horizon, double* cost, uint8_t* feas,
                         uint64_t* steps, void* stream) {
    if (!c || !u || !W || !states || !k_active || !cost || !feas || P < 1)
        return fail(c, SMC_EINVAL, "smc_k_rollout: bad arguments");
    smc_status vs = check_horizon(c, horizon);
    if (vs) return vs;
    RolloutParams rp = c->rp;
    rp.H = horizon;
    rp.P = P;
    HIP_OK(c, do_rollout(c, rp,
                             rollout_arrays(c, u, W, states, k_active, cost, feas,
                                            (unsigned long long*)steps),
                             pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_reduce_product(smc_ctx* c, int32_t P, int32_t M, const double* cost,
                                const uint8_t* feas, double* chat, uint8_t* feas_pn, double* logw,
                                void* stream) {
    if (!c || !cost || !feas || !chat || !feas_pn || !logw || P < 1 || M < 1 || M > c->M)
        return fail(c, SMC_EINVAL, "smc_k_reduce_product: bad arguments");
    HIP_OK(c, launch_reduce_product(P, M, c->N, cost, feas, chat, feas_pn, logw, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_reduce(smc_ctx* c, int32_t P, const double* cost, const uint8_t* feas, double beta,
                        double* chat, uint8_t* feas_pn, double* logw, void* stream) {
    if (!c || !cost || !feas || !chat || !feas_pn || !logw || P < 1)
        return fail(c, SMC_EINVAL, "smc_k_reduce: bad arguments");
    HIP_OK(c, launch_reduce(P, c->M, c->N, cost, feas, beta, chat, feas_pn, logw, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_resample_offsets(smc_ctx* c, int64_t mpc_step, int32_t iter, uint32_t* U,
                                  void* stream) {
    if (!c || !U) return fail(c, SMC_EINVAL, "smc_k_resample_offsets: bad arguments");
    HIP_OK(c, launch_resample_offsets(make_stream(c->seed, mpc_step, iter, P_RESAMPLE, c->scen_id),
                                      c->N, U, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_resample(smc_ctx* c, int32_t P, const double* logw, const uint32_t* U,
                          int32_t* anc, double* ess, void* stream) {
    if (!c || !logw || !U || !anc || P < 1) return fail(c, SMC_EINVAL, "smc_k_resample: bad arguments");
    if (P > c->L) {
        // the scan scratch holds N x L doubles
        return fail(c, SMC_EINVAL, "smc_k_resample: P exceeds the context's n_particles");
    }
    HIP_OK(c, launch_resample(P, c->N, logw, U, c->d_scan, anc, ess, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_resample_noalloc(int32_t N, int32_t P, const double* logw, const uint32_t* U,
                                  int32_t* anc, double* ess, void* stream) {
    if (!logw || !U || !anc || N < 1 || N > SMC_MAX_AIRCRAFT || P < 1)
        return fail(nullptr, SMC_EINVAL, "smc_k_resample_noalloc: bad arguments");
    if ((int64_t)N * P > kStaticScanDoubles)
        return fail(nullptr, SMC_EINVAL,
                    "smc_k_resample_noalloc: N * P = %lld exceeds the static workspace of %lld",
                    (long long)N * P, (long long)kStaticScanDoubles);
    const hipError_t e = launch_resample_static(P, N, logw, U, anc, ess, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(nullptr, SMC_EDEVICE, "smc_k_resample_noalloc: %s", hipGetErrorString(e));
    return SMC_OK;
}

smc_status smc_k_gather_move(smc_ctx* c, int32_t P, const void* u_in, const int32_t* anc,
                             void* u_out, int64_t mpc_step, int32_t iter, int32_t jitter,
                             void* stream) {
    if (!c || !u_in || !anc || !u_out || P < 1 || u_in == u_out)
        return fail(c, SMC_EINVAL, "smc_k_gather_move: bad arguments");
    HIP_OK(c, launch_gather_move(c->prec, P, c->N, c->S * 3, u_in, anc, u_out,
                                 make_stream(c->seed, mpc_step, iter, P_MOVE, c->scen_id),
                                 c->sigma_move, jitter, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_propose(smc_ctx* c, int32_t P, const void* u, void* u_prop, int64_t mpc_step,
                         int32_t iter, void* stream) {
    if (!c || !u || !u_prop || P < 1) return fail(c, SMC_EINVAL, "smc_k_propose: bad arguments");
    HIP_OK(c, launch_propose(c->prec, (int64_t)P * c->N * c->S * 3, u, u_prop,
                             make_stream(c->seed, mpc_step, iter, P_MOVE, c->scen_id), c->sigma_move,
                             pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_accept(smc_ctx* c, int32_t P, void* u, const void* u_prop, double* chat,
                        const double* chat_prop, uint8_t* feas_pn, const uint8_t* feas_prop,
                        double* logw, const double* logw_prop, int64_t mpc_step, int32_t iter,
                        int32_t* accepted, void* stream) {
    if (!c || !u || !u_prop || !chat || !chat_prop || !feas_pn || !feas_prop || !logw || !logw_prop ||
        P < 1)
        return fail(c, SMC_EINVAL, "smc_k_accept: bad arguments");
    if (!accepted && P > c->L) return fail(c, SMC_EINVAL, "smc_k_accept: P exceeds n_particles");
    HIP_OK(c, launch_accept(c->prec, P, c->N, c->S * 3, u, u_prop, chat, chat_prop, feas_pn, feas_prop,
                            logw, logw_prop,
                            make_stream(c->seed, mpc_step, iter, P_ACCEPT, c->scen_id), accepted,
                            c->d_flags, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_rollout_grad(smc_ctx* c, const void* u, int32_t P, const void* W,
                              const double* states, const int32_t* k_active, int32_t horizon,
                              double* grad, void* stream) {
    if (!c || !u || !W || !states || !k_active || !grad || P < 1)
        return fail(c, SMC_EINVAL, "smc_k_rollout_grad: bad arguments");
    if (c->wind_model != SMC_WIND_SE)
        return fail(c, SMC_EINVAL, "smc_k_rollout_grad: static wind model only");
    smc_status vs = check_horizon(c, horizon);
    if (vs) return vs;
    if (!grad_supported(horizon, c->S))
        return fail(c, SMC_EINVAL, "gradient supports at most 16 segments and 400 steps");
    if (c->M > 64 && P > c->L)
        return fail(c, SMC_EINVAL, "smc_k_rollout_grad: P exceeds n_particles with more than 64 samples");
    RolloutParams rp = c->rp;
    rp.H = horizon;
    rp.P = P;
    HIP_OK(c, launch_rollout_grad(c->prec, rp, u, W, states, k_active, c->d_acpar, c->d_targets,
                                  c->d_kind, c->d_Wt, c->d_gpart, grad, pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_mala_propose(smc_ctx* c, int32_t P, const void* u, const double* grad,
                              double beta, void* u_prop, int64_t mpc_step, int32_t iter,
                              void* stream) {
    if (!c || !u || !grad || !u_prop || P < 1) return fail(c, SMC_EINVAL, "smc_k_mala_propose: bad arguments");
    HIP_OK(c, launch_mala_propose(c->prec, (int64_t)P * c->N * c->S * 3, u, grad,
                                  -beta / (double)c->M, c->mala_step,
                                  make_stream(c->seed, mpc_step, iter, P_MALA, c->scen_id), u_prop,
                                  pick(c, stream)));
    return SMC_OK;
}

smc_status smc_k_mala_accept(smc_ctx* c, int32_t P, void* u, const void* u_prop, const double* grad,
                             const double* grad_prop, double beta, double* chat,
                             const double* chat_prop, uint8_t* feas_pn, const uint8_t* feas_prop,
                             double* logw, const double* logw_prop, int64_t mpc_step, int32_t iter,
                             int32_t* accepted, void* stream) {
    if (!c || !u || !u_prop || !grad || !grad_prop || !chat || !chat_prop || !feas_pn || !feas_prop ||
        !logw || !logw_prop || !accepted || P < 1)
        return fail(c, SMC_EINVAL, "smc_k_mala_accept: bad arguments");
    const int D = c->S * 3;
    hipStream_t st = pick(c, stream);
    HIP_OK(c, launch_mala_decide(c->prec, P, c->N, D, u, u_prop, grad, grad_prop, -beta / (double)c->M,
                                 c->mala_step, logw, logw_prop,
                                 make_stream(c->seed, mpc_step, iter, P_ACCEPT, c->scen_id), accepted,
                                 st));
    HIP_OK(c, launch_accept_apply(c->prec, P, c->N, D, u, u_prop, chat, chat_prop, feas_pn, feas_prop,
                                  logw, logw_prop, accepted, st));
    return SMC_OK;
}

smc_status smc_set_rollout_layout(smc_ctx* c, int32_t layout) {
    if (!c || layout < 0 || layout > 4) return fail(c, SMC_EINVAL, "smc_set_rollout_layout: bad arguments");
    if (layout == 2 && !rollout_wm_supported(c->N))
        return fail(c, SMC_EINVAL, "world-per-lane rollout supports at most %d aircraft", kWorldLaneMaxN);
    if (c->rp.control_model == SMC_CONTROLS_PAPER && layout != 0 && layout != 2)
        return fail(c, SMC_EINVAL, "the paper's controls run the world-per-lane rollout only");
    if ((layout == 3 && !rollout_pw_supported(c->N, c->prec)) ||
        (layout == 4 && !rollout_pt_supported(c->N, c->prec)))
        return fail(c, SMC_EINVAL, "particle-per-wave and particle-tile rollouts: FP32 contexts only");
    if ((layout == 1 || layout == 3 || layout == 4) && c->wind_model != SMC_WIND_SE)
        return fail(c, SMC_EINVAL, "time-correlated wind runs the world-per-lane rollout only");
    c->layout = layout;
    return SMC_OK;
}

smc_status smc_k_select(smc_ctx* c, int32_t P, const double* logw, const double* chat, double beta,
                        int32_t* best, void* stream) {
    if (!c || !logw || !chat || !best || P < 1) return fail(c, SMC_EINVAL, "smc_k_select: bad arguments");
    HIP_OK(c, launch_select(P, c->N, logw, chat, beta, best, pick(c, stream)));
    return SMC_OK;
}

}  // extern "C"
