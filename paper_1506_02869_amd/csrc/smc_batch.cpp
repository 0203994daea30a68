// Host side of the batched engine: validation across the batch, the
// concatenated device buffers, the work plan of the persistent rollout, the
// update's launch sequence (Alg. 1 for every scenario at once), its capture
// in a HIP graph, and the launch-shape autotuner.
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
#include "smc_batch.h"

using namespace smc;

namespace {

std::string g_batch_error;

}  // namespace

struct smc_batch {
    int ns = 0, L = 0, M = 0, K = 0, G = 0, prec = 0, move = 0;
    size_t rsz = 8;
    std::vector<int> N, S, Hmax, bucket;
    std::vector<int> off_n;                             // ns + 1
    std::vector<int64_t> off_u, off_pn, off_ctrl, off_cost;  // ns + 1
    int rows = 0;                                       // sum N
    int64_t max_count = 0, max_pn = 0;                  // max L N D, max L N
    size_t gpart_elems = 1;                             // largest adjoint chunk partials
    int64_t n_items = 0;
    int bstart[kNumBuckets] = {}, bcount[kNumBuckets] = {};
    std::vector<int> plan_h;   // horizons of the current plan
    int plan_order = -1;
    smc_batch_tuning tune;
    int cus = 0;
    int grid[kNumBuckets] = {};   // persistent rollout workgroups per bucket

    // host mirrors (pinned): table, step header, wind means, items
    BatchScen* h_tab = nullptr;
    BatchStep* h_hdr = nullptr;
    double* h_wmean = nullptr;
    BatchItem* h_items = nullptr;

    // device
    BatchScen* d_tab = nullptr;
    BatchStep* d_hdr = nullptr;
    double* d_wmean = nullptr;
    BatchItem* d_items = nullptr;
    int32_t* d_row_scen = nullptr;
    double* d_beta = nullptr;
    void* d_acR = nullptr;
    double *d_acpar = nullptr, *d_targets = nullptr;
    int8_t* d_kind = nullptr;
    void *d_Lfac = nullptr, *d_Z = nullptr, *d_W = nullptr;
    void* d_wpart = nullptr;   // wind GEMM chunk products (few-tile shapes)
    // the fields' grouped product, as the single-scenario context: sigma
    // Lx (x) Ly [nh][nh] real, L_z double, the level-mixed normals
    bool wind_grouped = false;
    int nx = 0, ny = 0, nz = 0;
    void *d_Lh = nullptr, *d_Y = nullptr;
    double *d_Lzd = nullptr, *d_one = nullptr;
    void *d_u = nullptr, *d_u2 = nullptr, *d_up = nullptr;
    // Langevin moves: the adjoint's gradients of the particles and of the
    // proposals (laid out like the particles), its chunk partials and its
    // sample-interleaved copy of one scenario's fields (reused scenario by
    // scenario)
    double *d_g = nullptr, *d_g2 = nullptr, *d_gpart = nullptr;
    void* d_Wt = nullptr;
    double* d_cost = nullptr;
    uint8_t* d_feas = nullptr;
    double *d_chat = nullptr, *d_logw = nullptr, *d_chat2 = nullptr, *d_logw2 = nullptr;
    uint8_t *d_feaspn = nullptr, *d_feaspn2 = nullptr;
    int32_t* d_anc = nullptr;
    double* d_scan = nullptr;
    uint32_t* d_U = nullptr;
    int32_t* d_flags = nullptr;
    int32_t* d_best = nullptr;
    double* d_states = nullptr;
    int32_t* d_kact = nullptr;
    double *d_ctrl = nullptr, *d_costout = nullptr;
    int32_t* d_status = nullptr;
    // counters (uint32): [queues 2 K kNumBuckets][steps 2 kStepSlots u64][accepted ns]
    uint32_t* d_cnt = nullptr;
    int64_t n_cnt = 0, cnt_steps = 0, cnt_acc = 0;

    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_up = nullptr;
    std::vector<hipEvent_t> ev_pass;   // pairs bracketing the rollout passes (timed updates)
    bool up_pending = false;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    std::vector<void*> bufs, pinned;
    std::string err;
};

namespace {

smc_status bfail(smc_batch* b, smc_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf; else g_batch_error = buf;
    return code;
}

#define BHIP(b, expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), SMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
smc_status balloc(smc_batch* b, T** p, size_t count, size_t elem = sizeof(T)) {
    size_t bytes = count * elem;
    if (bytes == 0) bytes = 16;
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return bfail(b, SMC_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    b->bufs.push_back(v);
    *p = (T*)v;
    return SMC_OK;
}

template <typename T>
smc_status halloc(smc_batch* b, T** p, size_t count) {
    void* v = nullptr;
    hipError_t e = hipHostMalloc(&v, std::max<size_t>(count * sizeof(T), 16), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return bfail(b, SMC_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    b->pinned.push_back(v);
    *p = (T*)v;
    return SMC_OK;
}

bool same3(const double* a, const double* b) { return a[0] == b[0] && a[1] == b[1] && a[2] == b[2]; }

smc_status validate_batch(const smc_scenario* sc, int ns) {
    if (!sc) return bfail(nullptr, SMC_EINVAL, "scenarios is NULL");
    if (ns < 1 || ns > SMC_BATCH_MAX_SCENARIOS)
        return bfail(nullptr, SMC_EINVAL, "n_scen must be in [1, %d]", SMC_BATCH_MAX_SCENARIOS);
    const smc_scenario& a = sc[0];
    int64_t rows = 0;
    for (int s = 0; s < ns; ++s) {
        std::string msg;
        if (sc[s].weighting != SMC_WEIGHT_TEMPERED)
            return bfail(nullptr, SMC_EINVAL, "scenario %d: the batched form takes the tempered weighting only", s);
        if (sc[s].wind_model != SMC_WIND_SE)
            return bfail(nullptr, SMC_EINVAL, "scenario %d: the batched form takes the static wind model only", s);
        if (sc[s].warm_start != 0)
            return bfail(nullptr, SMC_EINVAL, "scenario %d: warm_start is not supported in the batched form", s);
        if (sc[s].control_model != SMC_CONTROLS_KINEMATIC)
            return bfail(nullptr, SMC_EINVAL, "scenario %d: the batched form takes the kinematic controls only", s);
        if (host::validate_scenario(&sc[s], msg))
            return bfail(nullptr, SMC_EINVAL, "scenario %d: %s", s, msg.c_str());
        const smc_scenario& x = sc[s];
        if (x.n_aircraft > SMC_BATCH_MAX_AIRCRAFT)
            return bfail(nullptr, SMC_EINVAL, "scenario %d: batched form takes at most %d aircraft",
                         s, SMC_BATCH_MAX_AIRCRAFT);
        if (x.n_particles != a.n_particles || x.n_wind != a.n_wind || x.n_iters != a.n_iters)
            return bfail(nullptr, SMC_EINVAL,
                         "scenario %d: n_particles, n_wind and n_iters must match scenario 0", s);
        if (x.precision != a.precision || x.move != a.move)
            return bfail(nullptr, SMC_EINVAL, "scenario %d: precision and move must match scenario 0", s);
        if (x.grid_n[0] != a.grid_n[0] || x.grid_n[1] != a.grid_n[1] || x.grid_n[2] != a.grid_n[2] ||
            !same3(x.box, a.box) || x.wind_sigma != a.wind_sigma || x.wind_ell != a.wind_ell ||
            x.wind_nugget != a.wind_nugget)
            return bfail(nullptr, SMC_EINVAL,
                         "scenario %d: wind grid, box and covariance must match scenario 0 "
                         "(one shared factor)", s);
        rows += x.n_aircraft;
    }
    const double G = (double)a.grid_n[0] * a.grid_n[1] * a.grid_n[2];
    if (G * 2.0 * a.n_wind * ns >= 2147483647.0)
        return bfail(nullptr, SMC_EINVAL, "batch wind matrix exceeds 2^31 elements");
    if ((double)rows * a.n_particles >= 2147483647.0)
        return bfail(nullptr, SMC_EINVAL, "batch resampling rows exceed 2^31 elements");
    return SMC_OK;
}

// Work plan: items of 64 worlds per scenario, grouped by bucket; within a
// bucket scenarios by decreasing N^2 H (ties: lower index first) or in
// scenario order.
smc_status make_plan(int ns, const int32_t* Nv, const int32_t* Hv, int L, int M, int order,
                     int* bstart, int* bcount, int32_t* iscen, int32_t* iworld,
                     int64_t capacity, int64_t* n_items, std::string& msg) {
    const int64_t worlds = (int64_t)L * M;
    const int64_t per = (worlds + kItemWorlds - 1) / kItemWorlds;
    const int64_t total = per * ns;
    if (n_items) *n_items = total;
    if (worlds > 2147483647LL - kItemWorlds) { msg = "L M exceeds 2^31"; return SMC_EINVAL; }
    if (capacity < total) { msg = "item capacity below the item count"; return SMC_EINVAL; }
    std::vector<int> order_idx(ns);
    for (int s = 0; s < ns; ++s) order_idx[s] = s;
    if (order == 0)
        std::stable_sort(order_idx.begin(), order_idx.end(), [&](int x, int y) {
            const double cx = (double)Nv[x] * Nv[x] * Hv[x], cy = (double)Nv[y] * Nv[y] * Hv[y];
            return cx > cy;
        });
    int64_t pos = 0;
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        bstart[bk] = (int)pos;
        for (int q = 0; q < ns; ++q) {
            const int s = order_idx[q];
            if (bucket_of(Nv[s]) != bk) continue;
            for (int64_t t = 0; t < per; ++t) {
                iscen[pos] = s;
                iworld[pos] = (int32_t)(t * kItemWorlds);
                ++pos;
            }
        }
        bcount[bk] = (int)(pos - bstart[bk]);
    }
    return SMC_OK;
}

// Default lanes per workgroup: 256 (FP32) / 128 (FP64), the single-scenario
// kernel's choice, which keeps the staged controls within 64 KB of LDS.
int tune_block(const smc_batch* b, int bk) {
    return b->tune.block[bk] ? b->tune.block[bk] : (b->prec == SMC_FP64 ? 128 : 256);
}
int tune_mult(const smc_batch* b, int bk) { return b->tune.grid_mult[bk] ? b->tune.grid_mult[bk] : 1; }

int rollout_grid(const smc_batch* b, int bk, int block, int mult) {
    const int res = std::max(1, b_rollout_resident(b->prec, bk, block));
    const int64_t cap = (int64_t)b->cus * res * mult;
    const int64_t need = ((int64_t)b->bcount[bk] * kItemWorlds + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min(cap, need));
}

// Workgroups of each bucket's persistent launch for the installed tuning
// (occupancy queries stay out of the update, which may be under capture).
void refresh_grids(smc_batch* b) {
    for (int bk = 0; bk < kNumBuckets; ++bk)
        b->grid[bk] = b->bcount[bk] ? rollout_grid(b, bk, tune_block(b, bk), tune_mult(b, bk)) : 0;
}

void drop_graph(smc_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

// One rollout pass over every bucket present; `pass` selects the queue
// counters of this pass.
hipError_t rollout_pass(smc_batch* b, int pass, const void* u, int* launches, hipStream_t st) {
    unsigned long long* steps = reinterpret_cast<unsigned long long*>(b->d_cnt + b->cnt_steps);
    for (int bk = kNumBuckets - 1; bk >= 0; --bk) {
        if (!b->bcount[bk]) continue;
        hipError_t e = launch_b_rollout(b->prec, bk, b->d_tab, b->d_items + b->bstart[bk],
                                        b->bcount[bk], b->d_cnt + (int64_t)pass * kNumBuckets + bk,
                                        u, steps, tune_block(b, bk), b->grid[bk], st);
        if (e != hipSuccess) return e;
        if (launches) ++*launches;
    }
    return hipSuccess;
}

// Gradient of the fuel + time cost of particles `u` for every scenario (one
// adjoint launch per scenario, on its fields, states and aircraft tables;
// the horizon is this update's).
hipError_t batch_grad(smc_batch* b, const void* u, double* g, hipStream_t st) {
    for (int s = 0; s < b->ns; ++s) {
        const BatchScen& t = b->h_tab[s];
        const hipError_t e = launch_rollout_grad(
            b->prec, t.rp, (const char*)u + (size_t)t.off_u * b->rsz, t.ra.W, t.ra.states,
            t.ra.k_active, t.ra.acpar, t.ra.targets, t.ra.kind, b->d_Wt, b->d_gpart, g + t.off_u,
            st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The device work of one update; every per-update input is already in the
// batch's device buffers (table, header, wind means, states, items).
// Every scenario's fields from its normals: W = wbar_s + L Z, through the
// same grouped product as the single-scenario context (levels' factor, then
// the horizontal factor's GEMM) or the dense factor, so that a scenario's
// fields equal its own context's bit for bit.
hipError_t batch_wind_fields(smc_batch* b, hipStream_t st) {
    if (!b->wind_grouped)
        return launch_wind_gemm_grouped(b->prec, b->d_Lfac, b->d_Z, b->d_wmean, b->M, b->G,
                                        b->ns * b->M, b->d_W, b->d_wpart, st);
    const int nh = b->nx * b->ny;
    const hipError_t e = launch_wind_levels(b->prec, b->d_Z, b->d_Lzd, nh, b->nz, b->ns * b->M,
                                            b->d_Y, st);
    if (e != hipSuccess) return e;
    return launch_wind_gemm_levels_grouped(b->prec, b->d_Lh, b->d_Y, b->d_wmean, b->M, nh, b->nz,
                                           b->ns * b->M, b->d_W, b->d_wpart, st);
}

hipError_t enqueue_update(smc_batch* b, hipStream_t st, int* launches, bool timed) {
    hipError_t e;
#define Q(expr) do { if ((e = (expr)) != hipSuccess) return e; } while (0)
    auto mark = [&](int q) { return timed ? hipEventRecord(b->ev_pass[q], st) : hipSuccess; };
    const int ns = b->ns, L = b->L, M = b->M, K = b->K;
    Q(launch_b_fill(b->d_cnt, b->n_cnt, st));
    void* u = b->d_u;
    void* u2 = b->d_u2;
    Q(launch_b_init(b->prec, b->d_tab, b->d_hdr, ns, b->max_count, u, st));
    int pass = 0;
    for (int J = 0; J < K; ++J) {
        Q(launch_b_normals(b->prec, b->d_tab, b->d_hdr, ns, J, b->G, M, b->d_Z, st));
        Q(batch_wind_fields(b, st));
        Q(mark(2 * pass));
        Q(rollout_pass(b, pass, u, launches, st));
        Q(mark(2 * pass + 1));
        ++pass;
        Q(launch_b_reduce(b->d_tab, ns, J, b->max_pn, b->d_chat, b->d_feaspn, b->d_logw, st));
        if (b->move == SMC_MOVE_MALA) {
            // Langevin: gradients of the particles, proposals, their rollout
            // and gradients, the decision (one adjoint launch per scenario)
            Q(batch_grad(b, u, b->d_g, st));
            Q(launch_b_mala_propose(b->prec, b->d_tab, b->d_hdr, ns, J, b->max_count, u, b->d_g,
                                    b->d_up, st));
            Q(mark(2 * pass));
            Q(rollout_pass(b, pass, b->d_up, launches, st));
            Q(mark(2 * pass + 1));
            ++pass;
            Q(launch_b_reduce(b->d_tab, ns, J, b->max_pn, b->d_chat2, b->d_feaspn2, b->d_logw2, st));
            Q(batch_grad(b, b->d_up, b->d_g2, st));
            Q(launch_b_mala_accept(b->prec, b->d_tab, b->d_hdr, ns, J, L, b->max_count, u, b->d_up,
                                   b->d_g, b->d_g2, b->d_chat, b->d_chat2, b->d_feaspn,
                                   b->d_feaspn2, b->d_logw, b->d_logw2, b->d_flags,
                                   b->d_cnt + b->cnt_acc, st));
        }
        if (b->move == SMC_MOVE_RWMH) {
            Q(launch_b_propose(b->prec, b->d_tab, b->d_hdr, ns, J, b->max_count, u, b->d_up, st));
            Q(mark(2 * pass));
            Q(rollout_pass(b, pass, b->d_up, launches, st));
            Q(mark(2 * pass + 1));
            ++pass;
            Q(launch_b_reduce(b->d_tab, ns, J, b->max_pn, b->d_chat2, b->d_feaspn2, b->d_logw2, st));
            Q(launch_b_accept(b->prec, b->d_tab, b->d_hdr, ns, J, L, b->max_count, u, b->d_up,
                              b->d_chat, b->d_chat2, b->d_feaspn, b->d_feaspn2, b->d_logw,
                              b->d_logw2, b->d_flags, b->d_cnt + b->cnt_acc, st));
        }
        if (J == K - 1) break;
        Q(launch_b_resample_offsets(b->d_tab, b->d_hdr, b->d_row_scen, b->rows, J, b->d_U, st));
        Q(launch_b_resample(b->d_tab, b->d_row_scen, b->rows, L, b->d_logw, b->d_U, b->d_scan,
                            b->d_anc, st));
        Q(launch_b_gather_move(b->prec, b->d_tab, b->d_hdr, ns, J, b->max_count, u, b->d_anc, u2,
                               b->move == SMC_MOVE_JITTER ? 1 : 0, st));
        std::swap(u, u2);
    }
    Q(launch_b_select(b->d_tab, ns, K - 1, L, b->d_logw, b->d_chat, b->d_best, st));
    Q(launch_b_write_result(b->prec, b->d_tab, ns, u, b->d_best, b->d_chat, b->d_ctrl,
                            b->d_costout, b->d_status, st));
#undef Q
    return hipSuccess;
}

smc_status check_inputs(smc_batch* b, const double* wind_mean, const int32_t* horizons) {
    if (!wind_mean || !horizons) return bfail(b, SMC_EINVAL, "wind_mean and horizons are required");
    for (int s = 0; s < b->ns; ++s) {
        const int h = horizons[s];
        if (h < 1 || h > b->Hmax[s])
            return bfail(b, SMC_EINVAL, "scenario %d: horizon %d outside [1, %d]", s, h, b->Hmax[s]);
        if (h < b->S[s])
            return bfail(b, SMC_EINVAL, "scenario %d: horizon %d shorter than n_segments %d", s, h,
                         b->S[s]);
    }
    return SMC_OK;
}

// Per-update inputs into the device buffers: table (horizons), header,
// wind means, work plan (when horizons or order changed), states.
smc_status upload(smc_batch* b, int64_t mpc_step, const double* states, const int32_t* kact,
                  bool dev_inputs, const double* wind_mean, const int32_t* horizons,
                  hipStream_t st) {
    if (b->up_pending) {   // staging buffers are in use until the last upload finished
        BHIP(b, hipEventSynchronize(b->ev_up));
        b->up_pending = false;
    }
    const int ns = b->ns;
    for (int s = 0; s < ns; ++s) b->h_tab[s].rp.H = horizons[s];
    b->h_hdr->mpc_step = mpc_step;
    std::memcpy(b->h_wmean, wind_mean, sizeof(double) * 2 * ns);
    bool replan = b->plan_order != b->tune.order ||
                  !std::equal(b->plan_h.begin(), b->plan_h.end(), horizons);
    if (replan) {
        std::vector<int32_t> is(b->n_items), iw(b->n_items);
        std::string msg;
        int64_t n = 0;
        if (make_plan(ns, b->N.data(), horizons, b->L, b->M, b->tune.order, b->bstart, b->bcount,
                      is.data(), iw.data(), b->n_items, &n, msg))
            return bfail(b, SMC_EINVAL, "plan: %s", msg.c_str());
        for (int64_t q = 0; q < b->n_items; ++q) b->h_items[q] = BatchItem{is[q], iw[q]};
        b->plan_h.assign(horizons, horizons + ns);
        b->plan_order = b->tune.order;
        // the adjoint's launches take the horizons as arguments: a captured
        // graph of a Langevin batch holds the old ones
        if (b->move == SMC_MOVE_MALA) drop_graph(b);
        BHIP(b, hipMemcpyAsync(b->d_items, b->h_items, sizeof(BatchItem) * b->n_items,
                               hipMemcpyHostToDevice, st));
    }
    BHIP(b, hipMemcpyAsync(b->d_tab, b->h_tab, sizeof(BatchScen) * ns, hipMemcpyHostToDevice, st));
    BHIP(b, hipMemcpyAsync(b->d_hdr, b->h_hdr, sizeof(BatchStep), hipMemcpyHostToDevice, st));
    BHIP(b, hipMemcpyAsync(b->d_wmean, b->h_wmean, sizeof(double) * 2 * ns, hipMemcpyHostToDevice, st));
    const hipMemcpyKind k = dev_inputs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    BHIP(b, hipMemcpyAsync(b->d_states, states, sizeof(double) * 6 * b->rows, k, st));
    BHIP(b, hipMemcpyAsync(b->d_kact, kact, sizeof(int32_t) * b->rows, k, st));
    BHIP(b, hipEventRecord(b->ev_up, st));
    b->up_pending = true;
    return SMC_OK;
}

smc_status run_update(smc_batch* b, int64_t mpc_step, const double* states, const int32_t* kact,
                      bool dev_inputs, const double* wind_mean, const int32_t* horizons,
                      smc_batch_info* info, hipStream_t st) {
    smc_status r = check_inputs(b, wind_mean, horizons);
    if (r) return r;
    if ((r = upload(b, mpc_step, states, kact, dev_inputs, wind_mean, horizons, st))) return r;
    if (info) BHIP(b, hipEventRecord(b->ev0, st));
    int launches = 0;
    if (b->use_graph) {
        if (!b->gexec) {
            BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue_update(b, b->stream, nullptr, false);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bfail(b, SMC_EDEVICE, "graph capture failed: %s",
                             hipGetErrorString(e != hipSuccess ? e : e2));
            }
            b->graph = g;
            hipError_t e3 = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
            if (e3 != hipSuccess) {
                drop_graph(b);
                return bfail(b, SMC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
            }
        }
        BHIP(b, hipGraphLaunch(b->gexec, st));
        for (int bk = 0; bk < kNumBuckets; ++bk)
            if (b->bcount[bk]) launches += b->K * (b->move != SMC_MOVE_JITTER ? 2 : 1);
    } else {
        BHIP(b, enqueue_update(b, st, &launches, info != nullptr));
    }
    if (!info) return SMC_OK;
    BHIP(b, hipEventRecord(b->ev1, st));
    BHIP(b, hipEventSynchronize(b->ev1));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
    std::vector<uint32_t> cnt(b->n_cnt);
    BHIP(b, hipMemcpy(cnt.data(), b->d_cnt, sizeof(uint32_t) * b->n_cnt, hipMemcpyDeviceToHost));
    std::vector<uint8_t> fe((size_t)b->L * b->rows);
    BHIP(b, hipMemcpy(fe.data(), b->d_feaspn, fe.size(), hipMemcpyDeviceToHost));
    unsigned long long steps[2 * kStepSlots];
    std::memcpy(steps, cnt.data() + b->cnt_steps, sizeof steps);
    unsigned long long tot = 0, totp = 0;
    for (int q = 0; q < kStepSlots; ++q) { tot += steps[q]; totp += steps[kStepSlots + q]; }
    uint64_t acc = 0;
    for (int s = 0; s < b->ns; ++s) acc += cnt[b->cnt_acc + s];
    uint64_t nf = 0;
    for (uint8_t f : fe) nf += f;
    info->n_scenarios = b->ns;
    info->iterations = b->K;
    info->aircraft_steps = (int64_t)tot;
    info->pair_tests = (int64_t)totp;
    info->ms_total = ms;
    info->accept_rate = b->move != SMC_MOVE_JITTER
                            ? (double)acc / ((double)b->K * b->L * b->ns) : 0.0;
    info->feasible_frac = fe.empty() ? 0.0 : (double)nf / (double)fe.size();
    info->graph = b->use_graph ? 1 : 0;
    info->rollout_launches = launches;
    info->rollout_passes = b->K * (b->move != SMC_MOVE_JITTER ? 2 : 1);
    info->ms_rollout = 0.0;
    if (!b->use_graph)
        for (int q = 0; q < info->rollout_passes; ++q) {
            float t = 0.f;
            BHIP(b, hipEventElapsedTime(&t, b->ev_pass[2 * q], b->ev_pass[2 * q + 1]));
            info->ms_rollout += t;
        }
    return SMC_OK;
}

smc_status check_tuning(smc_batch* b, const smc_batch_tuning* t) {
    if (!t) return bfail(b, SMC_EINVAL, "tuning is NULL");
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        const int bl = t->block[bk], gm = t->grid_mult[bk];
        if (bl != 0 && bl != 64 && bl != 128 && bl != 256)
            return bfail(b, SMC_EINVAL, "block[%d] must be 0, 64, 128 or 256", bk);
        if (gm < 0 || gm > 4) return bfail(b, SMC_EINVAL, "grid_mult[%d] must be in [0, 4]", bk);
    }
    if (t->order != 0 && t->order != 1) return bfail(b, SMC_EINVAL, "order must be 0 or 1");
    return SMC_OK;
}

}  // namespace

extern "C" {

const char* smc_batch_last_error(const smc_batch* b) {
    return b ? b->err.c_str() : g_batch_error.c_str();
}

void smc_batch_destroy(smc_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();   // device-form calls may be queued on caller streams
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (void* p : b->bufs) (void)hipFree(p);
    for (void* p : b->pinned) (void)hipHostFree(p);
    for (hipEvent_t e : {b->ev0, b->ev1, b->ev_up})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->ev_pass)
        if (e) (void)hipEventDestroy(e);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

smc_status smc_batch_plan(int32_t n_scen, const int32_t* n_aircraft, const int32_t* horizons,
                          int32_t n_particles, int32_t n_wind, int32_t order,
                          int32_t* bucket_start, int32_t* bucket_count, int32_t* item_scen,
                          int32_t* item_world0, int64_t capacity, int64_t* n_items) {
    if (n_scen < 1 || !n_aircraft || !horizons || !bucket_start || !bucket_count ||
        (capacity > 0 && (!item_scen || !item_world0)))
        return bfail(nullptr, SMC_EINVAL, "smc_batch_plan: bad arguments");
    if (n_particles < 1 || n_wind < 1 || (order != 0 && order != 1))
        return bfail(nullptr, SMC_EINVAL, "smc_batch_plan: bad sizes or order");
    for (int s = 0; s < n_scen; ++s)
        if (n_aircraft[s] < 1 || n_aircraft[s] > SMC_BATCH_MAX_AIRCRAFT || horizons[s] < 1)
            return bfail(nullptr, SMC_EINVAL, "smc_batch_plan: scenario %d out of range", s);
    std::string msg;
    int bs[kNumBuckets], bc[kNumBuckets];
    const smc_status r = make_plan(n_scen, n_aircraft, horizons, n_particles, n_wind, order, bs, bc,
                                   item_scen, item_world0, capacity, n_items, msg);
    if (r) return bfail(nullptr, r, "smc_batch_plan: %s", msg.c_str());
    for (int bk = 0; bk < kNumBuckets; ++bk) { bucket_start[bk] = bs[bk]; bucket_count[bk] = bc[bk]; }
    return SMC_OK;
}

smc_status smc_batch_init(const smc_scenario* sc, int32_t ns, smc_batch** out) {
    if (!out) return bfail(nullptr, SMC_EINVAL, "out is NULL");
    *out = nullptr;
    smc_status vs = validate_batch(sc, ns);
    if (vs) return vs;
    smc_batch* b = new (std::nothrow) smc_batch();
    if (!b) return bfail(nullptr, SMC_ENOMEM, "host allocation failed");
    auto bail = [&](smc_status code) {
        g_batch_error = b->err;
        smc_batch_destroy(b);
        return code;
    };
    const smc_scenario& a = sc[0];
    b->ns = ns; b->L = a.n_particles; b->M = a.n_wind; b->K = a.n_iters;
    b->G = a.grid_n[0] * a.grid_n[1] * a.grid_n[2];
    b->nx = a.grid_n[0]; b->ny = a.grid_n[1]; b->nz = a.grid_n[2];
    b->wind_grouped = b->nz <= kMaxWindLevels;   // as the single-scenario context
    b->prec = a.precision; b->move = a.move;
    b->rsz = b->prec == SMC_FP64 ? sizeof(double) : sizeof(float);
    std::memset(&b->tune, 0, sizeof b->tune);
    b->off_n.assign(ns + 1, 0);
    for (auto* v : {&b->off_u, &b->off_pn, &b->off_ctrl, &b->off_cost}) v->assign(ns + 1, 0);
    for (int s = 0; s < ns; ++s) {
        const int N = sc[s].n_aircraft, S = sc[s].n_segments;
        b->N.push_back(N); b->S.push_back(S); b->Hmax.push_back(sc[s].horizon_max);
        b->bucket.push_back(bucket_of(N));
        const int64_t cnt = (int64_t)b->L * N * S * 3;
        b->off_n[s + 1] = b->off_n[s] + N;
        b->off_u[s + 1] = b->off_u[s] + cnt;
        b->off_pn[s + 1] = b->off_pn[s] + (int64_t)b->L * N;
        b->off_ctrl[s + 1] = b->off_ctrl[s] + (int64_t)N * S * 3;
        b->off_cost[s + 1] = b->off_cost[s] + 1 + N;
        b->max_count = std::max(b->max_count, cnt);
        b->max_pn = std::max(b->max_pn, (int64_t)b->L * N);
        b->gpart_elems = std::max(b->gpart_elems, grad_partial_elems(b->L, N, S, b->M));
    }
    b->rows = b->off_n[ns];
    b->n_items = (int64_t)ns * (((int64_t)b->L * b->M + kItemWorlds - 1) / kItemWorlds);
    if (b->n_items >= 2147483647LL) {
        bfail(b, SMC_EINVAL, "batch has more than 2^31 work items");
        return bail(SMC_EINVAL);
    }

    std::vector<double> Lx, Ly, Lz;
    if (!host::axis_factor(a.grid_n[0], -0.5 * a.box[0], 0.5 * a.box[0], a.wind_ell, a.wind_nugget, Lx) ||
        !host::axis_factor(a.grid_n[1], -0.5 * a.box[1], 0.5 * a.box[1], a.wind_ell, a.wind_nugget, Ly) ||
        !host::axis_factor(a.grid_n[2], 0.0, a.box[2], a.wind_ell, a.wind_nugget, Lz)) {
        bfail(b, SMC_ENOTSPD, "wind covariance not positive definite (raise wind_nugget)");
        return bail(SMC_ENOTSPD);
    }
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            bfail(b, SMC_EDEVICE, "no HIP device");
            return bail(SMC_EDEVICE);
        }
        b->cus = prop.multiProcessorCount;
    }
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_up, hipEventDisableTiming) != hipSuccess) {
        bfail(b, SMC_EDEVICE, "stream / event creation failed");
        return bail(SMC_EDEVICE);
    }
    b->ev_pass.assign((size_t)4 * b->K, nullptr);
    for (auto& e : b->ev_pass)
        if (hipEventCreate(&e) != hipSuccess) {
            bfail(b, SMC_EDEVICE, "event creation failed");
            return bail(SMC_EDEVICE);
        }
    const size_t L = b->L, M = b->M, G = b->G, rows = b->rows, nsz = ns;
    const size_t nu = (size_t)b->off_u[ns], npn = (size_t)b->off_pn[ns];
    b->cnt_steps = 2 * (int64_t)b->K * kNumBuckets;           // even: 8-byte aligned u64 slots
    b->cnt_acc = b->cnt_steps + 4 * kStepSlots;
    b->n_cnt = b->cnt_acc + ns;
    double *d_Lx = nullptr, *d_Ly = nullptr, *d_Lz = nullptr;
    smc_status st;
    if ((st = balloc(b, &b->d_tab, nsz)) || (st = balloc(b, &b->d_hdr, 1)) ||
        (st = balloc(b, &b->d_wmean, 2 * nsz)) || (st = balloc(b, &b->d_items, (size_t)b->n_items)) ||
        (st = balloc(b, &b->d_row_scen, rows)) || (st = balloc(b, &b->d_beta, nsz * b->K)) ||
        (st = balloc<char>(b, (char**)&b->d_acR, rows * kAcR, b->rsz)) ||
        (st = balloc(b, &b->d_acpar, rows * SMC_AC_NPAR)) || (st = balloc(b, &b->d_targets, rows * 4)) ||
        (st = balloc(b, &b->d_kind, rows)) ||
        (st = balloc<char>(b, (char**)&b->d_Lfac, G * G, b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_Z, G * 2 * M * nsz, b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_W, G * 2 * M * nsz, b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_wpart,
                           std::max<size_t>({wind_gemm_part_elems((int)G, (int)(M * nsz)),
                                             b->wind_grouped ? wind_gemm_part_elems(
                                                                   a.grid_n[0] * a.grid_n[1],
                                                                   (int)(M * nsz) * a.grid_n[2])
                                                             : 0,
                                             (size_t)1}),
                           b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_u, nu, b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_u2, nu, b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_up, b->move != SMC_MOVE_JITTER ? nu : 1, b->rsz)) ||
        (st = balloc(b, &b->d_g, b->move == SMC_MOVE_MALA ? nu : 1)) ||
        (st = balloc(b, &b->d_g2, b->move == SMC_MOVE_MALA ? nu : 1)) ||
        (st = balloc<char>(b, (char**)&b->d_Wt, b->move == SMC_MOVE_MALA ? G * 2 * M : 1, b->rsz)) ||
        (st = balloc(b, &b->d_gpart, b->move == SMC_MOVE_MALA ? b->gpart_elems : 1)) ||
        (st = balloc<char>(b, (char**)&b->d_Lh,
                           b->wind_grouped ? (size_t)b->nx * b->ny * b->nx * b->ny : 1, b->rsz)) ||
        (st = balloc<char>(b, (char**)&b->d_Y, b->wind_grouped ? G * 2 * M * nsz : 1, b->rsz)) ||
        (st = balloc(b, &b->d_Lzd, (size_t)b->nz * b->nz)) || (st = balloc(b, &b->d_one, 1)) ||
        (st = balloc(b, &b->d_cost, M * npn)) || (st = balloc(b, &b->d_feas, M * npn)) ||
        (st = balloc(b, &b->d_chat, npn)) || (st = balloc(b, &b->d_logw, npn)) ||
        (st = balloc(b, &b->d_chat2, npn)) || (st = balloc(b, &b->d_logw2, npn)) ||
        (st = balloc(b, &b->d_feaspn, npn)) || (st = balloc(b, &b->d_feaspn2, npn)) ||
        (st = balloc(b, &b->d_anc, rows * L)) || (st = balloc(b, &b->d_scan, rows * L)) ||
        (st = balloc(b, &b->d_U, rows)) || (st = balloc(b, &b->d_flags, nsz * L)) ||
        (st = balloc(b, &b->d_best, 2 * nsz)) || (st = balloc(b, &b->d_states, rows * 6)) ||
        (st = balloc(b, &b->d_kact, rows)) || (st = balloc(b, &b->d_ctrl, (size_t)b->off_ctrl[ns])) ||
        (st = balloc(b, &b->d_costout, (size_t)b->off_cost[ns])) ||
        (st = balloc(b, &b->d_status, nsz)) || (st = balloc(b, &b->d_cnt, (size_t)b->n_cnt)) ||
        (st = balloc(b, &d_Lx, Lx.size())) || (st = balloc(b, &d_Ly, Ly.size())) ||
        (st = balloc(b, &d_Lz, Lz.size())))
        return bail(st);
    if ((st = halloc(b, &b->h_tab, nsz)) || (st = halloc(b, &b->h_hdr, 1)) ||
        (st = halloc(b, &b->h_wmean, 2 * nsz)) || (st = halloc(b, &b->h_items, (size_t)b->n_items)))
        return bail(st);

    // per-aircraft rows, tempering, pop grids, table
    std::vector<double> acpar(rows * SMC_AC_NPAR), targets(rows * 4), acR(rows * kAcR), beta(nsz * b->K);
    std::vector<int8_t> kind(rows);
    std::vector<int32_t> row_scen(rows);
    std::vector<float*> pops(ns, nullptr);
    for (int s = 0; s < ns; ++s) {
        const smc_scenario& x = sc[s];
        const int N = x.n_aircraft, o = b->off_n[s];
        std::memcpy(&acpar[(size_t)o * SMC_AC_NPAR], x.aircraft, sizeof(double) * N * SMC_AC_NPAR);
        std::memcpy(&targets[(size_t)o * 4], x.targets, sizeof(double) * N * 4);
        std::memcpy(&kind[o], x.kind, N);
        std::vector<double> t;
        host::fill_acR(&x, t);
        std::copy(t.begin(), t.end(), acR.begin() + (size_t)o * kAcR);
        for (int i = 0; i < N; ++i) row_scen[o + i] = s;
        for (int J = 0; J < b->K; ++J) beta[(size_t)s * b->K + J] = x.kappa * host::sample_schedule(J);
        const bool use_noise = x.popdense != nullptr && x.cost_w[8] != 0.0;
        if (x.popdense) {
            const size_t np = (size_t)x.pop_n[0] * x.pop_n[1];
            if ((st = balloc(b, &pops[s], np))) return bail(st);
            if (hipMemcpy(pops[s], x.popdense, np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
                bfail(b, SMC_EDEVICE, "population grid upload failed");
                return bail(SMC_EDEVICE);
            }
        }
        (void)use_noise;
    }
    const size_t rz = b->rsz;
    for (int s = 0; s < ns; ++s) {
        const smc_scenario& x = sc[s];
        BatchScen& t = b->h_tab[s];
        std::memset(&t, 0, sizeof t);
        host::fill_rollout_params(&x, t.rp);
        const int o = b->off_n[s];
        t.ra.u = nullptr;
        t.ra.W = (const char*)b->d_W + (size_t)s * M * G * 2 * rz;
        t.ra.states = b->d_states + (size_t)o * 6;
        t.ra.k_active = b->d_kact + o;
        t.ra.acpar = b->d_acpar + (size_t)o * SMC_AC_NPAR;
        t.ra.targets = b->d_targets + (size_t)o * 4;
        t.ra.kind = b->d_kind + o;
        t.ra.pop = pops[s];
        t.ra.cost = b->d_cost + (size_t)M * b->off_pn[s];
        t.ra.feas = b->d_feas + (size_t)M * b->off_pn[s];
        t.ra.steps = nullptr;
        t.acR = (const char*)b->d_acR + (size_t)o * kAcR * rz;
        t.beta = b->d_beta + (size_t)s * b->K;
        t.seed = x.seed;
        t.scen_id = x.scenario_id;
        t.N = x.n_aircraft; t.S = x.n_segments; t.D = 3 * x.n_segments;
        t.off_n = o;
        t.off_u = b->off_u[s];
        t.off_pn = b->off_pn[s];
        t.off_ctrl = b->off_ctrl[s];
        t.off_cost = b->off_cost[s];
        t.sigma_move = x.sigma_move;
        t.mala_step = x.mala_step;
        for (int c = 0; c < 3; ++c) { t.box.lo[c] = x.ctrl_lo[c]; t.box.sp[c] = x.ctrl_hi[c] - x.ctrl_lo[c]; }
    }
#define IHIP(expr)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            bfail(b, SMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
            return bail(SMC_EDEVICE);                                                    \
        }                                                                                \
    } while (0)
    IHIP(hipMemcpy(b->d_acpar, acpar.data(), acpar.size() * sizeof(double), hipMemcpyHostToDevice));
    IHIP(hipMemcpy(b->d_targets, targets.data(), targets.size() * sizeof(double), hipMemcpyHostToDevice));
    IHIP(hipMemcpy(b->d_kind, kind.data(), kind.size(), hipMemcpyHostToDevice));
    IHIP(hipMemcpy(b->d_row_scen, row_scen.data(), row_scen.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    IHIP(hipMemcpy(b->d_beta, beta.data(), beta.size() * sizeof(double), hipMemcpyHostToDevice));
    if (b->prec == SMC_FP64) {
        IHIP(hipMemcpy(b->d_acR, acR.data(), acR.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(acR.begin(), acR.end());
        IHIP(hipMemcpy(b->d_acR, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    IHIP(hipMemcpy(d_Lx, Lx.data(), Lx.size() * sizeof(double), hipMemcpyHostToDevice));
    IHIP(hipMemcpy(d_Ly, Ly.data(), Ly.size() * sizeof(double), hipMemcpyHostToDevice));
    IHIP(hipMemcpy(d_Lz, Lz.data(), Lz.size() * sizeof(double), hipMemcpyHostToDevice));
    IHIP(launch_kron_expand(b->prec, d_Lx, d_Ly, d_Lz, a.grid_n[0], a.grid_n[1], a.grid_n[2],
                            a.wind_sigma, b->d_Lfac, b->stream));
    if (b->wind_grouped) {   // sigma Lx (x) Ly (d_one: the 1 x 1 factor 1), and L_z
        const double one = 1.0;
        IHIP(hipMemcpy(b->d_one, &one, sizeof(double), hipMemcpyHostToDevice));
        IHIP(launch_kron_expand(b->prec, d_Lx, d_Ly, b->d_one, a.grid_n[0], a.grid_n[1], 1,
                                a.wind_sigma, b->d_Lh, b->stream));
        IHIP(hipMemcpy(b->d_Lzd, Lz.data(), Lz.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    IHIP(hipStreamSynchronize(b->stream));
#undef IHIP
    {   // initial plan (horizon_max) so that the bucket sizes and grids are known
        std::vector<int32_t> is(b->n_items), iw(b->n_items);
        std::string msg;
        if (make_plan(ns, b->N.data(), b->Hmax.data(), b->L, b->M, 0, b->bstart, b->bcount,
                      is.data(), iw.data(), b->n_items, nullptr, msg)) {
            bfail(b, SMC_EINVAL, "plan: %s", msg.c_str());
            return bail(SMC_EINVAL);
        }
        refresh_grids(b);
    }
    *out = b;
    return SMC_OK;
}

smc_status smc_batch_step(smc_batch* b, int64_t mpc_step, const double* states,
                          const int32_t* k_active, const double* wind_mean,
                          const int32_t* horizons, double* controls_out, double* exp_cost_out,
                          int32_t* status_out, smc_batch_info* info) {
    if (!b) return bfail(nullptr, SMC_EINVAL, "batch is NULL");
    if (!states || !k_active || !controls_out || !exp_cost_out || !status_out)
        return bfail(b, SMC_EINVAL, "NULL argument");
    hipStream_t st = b->stream;
    smc_status r = run_update(b, mpc_step, states, k_active, false, wind_mean, horizons, info, st);
    if (r < 0) return r;
    BHIP(b, hipMemcpyAsync(controls_out, b->d_ctrl, sizeof(double) * b->off_ctrl[b->ns],
                           hipMemcpyDeviceToHost, st));
    BHIP(b, hipMemcpyAsync(exp_cost_out, b->d_costout, sizeof(double) * b->off_cost[b->ns],
                           hipMemcpyDeviceToHost, st));
    BHIP(b, hipMemcpyAsync(status_out, b->d_status, sizeof(int32_t) * b->ns, hipMemcpyDeviceToHost, st));
    BHIP(b, hipStreamSynchronize(st));
    for (int s = 0; s < b->ns; ++s)
        if (status_out[s]) return SMC_INFEASIBLE;
    return SMC_OK;
}

smc_status smc_batch_step_dev(smc_batch* b, int64_t mpc_step, const double* d_states,
                              const int32_t* d_k_active, const double* wind_mean,
                              const int32_t* horizons, double* d_controls_out,
                              double* d_exp_cost_out, int32_t* d_status_out,
                              smc_batch_info* info, void* stream) {
    if (!b) return bfail(nullptr, SMC_EINVAL, "batch is NULL");
    if (!d_states || !d_k_active || !d_controls_out || !d_exp_cost_out)
        return bfail(b, SMC_EINVAL, "NULL device pointer");
    // NULL is the null (legacy default) stream: ordered with the caller's
    // default-stream work, as in the single-scenario device form
    hipStream_t st = (hipStream_t)stream;
    smc_status r = run_update(b, mpc_step, d_states, d_k_active, true, wind_mean, horizons, info, st);
    if (r < 0) return r;
    BHIP(b, hipMemcpyAsync(d_controls_out, b->d_ctrl, sizeof(double) * b->off_ctrl[b->ns],
                           hipMemcpyDeviceToDevice, st));
    BHIP(b, hipMemcpyAsync(d_exp_cost_out, b->d_costout, sizeof(double) * b->off_cost[b->ns],
                           hipMemcpyDeviceToDevice, st));
    if (d_status_out)
        BHIP(b, hipMemcpyAsync(d_status_out, b->d_status, sizeof(int32_t) * b->ns,
                               hipMemcpyDeviceToDevice, st));
    return SMC_OK;
}

smc_status smc_batch_set_graph(smc_batch* b, int32_t enable) {
    if (!b) return bfail(nullptr, SMC_EINVAL, "batch is NULL");
    if (enable != 0 && enable != 1) return bfail(b, SMC_EINVAL, "enable must be 0 or 1");
    if (!enable) drop_graph(b);
    b->use_graph = enable != 0;
    return SMC_OK;
}

smc_status smc_batch_get_tuning(const smc_batch* b, smc_batch_tuning* out) {
    if (!b || !out) return bfail(nullptr, SMC_EINVAL, "NULL argument");
    *out = b->tune;
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        out->block[bk] = tune_block(b, bk);
        out->grid_mult[bk] = tune_mult(b, bk);
    }
    return SMC_OK;
}

smc_status smc_batch_set_tuning(smc_batch* b, const smc_batch_tuning* t) {
    if (!b) return bfail(nullptr, SMC_EINVAL, "batch is NULL");
    smc_status r = check_tuning(b, t);
    if (r) return r;
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        const int bl = t->block[bk] ? t->block[bk] : (b->prec == SMC_FP64 ? 128 : 256);
        if (b->bcount[bk] && b_rollout_resident(b->prec, bk, bl) < 1)
            return bfail(b, SMC_EINVAL, "block[%d] = %d does not fit the device (LDS / registers)",
                         bk, bl);
    }
    if (b->stream) BHIP(b, hipStreamSynchronize(b->stream));
    b->tune = *t;
    refresh_grids(b);
    drop_graph(b);
    return SMC_OK;
}

smc_status smc_batch_autotune(smc_batch* b, int64_t mpc_step, const double* states,
                              const int32_t* k_active, const double* wind_mean,
                              const int32_t* horizons, int32_t reps, smc_batch_tuning* out) {
    if (!b) return bfail(nullptr, SMC_EINVAL, "batch is NULL");
    if (!states || !k_active) return bfail(b, SMC_EINVAL, "NULL argument");
    if (reps < 1 || reps > 100) return bfail(b, SMC_EINVAL, "reps must be in [1, 100]");
    hipStream_t st = b->stream;
    smc_status r = check_inputs(b, wind_mean, horizons);
    if (r) return r;
    if ((r = upload(b, mpc_step, states, k_active, false, wind_mean, horizons, st))) return r;
    // the first iteration's particles and wind fields
    BHIP(b, launch_b_fill(b->d_cnt, b->n_cnt, st));
    BHIP(b, launch_b_init(b->prec, b->d_tab, b->d_hdr, b->ns, b->max_count, b->d_u, st));
    BHIP(b, launch_b_normals(b->prec, b->d_tab, b->d_hdr, b->ns, 0, b->G, b->M, b->d_Z, st));
    BHIP(b, batch_wind_fields(b, st));
    unsigned long long* steps = reinterpret_cast<unsigned long long*>(b->d_cnt + b->cnt_steps);
    smc_batch_tuning best = b->tune;
    const int blocks[3] = {64, 128, 256};
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        if (!b->bcount[bk]) continue;
        float best_ms = 0.f;
        bool have = false;
        for (int bi = 0; bi < 3; ++bi)
            for (int gm = 1; gm <= 2; ++gm) {
                const int block = blocks[bi];
                if (b_rollout_resident(b->prec, bk, block) < 1) continue;
                const int grid = rollout_grid(b, bk, block, gm);
                std::vector<float> t;
                for (int q = 0; q < reps; ++q) {
                    BHIP(b, launch_b_fill(b->d_cnt + bk, 1, st));
                    BHIP(b, hipEventRecord(b->ev0, st));
                    BHIP(b, launch_b_rollout(b->prec, bk, b->d_tab, b->d_items + b->bstart[bk],
                                             b->bcount[bk], b->d_cnt + bk, b->d_u, steps, block,
                                             grid, st));
                    BHIP(b, hipEventRecord(b->ev1, st));
                    BHIP(b, hipEventSynchronize(b->ev1));
                    float ms = 0.f;
                    BHIP(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
                    t.push_back(ms);
                }
                std::sort(t.begin(), t.end());
                const float med = t[t.size() / 2];
                if (!have || med < best_ms) {
                    have = true;
                    best_ms = med;
                    best.block[bk] = block;
                    best.grid_mult[bk] = gm;
                }
            }
    }
    BHIP(b, hipStreamSynchronize(st));
    b->tune = best;
    refresh_grids(b);
    drop_graph(b);
    if (out) return smc_batch_get_tuning(b, out);
    return SMC_OK;
}

}  // extern "C"
