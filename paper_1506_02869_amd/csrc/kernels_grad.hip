// Hand-written adjoint of the rollout for the fuel + time part of the cost
// (the differentiable elements used by the gradient-informed move), with
// segment checkpointing, and the Langevin (MALA) proposal / acceptance.
//
// Lanes: one per (particle l, aircraft i, wind sample m), the samples of one
// (l, i) in consecutive lanes (padded to a power of two up to 64, or to
// multiples of 64), so the sum over samples is a wave reduction.  Forward:
// the rollout of the aircraft, storing its state every CK steps and its
// landing step.  Reverse: for each segment from the last, recompute the
// segment's states from its checkpoint into a per-lane tape, then sweep the
// steps backwards, recomputing each step's intermediates and applying the
// chain rule to the adjoint (x, y, z, v, chi, burn) and to the segment's
// controls.  Discrete events (landing) carry no derivative; clamps,
// max(T, 0) and min(t, 1) take the derivative of the active branch.
#include "rollout_math.h"
#include "smc_steps.h"

namespace smc {

constexpr int GR_CK = 25;        // checkpoint interval [steps]
constexpr int GR_IN = 5;         // inner checkpoint interval within a segment [steps]
constexpr int GR_NIN = GR_CK / GR_IN;
static_assert(GR_CK % GR_IN == 0, "inner blocks tile a segment");
constexpr int GR_BLOCK = 256;    // lanes per workgroup
constexpr int GR_MAXSEG = 16;    // horizons up to 400 steps
constexpr int GR_MAXS = 16;      // control segments

struct GradParams {
    RolloutParams rp;
    int Mp;          // lanes per (particle, aircraft) group
    int chunks;      // partial sums per group (Mp / 64 when Mp > 64, else 1)
};

template <typename R>
struct StepFwd {     // intermediates of one step, recomputed in the reverse sweep
    R wx, wy, dwx[3], dwy[3];
    R sg, cg, tphi, icphi, rho, drho_dz, qd, mass, CL, D, vn, T, eta, f;
    R sc, cc;
};

// The wind's grid cell at (x, y, z): clamped coordinates, the interpolation
// weights, the derivative of each grid coordinate (zero along a clamped
// one) and the eight corners c[4 dx + 2 dy + dz] of the lane's sample.
template <typename R>
struct WindCell {
    typename V2<R>::t c[8];
    R tx, ty, tz, jx, jy, jz;
};

// Cell index ((ix ny + iy) nz + iz) and weights of (x, y, z).  With NARROW
// the index arithmetic is 24-bit (grids below 2^24 cells).
template <typename R, bool NARROW = false>
__device__ __forceinline__ int wind_locate(const RolloutParams& p, R x, R y, R z, WindCell<R>& w) {
    const R ux = (x + (R)p.half_wx) * (R)p.inv_hx;
    const R uy = (y + (R)p.half_wy) * (R)p.inv_hy;
    const R uz = z * (R)p.inv_hz;
    const R fx = clampr(ux, (R)0, (R)(p.nx - 1));
    const R fy = clampr(uy, (R)0, (R)(p.ny - 1));
    const R fz = clampr(uz, (R)0, (R)(p.nz - 1));
    w.jx = (ux >= (R)0 && ux <= (R)(p.nx - 1)) ? (R)p.inv_hx : (R)0;
    w.jy = (uy >= (R)0 && uy <= (R)(p.ny - 1)) ? (R)p.inv_hy : (R)0;
    w.jz = (uz >= (R)0 && uz <= (R)(p.nz - 1)) ? (R)p.inv_hz : (R)0;
    const int ix = min((int)fx, p.nx - 2), iy = min((int)fy, p.ny - 2), iz = min((int)fz, p.nz - 2);
    w.tx = fx - (R)ix; w.ty = fy - (R)iy; w.tz = fz - (R)iz;
    if constexpr (NARROW)
        return (int)(__umul24(__umul24((unsigned)ix, (unsigned)p.ny) + (unsigned)iy, (unsigned)p.nz) +
                     (unsigned)iz);
    return (ix * p.ny + iy) * p.nz + iz;
}

// Corners of cell g from the sample-interleaved field Wt[g][m] (row stride
// M); Wm points at the lane's sample, so the lanes of a wave, which hold the
// samples of one (particle, aircraft), read adjacent elements wherever their
// positions share a cell.
template <typename R, bool NARROW = false>
__device__ __forceinline__ void wind_corners(const typename V2<R>::t* Wm, const RolloutParams& p,
                                             int g, WindCell<R>& w) {
    typedef typename V2<R>::t R2;
    const int M = p.M, nzz = p.nz * M, nyz = p.ny * p.nz * M;
    // NARROW: g < 2^24 and M < 2^24, a 24-bit multiply
    const R2* Wg = Wm + (NARROW ? (int64_t)__umul24((unsigned)g, (unsigned)M) : (int64_t)g * M);
    w.c[0] = Wg[0]; w.c[1] = Wg[M]; w.c[2] = Wg[nzz]; w.c[3] = Wg[nzz + M];
    w.c[4] = Wg[nyz]; w.c[5] = Wg[nyz + M]; w.c[6] = Wg[nyz + nzz]; w.c[7] = Wg[nyz + nzz + M];
}

// Trilinear wind value.
template <typename R>
__device__ __forceinline__ void wind_interp(const WindCell<R>& w, R& wx, R& wy) {
    const R tx = w.tx, ty = w.ty, tz = w.tz;
    {
        const R a00 = w.c[0].x + tz * (w.c[1].x - w.c[0].x), a01 = w.c[2].x + tz * (w.c[3].x - w.c[2].x);
        const R a10 = w.c[4].x + tz * (w.c[5].x - w.c[4].x), a11 = w.c[6].x + tz * (w.c[7].x - w.c[6].x);
        const R b0 = a00 + ty * (a01 - a00), b1 = a10 + ty * (a11 - a10);
        wx = b0 + tx * (b1 - b0);
    }
    {
        const R a00 = w.c[0].y + tz * (w.c[1].y - w.c[0].y), a01 = w.c[2].y + tz * (w.c[3].y - w.c[2].y);
        const R a10 = w.c[4].y + tz * (w.c[5].y - w.c[4].y), a11 = w.c[6].y + tz * (w.c[7].y - w.c[6].y);
        const R b0 = a00 + ty * (a01 - a00), b1 = a10 + ty * (a11 - a10);
        wy = b0 + tx * (b1 - b0);
    }
}

// Trilinear wind and its derivative with respect to (x, y, z), by the same
// expressions for the value.
template <typename R>
__device__ __forceinline__ void wind_interp_grad(const WindCell<R>& w, StepFwd<R>& o) {
    const R tx = w.tx, ty = w.ty, tz = w.tz;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        R c[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = comp == 0 ? w.c[q].x : w.c[q].y;
        const R a00 = c[0] + tz * (c[1] - c[0]), a01 = c[2] + tz * (c[3] - c[2]);
        const R a10 = c[4] + tz * (c[5] - c[4]), a11 = c[6] + tz * (c[7] - c[6]);
        const R b0 = a00 + ty * (a01 - a00), b1 = a10 + ty * (a11 - a10);
        const R val = b0 + tx * (b1 - b0);
        const R d_tx = b1 - b0;
        const R d_ty = ((R)1 - tx) * (a01 - a00) + tx * (a11 - a10);
        const R dz0 = ((R)1 - ty) * (c[1] - c[0]) + ty * (c[3] - c[2]);
        const R dz1 = ((R)1 - ty) * (c[5] - c[4]) + ty * (c[7] - c[6]);
        const R d_tz = ((R)1 - tx) * dz0 + tx * dz1;
        R* d = comp == 0 ? o.dwx : o.dwy;
        (comp == 0 ? o.wx : o.wy) = val;
        d[0] = d_tx * w.jx; d[1] = d_ty * w.jy; d[2] = d_tz * w.jz;
    }
}

template <typename R, bool NARROW = false>
__device__ __forceinline__ void wind_and_grad(const typename V2<R>::t* Wm, const RolloutParams& p,
                                              R x, R y, R z, StepFwd<R>& o) {
    WindCell<R> w;
    const int g = wind_locate<R, NARROW>(p, x, y, z, w);
    wind_corners<R, NARROW>(Wm, p, g, w);
    wind_interp_grad<R>(w, o);
}

struct AcConst {
    double Sw, cd0, cd2, cf1, cf2, tmax, dtma, m0;
    bool arr;
};

template <typename R, bool NARROW = false>
__device__ __forceinline__ void wind_value(const typename V2<R>::t* Wm, const RolloutParams& p,
                                           R x, R y, R z, R& wx, R& wy) {
    WindCell<R> w;
    const int g = wind_locate<R, NARROW>(p, x, y, z, w);
    wind_corners<R, NARROW>(Wm, p, g, w);
    wind_interp<R>(w, wx, wy);
}

// Climb, bank, density, drag, thrust and fuel of one step (the rollout's
// arithmetic), shared by the light and the full step.
template <typename R>
__device__ __forceinline__ void step_core(const RolloutParams& p, const AcConst& ac, R z, R v,
                                          R chi, R B, R cd, R vc, R zd, R ir, StepFwd<R>& o) {
    typedef Ops<R> O;
    const R g0 = (R)kG0;
    o.sg = zd * O::rcp(v);
    o.cg = O::sqrt((R)1 - o.sg * o.sg);
    o.tphi = v * cd * (R)(1.0 / kG0);
    o.icphi = O::sqrt((R)1 + o.tphi * o.tphi);
    const R isa_c = (R)(kLapse / kT0), isa_e = (R)(kG0 / (kRair * kLapse) - 1.0);
    const R zc = clampr(z, (R)0, (R)11000);
    const R base = (R)1 - isa_c * zc;
    o.rho = (R)kRho0 * O::pow_pos(base, isa_e);
    o.qd = (R)0.5 * o.rho * v * v;
    o.mass = (R)ac.m0 - B;
    o.CL = O::div(o.mass * g0 * o.icphi, o.qd * (R)ac.Sw);
    o.D = o.qd * (R)ac.Sw * ((R)ac.cd0 + (R)ac.cd2 * o.CL * o.CL);
    o.vn = v + (vc - v) * ir;
    o.T = o.mass * (o.vn - v) * (R)(1.0 / p.dt) + o.D + o.mass * g0 * o.sg;
    o.eta = (R)ac.cf1 * ((R)1 + v * (R)(1.0 / ac.cf2));
    o.f = (R)p.dt * o.eta * m_max(o.T, (R)0);
    O::sincos(chi, &o.sc, &o.cc);
}

// One full step: the intermediates the reverse sweep needs, with the wind's
// spatial derivative and the density's altitude derivative.
template <typename R>
__device__ __forceinline__ void step_forward(const typename V2<R>::t* Wm, const RolloutParams& p,
                                             const AcConst& ac, R x, R y, R z, R v, R chi, R B,
                                             R cd, R vc, R zd, R ir, StepFwd<R>& o) {
    typedef Ops<R> O;
    wind_and_grad<R>(Wm, p, x, y, z, o);
    step_core<R>(p, ac, z, v, chi, B, cd, vc, zd, ir, o);
    const R isa_c = (R)(kLapse / kT0), isa_e = (R)(kG0 / (kRair * kLapse) - 1.0);
    const bool zin = z > (R)0 && z < (R)11000;
    const R zc = clampr(z, (R)0, (R)11000);
    const R base = (R)1 - isa_c * zc;
    o.drho_dz = zin ? -o.rho * isa_e * isa_c * O::rcp(base) : (R)0;
}

// One light step: the next state (x, y, z, v, chi, burn) only.
template <typename R>
__device__ __forceinline__ void step_state(const typename V2<R>::t* Wm, const RolloutParams& p,
                                           const AcConst& ac, R& x, R& y, R& z, R& v, R& chi,
                                           R& B, R cd, R vc, R zd, R ir) {
    StepFwd<R> o;
    wind_value<R>(Wm, p, x, y, z, o.wx, o.wy);
    step_core<R>(p, ac, z, v, chi, B, cd, vc, zd, ir, o);
    x = x + (R)p.dt * (v * o.cc * o.cg + o.wx);
    y = y + (R)p.dt * (v * o.sc * o.cg + o.wy);
    z = z + (R)p.dt * (v * o.sg);
    chi = chi + (R)p.dt * cd;
    v = o.vn;
    B = B + o.f;
}

// time-to-go element at a new state and its derivative w.r.t. (x, y, v)
template <typename R>
__device__ __forceinline__ R time_elem(const RolloutParams& p, const AcConst& ac, R x, R y, R v,
                                       R* dx, R* dy, R* dv) {
    typedef Ops<R> O;
    const R vmin = (R)p.vmin;
    const R vv = m_max(v, vmin);
    const R ivv = O::rcp(vv);
    const R itn = (R)(1.0 / p.time_norm);
    const R r = O::sqrt(x * x + y * y);
    R num, dn_dx, dn_dy;
    if (ac.arr) {
        const R th = O::atan2(y, x);
        const R tha = m_abs(th);
        const R sgn = th < (R)0 ? (R)-1 : (R)1;
        const R ir = r > (R)0 ? O::rcp(r) : (R)0;
        R ratio, dratio;
        if (tha > (R)1e-4) {
            // tha = |atan2(y, x)| in [0, pi]: sin(tha) = |y| / r, cos(tha) = x / r
            const R s = m_abs(y) * ir;
            if (s > (R)1e-6) {
                ratio = tha * O::rcp(s);
                const R c = x * ir;
                dratio = (s - tha * c) * O::rcp(s * s);
            } else {
                ratio = tha * (R)1e6;
                dratio = (R)1e6;
            }
        } else {
            ratio = (R)1 + tha * tha * (R)(1.0 / 6.0);
            dratio = tha * (R)(1.0 / 3.0);
        }
        num = r * ratio;
        const R ir2 = ir * ir;
        // d theta / dx = -y / r^2, d theta / dy = x / r^2
        dn_dx = x * ir * ratio + r * dratio * sgn * (-y * ir2);
        dn_dy = y * ir * ratio + r * dratio * sgn * (x * ir2);
    } else {
        const R gap = (R)ac.dtma - r;
        if (gap > (R)0) {
            num = gap;
            const R ir = r > (R)0 ? O::rcp(r) : (R)0;
            dn_dx = -x * ir;
            dn_dy = -y * ir;
        } else {
            num = (R)0; dn_dx = (R)0; dn_dy = (R)0;
        }
    }
    const R t = num * ivv * itn;
    if (t >= (R)1) { *dx = (R)0; *dy = (R)0; *dv = (R)0; return (R)1; }
    *dx = dn_dx * ivv * itn;
    *dy = dn_dy * ivv * itn;
    *dv = v > vmin ? -t * ivv : (R)0;
    return t;
}

template <typename R>
__device__ __forceinline__ bool landed_at(const RolloutParams& p, R x, R y, R z, R v, R chi) {
    typedef Ops<R> O;
    const R r = O::sqrt(x * x + y * y);
    if (!(r <= (R)p.p_run)) return false;   // outside the runway radius: the angles are not needed
    const R th = O::atan2(y, x);
    const R tha = m_abs(th);
    const R ratio = tha > (R)1e-4 ? tha * O::rcp(m_max(O::sin(tha), (R)1e-6))
                                  : (R)1 + tha * tha * (R)(1.0 / 6.0);
    const R beta = O::atan2(z, r * ratio);
    return r <= (R)p.p_run && beta <= (R)p.p_beta && tha <= (R)p.p_chi &&
           m_abs(wrap_angle<R>(chi - Consts<R>::pi)) <= (R)p.p_chi && v <= (R)p.p_vs;
}

// Physical controls of segment s of a lane's particle.
template <typename R>
__device__ __forceinline__ void seg_controls(const R* ub, int s, const double* lo, const double* sp,
                                             R& cd, R& vc, R& zd) {
    cd = (R)(lo[0] + (double)ub[s * 3 + 0] * sp[0]);
    vc = (R)(lo[1] + (double)ub[s * 3 + 1] * sp[1]);
    zd = (R)(lo[2] + (double)ub[s * 3 + 2] * sp[2]);
}

// Sum of a segment's gradient over the wind samples of each group (a wave
// reduction in FP64), written by the group's first lane.
template <typename R>
__device__ __forceinline__ void flush_segment(const GradParams& gp, int s, const R* gc,
                                              const double* sp, int m, int64_t grp, int64_t ngrp,
                                              int l, int i, double* __restrict__ out) {
    const RolloutParams& p = gp.rp;
    const int width = gp.Mp < 64 ? gp.Mp : 64;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double vsum = (double)gc[c] * sp[c];   // d u_phys / d u_norm
        for (int off = width >> 1; off > 0; off >>= 1) vsum += __shfl_xor(vsum, off, width);
        if ((m % width) == 0 && grp < ngrp) {
            const int chunk = m / width;
            out[(((int64_t)chunk * p.P + l) * p.N + i) * p.S * 3 + s * 3 + c] = vsum;
        }
    }
}

// One step of the reverse sweep at step k: recompute the step's
// intermediates from its start state, add the time element's derivative at
// the new state (unless the step lands) and the fuel's, and carry the
// adjoint (ax, ay, az, av, achi, aB) of the state back over the step, adding
// the step's share of the segment's control gradient to gc.
template <typename R>
__device__ __forceinline__ void grad_reverse_step(const typename V2<R>::t* Wm,
                                                  const RolloutParams& p, const AcConst& ac, int k,
                                                  int k_land, R x0, R y0, R z0, R v0, R chi0,
                                                  R B0, R cd, R vc, R zd, R ir, R kt, R& ax,
                                                  R& ay, R& az, R& av, R& achi, R& aB, R* gc) {
    const R dt = (R)p.dt;
    StepFwd<R> o;
    step_forward<R>(Wm, p, ac, x0, y0, z0, v0, chi0, B0, cd, vc, zd, ir, o);
    const R xn = x0 + dt * (v0 * o.cc * o.cg + o.wx);
    const R yn = y0 + dt * (v0 * o.sc * o.cg + o.wy);
    // time element at the new state (counted unless this step lands)
    if (k < k_land) {
        R dx, dy, dv;
        time_elem<R>(p, ac, xn, yn, o.vn, &dx, &dy, &dv);
        ax += kt * dx; ay += kt * dy; av += kt * dv;
    }
    // fuel f = dt eta max(T, 0)
    R df_dv = 0, df_dvc = 0, df_dzd = 0, df_dcd = 0, df_dz = 0, df_dm = 0;
    if (o.T > (R)0) {
        const R g0 = (R)kG0;
        const R A0 = o.qd * (R)ac.Sw;
        const R dD_dA0 = (R)ac.cd0 - (R)ac.cd2 * o.CL * o.CL;
        const R dD_dK = (R)2 * (R)ac.cd2 * o.CL;
        const R inv_dt = (R)(1.0 / p.dt);
        const R dT_dv = -o.mass * ir * inv_dt + dD_dA0 * ((R)2 * A0 * Ops<R>::rcp(v0)) +
                        dD_dK * o.mass * g0 * (o.tphi * Ops<R>::rcp(o.icphi)) * (cd * (R)(1.0 / kG0)) -
                        o.mass * g0 * o.sg * Ops<R>::rcp(v0);
        const R dT_dvc = o.mass * ir * inv_dt;
        const R dT_dzd = o.mass * g0 * Ops<R>::rcp(v0);
        const R dT_dcd = dD_dK * o.mass * g0 * (o.tphi * Ops<R>::rcp(o.icphi)) * (v0 * (R)(1.0 / kG0));
        const R dT_dz = dD_dA0 * (A0 * Ops<R>::rcp(o.rho)) * o.drho_dz;
        const R dT_dm = (o.vn - v0) * inv_dt + dD_dK * g0 * o.icphi + g0 * o.sg;
        const R dt_eta = dt * o.eta;
        df_dv = dt * (R)(ac.cf1 / ac.cf2) * o.T + dt_eta * dT_dv;
        df_dvc = dt_eta * dT_dvc;
        df_dzd = dt_eta * dT_dzd;
        df_dcd = dt_eta * dT_dcd;
        df_dz = dt_eta * dT_dz;
        df_dm = dt_eta * dT_dm;
    }
    const R icg = Ops<R>::rcp(o.cg);
    // adjoints of the step's inputs
    const R nx_ = ax * ((R)1 + dt * o.dwx[0]) + ay * dt * o.dwy[0];
    const R ny_ = ax * dt * o.dwx[1] + ay * ((R)1 + dt * o.dwy[1]);
    const R nz_ = az + ax * dt * o.dwx[2] + ay * dt * o.dwy[2] + aB * df_dz;
    const R nchi = achi + ax * dt * (-v0 * o.sc * o.cg) + ay * dt * (v0 * o.cc * o.cg);
    const R nv = av * ((R)1 - ir) + ax * dt * o.cc * icg + ay * dt * o.sc * icg + aB * df_dv;
    const R nB = aB - aB * df_dm;
    gc[0] += achi * dt + aB * df_dcd;
    gc[1] += av * ir + aB * df_dvc;
    gc[2] += ax * dt * o.cc * (-o.sg * icg) + ay * dt * o.sc * (-o.sg * icg) + az * dt +
             aB * df_dzd;
    ax = nx_; ay = ny_; az = nz_; achi = nchi; av = nv; aB = nB;
}

// Segment checkpoints of a lane.  NSEG bounds the segment count of the
// horizon, (H + GR_CK - 1) / GR_CK.  With REG, every access names its slot
// at compile time (unrolled selects over the slots; the segment index j is
// the same for every lane of a wave), so the array stays in registers
// instead of scratch memory: worth its 6 NSEG registers for short horizons
// in FP32.  Otherwise the slot is indexed directly (scratch memory).
template <typename R, int NSEG, bool REG>
__device__ __forceinline__ void ck_put(R (&ck)[NSEG][6], int j, R x, R y, R z, R v, R chi, R B) {
    if constexpr (!REG) {
        ck[j][0] = x; ck[j][1] = y; ck[j][2] = z; ck[j][3] = v; ck[j][4] = chi; ck[j][5] = B;
        return;
    }
#pragma unroll
    for (int q = 0; q < NSEG; ++q) {   // selects, not branches: no store is merged into ck[j]
        const bool h = q == j;
        ck[q][0] = h ? x : ck[q][0]; ck[q][1] = h ? y : ck[q][1]; ck[q][2] = h ? z : ck[q][2];
        ck[q][3] = h ? v : ck[q][3]; ck[q][4] = h ? chi : ck[q][4]; ck[q][5] = h ? B : ck[q][5];
    }
}

template <typename R, int NSEG, bool REG>
__device__ __forceinline__ void ck_get(const R (&ck)[NSEG][6], int j, R& x, R& y, R& z, R& v,
                                       R& chi, R& B) {
    if constexpr (!REG) {
        x = ck[j][0]; y = ck[j][1]; z = ck[j][2]; v = ck[j][3]; chi = ck[j][4]; B = ck[j][5];
        return;
    }
    x = ck[0][0]; y = ck[0][1]; z = ck[0][2]; v = ck[0][3]; chi = ck[0][4]; B = ck[0][5];
#pragma unroll
    for (int q = 1; q < NSEG; ++q) {
        const bool h = q == j;
        x = h ? ck[q][0] : x; y = h ? ck[q][1] : y; z = h ? ck[q][2] : z;
        v = h ? ck[q][3] : v; chi = h ? ck[q][4] : chi; B = h ? ck[q][5] : B;
    }
}

// Adjoint of the fuel + time cost of one (particle, aircraft, wind sample)
// per lane.  The step loops run over absolute steps, the same for every lane
// of a wave (a lane takes part in the steps k0 <= k <= its last step), so the
// checkpoints sit at multiples of GR_CK and the tape of a segment's states is
// indexed by a wave-uniform step: it stays in registers.  A control
// segment's gradient is summed over its steps in three registers and reduced
// over the wind samples when the reverse sweep leaves the segment.
template <typename R, int NSEG, bool REG>
__global__ void __launch_bounds__(GR_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_rollout_grad(const GradParams gp, const R* __restrict__ u,
                                                      const R* __restrict__ W,
                                                      const double* __restrict__ states,
                                                      const int32_t* __restrict__ k_active,
                                                      const double* __restrict__ acpar,
                                                      const double* __restrict__ targets,
                                                      const int8_t* __restrict__ kind,
                                                      double* __restrict__ out) {
    typedef typename V2<R>::t R2;
    const RolloutParams& p = gp.rp;
    const int N = p.N, S = p.S, H = p.H, M = p.M, Mp = gp.Mp;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = (int)(t % Mp);
    const int64_t grp = t / Mp;                 // (l, i)
    const int64_t ngrp = (int64_t)p.P * N;
    const bool valid = grp < ngrp && m < M;
    const int l = grp < ngrp ? (int)(grp / N) : 0;
    const int i = grp < ngrp ? (int)(grp % N) : 0;
    const int mm = m < M ? m : 0;

    AcConst ac;
    ac.Sw = acpar[i * 9 + 0]; ac.cd0 = acpar[i * 9 + 1]; ac.cd2 = acpar[i * 9 + 2];
    ac.cf1 = acpar[i * 9 + 3]; ac.cf2 = acpar[i * 9 + 4]; ac.tmax = acpar[i * 9 + 5];
    ac.dtma = targets[i * 4 + 3]; ac.m0 = states[i * 6 + 5];
    ac.arr = kind[i] == 0;
    const int k0 = k_active[i];
    const bool active = valid && k0 >= 0 && k0 < H;
    const R2* Wm = (const R2*)W + mm;           // sample-interleaved field Wt[g][m]
    const R* ub = u + ((int64_t)l * N + i) * S * 3;
    const double lo[3] = {p.ctrl_lo[0], p.ctrl_lo[1], p.ctrl_lo[2]};
    const double sp[3] = {p.ctrl_span[0], p.ctrl_span[1], p.ctrl_span[2]};

    // forward sweep: checkpoints at every GR_CK-th step and the landing step
    R ck[NSEG][6];
    R x = (R)states[i * 6 + 0], y = (R)states[i * 6 + 1], z = (R)states[i * 6 + 2];
    R v = (R)states[i * 6 + 3], chi = (R)states[i * 6 + 4], B = (R)0;
    int k_land = H;   // step whose new state lands (H: none)
    bool flying = active;
    int s_cur = -1, k_end = 0;
    R cd = 0, vc = 0, zd = 0;
    for (int k = 0; k < H; ++k) {
        if ((k % GR_CK) == 0) ck_put<R, NSEG, REG>(ck, k / GR_CK, x, y, z, v, chi, B);
        const int s = (k * S) / H;
        if (s != s_cur) {   // wave-uniform
            s_cur = s;
            k_end = ((s + 1) * H + S - 1) / S;
            seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
        }
        if (flying && k >= k0) {
            step_state<R>(Wm, p, ac, x, y, z, v, chi, B, cd, vc, zd, Ops<R>::rcp((R)(k_end - k)));
            if (ac.arr && landed_at<R>(p, x, y, z, v, chi)) { k_land = k; flying = false; }
        }
    }

    // reverse sweep, segment by segment from the last.  Two levels of
    // recomputation keep the tape in registers: a pass over the segment
    // from its checkpoint stores the state every GR_IN steps in LDS (this
    // lane's column), then each block of GR_IN steps, from the last, is
    // recomputed into a tape indexed at compile time and swept backwards.
    __shared__ R ick[GR_NIN][6][GR_BLOCK];
    const int tl = threadIdx.x;
    const int k_last = min(k_land, H - 1);
    const int nsteps = H - k0;
    const double wf = ac.arr ? p.w[2] : p.w[4];
    const double denom = p.dt * (double)nsteps * ac.tmax * (ac.cf1 * (1.0 + p.vmax / ac.cf2));
    const R kf = (R)((1.0 - p.w[7] - p.w[8]) * wf / denom);
    const R kt = (R)(p.w[7] / (double)nsteps);
    R ax = 0, ay = 0, az = 0, av = 0, achi = 0, aB = kf;
    R gc[3] = {(R)0, (R)0, (R)0};
    const int nseg = (H + GR_CK - 1) / GR_CK;
    int s_grad = S - 1;      // segment whose gradient gc holds
    s_cur = -1;
    for (int j = nseg - 1; j >= 0; --j) {
        const int ka = j * GR_CK;
        const int kb = min(H, ka + GR_CK) - 1;
        {   // inner checkpoints: the state at the start of each block
            R x1, y1, z1, v1, chi1, B1;
            ck_get<R, NSEG, REG>(ck, j, x1, y1, z1, v1, chi1, B1);
            for (int k = ka; k <= kb; ++k) {
                if (((k - ka) % GR_IN) == 0) {
                    R* c = &ick[(k - ka) / GR_IN][0][tl];
                    c[0] = x1; c[GR_BLOCK] = y1; c[2 * GR_BLOCK] = z1; c[3 * GR_BLOCK] = v1;
                    c[4 * GR_BLOCK] = chi1; c[5 * GR_BLOCK] = B1;
                }
                if (k == kb) break;
                const int s = (k * S) / H;
                if (s != s_cur) {
                    s_cur = s;
                    k_end = ((s + 1) * H + S - 1) / S;
                    seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
                }
                if (active && k >= k0 && k <= k_last)
                    step_state<R>(Wm, p, ac, x1, y1, z1, v1, chi1, B1, cd, vc, zd,
                                  Ops<R>::rcp((R)(k_end - k)));
            }
        }
        for (int b = (kb - ka) / GR_IN; b >= 0; --b) {
            const int kc = ka + b * GR_IN;           // first step of the block
            const int kd = min(kb, kc + GR_IN - 1);  // last step of the block
            R tx_[GR_IN], ty_[GR_IN], tz_[GR_IN], tv_[GR_IN], tchi_[GR_IN], tB_[GR_IN];
            {   // the block's step-start states (the tape)
                const R* c = &ick[b][0][tl];
                R x1 = c[0], y1 = c[GR_BLOCK], z1 = c[2 * GR_BLOCK], v1 = c[3 * GR_BLOCK],
                  chi1 = c[4 * GR_BLOCK], B1 = c[5 * GR_BLOCK];
#pragma unroll
                for (int q = 0; q < GR_IN; ++q) {
                    const int k = kc + q;
                    tx_[q] = x1; ty_[q] = y1; tz_[q] = z1; tv_[q] = v1; tchi_[q] = chi1; tB_[q] = B1;
                    if (k >= kd) continue;           // uniform
                    const int s = (k * S) / H;
                    if (s != s_cur) {
                        s_cur = s;
                        k_end = ((s + 1) * H + S - 1) / S;
                        seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
                    }
                    if (active && k >= k0 && k <= k_last)
                        step_state<R>(Wm, p, ac, x1, y1, z1, v1, chi1, B1, cd, vc, zd,
                                      Ops<R>::rcp((R)(k_end - k)));
                }
            }
#pragma unroll
            for (int q = GR_IN - 1; q >= 0; --q) {
                const int k = kc + q;
                if (k > kd) continue;                // uniform
                const int s = (k * S) / H;
                if (s != s_grad) {   // wave-uniform: the reverse sweep leaves segment s_grad
                    flush_segment<R>(gp, s_grad, gc, sp, m, grp, ngrp, l, i, out);
                    gc[0] = gc[1] = gc[2] = (R)0;
                    s_grad = s;
                }
                if (s != s_cur) {
                    s_cur = s;
                    k_end = ((s + 1) * H + S - 1) / S;
                    seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
                }
                if (!(active && k >= k0 && k <= k_last)) continue;
                const R x0 = tx_[q], y0 = ty_[q], z0 = tz_[q], v0 = tv_[q], chi0 = tchi_[q],
                        B0 = tB_[q];
                grad_reverse_step<R>(Wm, p, ac, k, k_land, x0, y0, z0, v0, chi0, B0, cd, vc, zd,
                                     Ops<R>::rcp((R)(k_end - k)), kt, ax, ay, az, av, achi, aB,
                                     gc);
            }
        }
    }
    flush_segment<R>(gp, s_grad, gc, sp, m, grp, ngrp, l, i, out);
}

// ---- Adjoint with the sample-independent chain hoisted ----------------------------
//
// Of an aircraft's state only (x, y) depend on the wind sample: heading,
// speed, altitude and burn follow from the controls alone (eq. hor), and a
// sample's landing only ends that sample's steps.  So for 65 ... 128 samples
// a workgroup of two waves takes one (particle, aircraft), for 33 ... 64 one
// wave, for 17 ... 32 each half-wave: the group computes that chain and
// every step's reverse coefficients once, into an LDS record per step, and
// each lane then carries only its sample's (x, y) forward and the adjoint
// backward.  The adjoint of (z, v, chi, burn) stays per lane (it depends on
// the sample through the wind's altitude derivative and the landing step);
// its update is linear with the record's coefficients.  The step arithmetic
// is k_rollout_grad's (up to the order of some products).
//
// Per lane: a forward pass over (x, y) keeps a checkpoint every GS_CK steps
// and finds the landing step; then, block by block from the last, a pass
// from the block's checkpoint keeps (x, y) and the wind's spatial derivative
// at every step in registers, and the backward sweep over the block reads
// no field.  The field is the bound (every load comes from L2), so a lane
// fetches its cell's eight corners only when it enters another cell, which
// at these grid spacings holds several consecutive steps.
//
// Record of step k (reals), in its final form:
//   z_k, v cos(chi) cos(gamma), chi_k, v_{k+1}, 1 / (steps to the segment's
//   end), dt cos(chi) / cos(gamma), dt sin(chi) / cos(gamma), -sin(gamma),
//   d burn / d (z, v, mass, chi rate, commanded v, climb rate),
//   v sin(chi) cos(gamma)
// (record H holds the final z and chi).  While it is built, slots 0-2 hold
// z, v, chi (sequential pass), 3-7 the burn's step inputs (step-parallel
// pass) and 8-10 burn, lift coefficient and thrust (sequential burn pass);
// each pass writes only its own steps' records.
constexpr int GS_CK = 8;      // (x, y) checkpoint interval [steps]
constexpr int GS_REC = 16;    // reals per step record
constexpr int GS_MAXH = 160;  // horizons of the hoisted form (20 checkpoints)
constexpr int GS_MIN_M = 17;  // fewest samples for the hoisted form (idle lanes below)
enum {
    RS_Z = 0, RS_A, RS_CHI, RS_VN, RS_IR, RS_C1, RS_C2, RS_C3,
    RS_DFZ, RS_DFV, RS_DFM, RS_DFCD, RS_DFVC, RS_DFZD, RS_B
};

template <typename R, int NSEG>
__device__ __forceinline__ void ck2_put(R (&cx)[NSEG], R (&cy)[NSEG], int j, R x, R y) {
#pragma unroll
    for (int q = 0; q < NSEG; ++q) {   // selects: every slot named at compile time
        const bool h = q == j;
        cx[q] = h ? x : cx[q];
        cy[q] = h ? y : cy[q];
    }
}

template <typename R, int NSEG>
__device__ __forceinline__ void ck2_get(const R (&cx)[NSEG], const R (&cy)[NSEG], int j, R& x,
                                        R& y) {
    x = cx[0]; y = cy[0];
#pragma unroll
    for (int q = 1; q < NSEG; ++q) {
        const bool h = q == j;
        x = h ? cx[q] : x;
        y = h ? cy[q] : y;
    }
}

// (FP32: held to 168 registers, three waves per SIMD; one value spills,
// outside the step loops)
// MP lanes per (particle, aircraft): 128 (a workgroup of two waves, whose
// 64-lane partial sums go to the chunk buffer), 64 (one per wave) or 32 (two
// per wave, each half with its own records); gp.Mp == MP.
template <typename R, int MP>
__global__ void __launch_bounds__(MP > 64 ? MP : 64)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 1)))
k_rollout_grad_split(const GradParams gp, const R* __restrict__ u, const R* __restrict__ W,
                     const double* __restrict__ states, const int32_t* __restrict__ k_active,
                     const double* __restrict__ acpar, const double* __restrict__ targets,
                     const int8_t* __restrict__ kind, double* __restrict__ out) {
    typedef typename V2<R>::t R2;
    typedef Ops<R> O;
    static_assert(MP == 128 || MP == 64 || MP == 32, "two waves, one or half a wave per group");
    constexpr int NSEG = (GS_MAXH + GS_CK - 1) / GS_CK;
    constexpr int GPW = MP >= 64 ? 1 : 64 / MP;   // groups per workgroup
    extern __shared__ __align__(16) unsigned char gs_smem[];
    const RolloutParams& p = gp.rp;
    const int N = p.N, S = p.S, H = p.H, M = p.M;
    const int lane = threadIdx.x;
    // one group per wave: the group and everything read from its index stay
    // wave-uniform (scalar registers, scalar loads)
    const int slot = MP >= 64 ? 0 : lane / MP;    // the group's place in the wave
    const int m = MP >= 64 ? lane : lane % MP;    // wind sample
    const int64_t ngrp = (int64_t)p.P * N;
    const int64_t grp = (int64_t)blockIdx.x * GPW + slot;   // (l, i)
    const bool gin = grp < ngrp;
    const int l = gin ? (int)(grp / N) : 0, i = gin ? (int)(grp % N) : 0;
    const bool valid = gin && m < M;
    R* rec = (R*)gs_smem + slot * (H + 1) * GS_REC;   // [H + 1][GS_REC] per group

    AcConst ac;
    ac.Sw = acpar[i * 9 + 0]; ac.cd0 = acpar[i * 9 + 1]; ac.cd2 = acpar[i * 9 + 2];
    ac.cf1 = acpar[i * 9 + 3]; ac.cf2 = acpar[i * 9 + 4]; ac.tmax = acpar[i * 9 + 5];
    ac.dtma = targets[i * 4 + 3]; ac.m0 = states[i * 6 + 5];
    ac.arr = kind[i] == 0;
    const int k0 = k_active[i];
    const bool gact = gin && k0 >= 0 && k0 < H;   // the same for the whole group
    const bool active = valid && gact;
    const R2* Wm = (const R2*)W + (valid ? m : 0);   // sample-interleaved Wt[g][m]
    const R* ub = u + ((int64_t)l * N + i) * S * 3;
    const double lo[3] = {p.ctrl_lo[0], p.ctrl_lo[1], p.ctrl_lo[2]};
    const double sp[3] = {p.ctrl_span[0], p.ctrl_span[1], p.ctrl_span[2]};
    const R dt = (R)p.dt;

    // (1) sequential: z, v, chi at every step from k0 (a group's first lane
    // writes; the barriers sit outside the per-group branches)
    if (gact) {
        {
            R z = (R)states[i * 6 + 2], v = (R)states[i * 6 + 3], chi = (R)states[i * 6 + 4];
            int s_cur = -1, k_end = 0;
            R cd = 0, vc = 0, zd = 0;
            for (int k = k0; k < H; ++k) {
                const int s = (k * S) / H;
                if (s != s_cur) {
                    s_cur = s;
                    k_end = ((s + 1) * H + S - 1) / S;
                    seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
                }
                if (m == 0) {
                    R* r = rec + k * GS_REC;
                    r[0] = z; r[1] = v; r[2] = chi;
                }
                const R sg = zd * O::rcp(v);   // as step_core / step_state
                z = z + dt * (v * sg);
                chi = chi + dt * cd;
                v = v + (vc - v) * O::rcp((R)(k_end - k));
            }
            if (m == 0) {
                R* r = rec + H * GS_REC;
                r[0] = z; r[1] = v; r[2] = chi;
            }
        }
    }
    __syncthreads();
    // (2) step-parallel: the burn's inputs that do not depend on the mass
    if (gact) {
        for (int k = k0 + m; k < H; k += MP) {
            R* r = rec + k * GS_REC;
            const R z = r[0], v = r[1], chi = r[2];
            const int s = (k * S) / H;
            const int k_end = ((s + 1) * H + S - 1) / S;
            R cd, vc, zd;
            seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
            StepFwd<R> o;
            step_core<R>(p, ac, z, v, chi, (R)0, cd, vc, zd, O::rcp((R)(k_end - k)), o);
            r[3] = o.icphi; r[4] = o.qd * (R)ac.Sw; r[5] = o.vn - v; r[6] = o.sg;
            r[7] = (R)p.dt * o.eta;
        }
    }
    __syncthreads();
    // (3) sequential: the burn, by step_core's expressions
    if (gact) {
        {
            const R g0 = (R)kG0, inv_dt = (R)(1.0 / p.dt);
            R B = 0;
#pragma unroll 4
            for (int k = k0; k < H; ++k) {   // (unrolled: the record reads run ahead of the chain)
                R* r = rec + k * GS_REC;
                const R icphi = r[3], A0 = r[4], dv = r[5], sg = r[6], dteta = r[7];
                const R mass = (R)ac.m0 - B;
                const R CL = O::div(mass * g0 * icphi, A0);
                const R D = A0 * ((R)ac.cd0 + (R)ac.cd2 * CL * CL);
                const R T = mass * dv * inv_dt + D + mass * g0 * sg;
                if (m == 0) { r[8] = B; r[9] = CL; r[10] = T; }
                B = B + dteta * m_max(T, (R)0);
            }
        }
    }
    __syncthreads();
    // (4) step-parallel: the record (reverse coefficients)
    if (gact) {
        for (int k = k0 + m; k < H; k += MP) {
            R* r = rec + k * GS_REC;
            const R z = r[0], v = r[1], chi = r[2], B = r[8], CL = r[9], T = r[10];
            const int s = (k * S) / H;
            const int k_end = ((s + 1) * H + S - 1) / S;
            R cd, vc, zd;
            seg_controls<R>(ub, s, lo, sp, cd, vc, zd);
            const R ir = O::rcp((R)(k_end - k));
            StepFwd<R> o;
            step_core<R>(p, ac, z, v, chi, B, cd, vc, zd, ir, o);
            o.CL = CL; o.T = T;
            const R isa_c = (R)(kLapse / kT0), isa_e = (R)(kG0 / (kRair * kLapse) - 1.0);
            const bool zin = z > (R)0 && z < (R)11000;
            const R base = (R)1 - isa_c * clampr(z, (R)0, (R)11000);
            const R drho_dz = zin ? -o.rho * isa_e * isa_c * O::rcp(base) : (R)0;
            R df_dv = 0, df_dvc = 0, df_dzd = 0, df_dcd = 0, df_dz = 0, df_dm = 0;
            if (o.T > (R)0) {   // as grad_reverse_step
                const R g0 = (R)kG0;
                const R A0 = o.qd * (R)ac.Sw;
                const R dD_dA0 = (R)ac.cd0 - (R)ac.cd2 * o.CL * o.CL;
                const R dD_dK = (R)2 * (R)ac.cd2 * o.CL;
                const R inv_dt = (R)(1.0 / p.dt);
                const R dT_dv = -o.mass * ir * inv_dt + dD_dA0 * ((R)2 * A0 * O::rcp(v)) +
                                dD_dK * o.mass * g0 * (o.tphi * O::rcp(o.icphi)) * (cd * (R)(1.0 / kG0)) -
                                o.mass * g0 * o.sg * O::rcp(v);
                const R dT_dvc = o.mass * ir * inv_dt;
                const R dT_dzd = o.mass * g0 * O::rcp(v);
                const R dT_dcd = dD_dK * o.mass * g0 * (o.tphi * O::rcp(o.icphi)) * (v * (R)(1.0 / kG0));
                const R dT_dz = dD_dA0 * (A0 * O::rcp(o.rho)) * drho_dz;
                const R dT_dm = (o.vn - v) * inv_dt + dD_dK * g0 * o.icphi + g0 * o.sg;
                const R dt_eta = dt * o.eta;
                df_dv = dt * (R)(ac.cf1 / ac.cf2) * o.T + dt_eta * dT_dv;
                df_dvc = dt_eta * dT_dvc;
                df_dzd = dt_eta * dT_dzd;
                df_dcd = dt_eta * dT_dcd;
                df_dz = dt_eta * dT_dz;
                df_dm = dt_eta * dT_dm;
            }
            const R icg = O::rcp(o.cg);
            const R a = v * o.cc * o.cg, b = v * o.sc * o.cg;
            r[RS_Z] = z; r[RS_A] = a; r[RS_CHI] = chi; r[RS_VN] = o.vn; r[RS_IR] = ir;
            r[RS_C1] = dt * o.cc * icg; r[RS_C2] = dt * o.sc * icg; r[RS_C3] = -o.sg;
            r[RS_DFZ] = df_dz; r[RS_DFV] = df_dv; r[RS_DFM] = df_dm; r[RS_DFCD] = df_dcd;
            r[RS_DFVC] = df_dvc; r[RS_DFZD] = df_dzd; r[RS_B] = b;
        }
    }
    __syncthreads();

    // forward over the sample's (x, y): checkpoints every GS_CK steps, landing step
    R ckx[NSEG], cky[NSEG];
#pragma unroll
    for (int q = 0; q < NSEG; ++q) { ckx[q] = (R)0; cky[q] = (R)0; }
    R x = (R)states[i * 6 + 0], y = (R)states[i * 6 + 1];
    int k_land = H;
    bool flying = active;
    // the next step's record is read one step ahead (records before k0 are
    // read but not used; record H exists)
    R pz = rec[RS_Z], pa = rec[RS_A], pb = rec[RS_B];
    // a lane fetches its cell's corners only when it enters another cell
    // (a cell spans several steps); lanes that stay fetch nothing
    WindCell<R> wc;
    int gprev = -1;
    for (int k = 0; k < H; ++k) {
        const R rz = pz, ra = pa, rb = pb;
        {
            const R* rn = rec + (k + 1) * GS_REC;
            pz = rn[RS_Z]; pa = rn[RS_A]; pb = rn[RS_B];
        }
        if ((k % GS_CK) == 0) ck2_put<R, NSEG>(ckx, cky, k / GS_CK, x, y);
        if (flying && k >= k0) {
            const R* r = rec + k * GS_REC;
            const int g = wind_locate<R, true>(p, x, y, rz, wc);
            if (g != gprev) {
                wind_corners<R, true>(Wm, p, g, wc);
                gprev = g;
            }
            R wx, wy;
            wind_interp<R>(wc, wx, wy);
            x = x + dt * (ra + wx);
            y = y + dt * (rb + wy);
            if (ac.arr && landed_at<R>(p, x, y, pz, r[RS_VN], r[GS_REC + RS_CHI])) {
                k_land = k;
                flying = false;
            }
        }
    }

    // reverse, block by block of GS_CK steps from the last: the block's (x, y)
    // tape recomputed from its checkpoint, indexed at compile time
    const int k_last = min(k_land, H - 1);
    const int nsteps = H - k0;
    const double wf = ac.arr ? p.w[2] : p.w[4];
    const double denom = p.dt * (double)nsteps * ac.tmax * (ac.cf1 * (1.0 + p.vmax / ac.cf2));
    const R kf = (R)((1.0 - p.w[7] - p.w[8]) * wf / denom);
    const R kt = (R)(p.w[7] / (double)nsteps);
    R ax = 0, ay = 0, az = 0, av = 0, achi = 0, aB = kf;
    R gc[3] = {(R)0, (R)0, (R)0};
    int s_grad = S - 1;
    const int nblk = (H + GS_CK - 1) / GS_CK;
    for (int j = nblk - 1; j >= 0; --j) {
        const int kc = j * GS_CK;
        const int kd = min(H, kc + GS_CK) - 1;
        // the block's tape, indexed at compile time: (x, y) before each step
        // and after the last, and the wind's spatial derivative (times dt)
        // at each step, so the reverse sweep reads no field
        R tx_[GS_CK + 1], ty_[GS_CK + 1], tw_[GS_CK][6];
        {
            R x1, y1;
            ck2_get<R, NSEG>(ckx, cky, j, x1, y1);
            tx_[0] = x1; ty_[0] = y1;
            WindCell<R> wt;     // this pass's corner cache (not kept over the sweep below)
            int gt = -1;
#pragma unroll
            for (int q = 0; q < GS_CK; ++q) {
                const int k = kc + q;
#pragma unroll
                for (int c = 0; c < 6; ++c) tw_[q][c] = (R)0;
                tx_[q + 1] = x1; ty_[q + 1] = y1;
                if (k > kd) continue;   // uniform
                const R* r = rec + k * GS_REC;
                const R rz = r[RS_Z], ra = r[RS_A], rb = r[RS_B];   // ahead of the lane test
                if (active && k >= k0 && k <= k_last) {
                    StepFwd<R> o;
                    const int g = wind_locate<R, true>(p, x1, y1, rz, wt);
                    if (g != gt) {
                        wind_corners<R, true>(Wm, p, g, wt);
                        gt = g;
                    }
                    wind_interp_grad<R>(wt, o);
                    x1 = x1 + dt * (ra + o.wx);
                    y1 = y1 + dt * (rb + o.wy);
                    tx_[q + 1] = x1; ty_[q + 1] = y1;
                    tw_[q][0] = dt * o.dwx[0]; tw_[q][1] = dt * o.dwx[1]; tw_[q][2] = dt * o.dwx[2];
                    tw_[q][3] = dt * o.dwy[0]; tw_[q][4] = dt * o.dwy[1]; tw_[q][5] = dt * o.dwy[2];
                }
            }
        }
#pragma unroll
        for (int q = GS_CK - 1; q >= 0; --q) {
            const int k = kc + q;
            if (k > kd) continue;   // uniform
            const int s = (k * S) / H;
            if (s != s_grad) {      // uniform: the sweep leaves control segment s_grad
                flush_segment<R>(gp, s_grad, gc, sp, m, grp, ngrp, l, i, out);
                gc[0] = gc[1] = gc[2] = (R)0;
                s_grad = s;
            }
            if (!(active && k >= k0 && k <= k_last)) continue;
            const R* r = rec + k * GS_REC;
            const R xn = tx_[q + 1], yn = ty_[q + 1];
            if (k < k_land) {   // time element at the new state, unless this step lands
                R dx, dy, dv;
                time_elem<R>(p, ac, xn, yn, r[RS_VN], &dx, &dy, &dv);
                ax += kt * dx; ay += kt * dy; av += kt * dv;
            }
            const R ir = r[RS_IR];
            const R sx = r[RS_C1] * ax + r[RS_C2] * ay;   // dt (cos chi ax + sin chi ay) / cos gamma
            const R nx_ = ax * ((R)1 + tw_[q][0]) + ay * tw_[q][3];
            const R ny_ = ax * tw_[q][1] + ay * ((R)1 + tw_[q][4]);
            const R nz_ = az + ax * tw_[q][2] + ay * tw_[q][5] + aB * r[RS_DFZ];
            const R nchi = achi + dt * (ay * r[RS_A] - ax * r[RS_B]);
            const R nv = av * ((R)1 - ir) + sx + aB * r[RS_DFV];
            const R nB = aB - aB * r[RS_DFM];
            gc[0] += achi * dt + aB * r[RS_DFCD];
            gc[1] += av * ir + aB * r[RS_DFVC];
            gc[2] += r[RS_C3] * sx + az * dt + aB * r[RS_DFZD];
            ax = nx_; ay = ny_; az = nz_; achi = nchi; av = nv; aB = nB;
        }
    }
    flush_segment<R>(gp, s_grad, gc, sp, m, grp, ngrp, l, i, out);
}

// W[m][g] -> Wt[m / B][g][m % B] (pairs of reals), one 32 x 32 tile per
// workgroup through LDS so that both the reads and the writes are coalesced.
template <typename R>
__global__ void __launch_bounds__(256) k_wind_transpose(const typename V2<R>::t* __restrict__ W,
                                                        int M, int G, int B,
                                                        typename V2<R>::t* __restrict__ Wt) {
    typedef typename V2<R>::t R2;
    __shared__ R2 tile[32][33];
    const int g0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int m = m0 + r, g = g0 + tx;
        if (m < M && g < G) tile[r][tx] = W[(int64_t)m * G + g];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int g = g0 + r, m = m0 + tx;
        if (m < M && g < G) Wt[((int64_t)(m / B) * G + g) * B + m % B] = tile[tx][r];
    }
}

// Sum of chunk partials (only when more than 64 samples).
__global__ void k_grad_chunks(int64_t n, int chunks, const double* __restrict__ part,
                              double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + e];
    out[e] = s;
}

int grad_lanes_per_group(int M) {
    if (M > 64) return ((M + 63) / 64) * 64;
    int mp = 1;
    while (mp < M) mp <<= 1;
    return mp;
}

size_t grad_partial_elems(int P, int N, int S, int M) {
    const int mp = grad_lanes_per_group(M);
    const int chunks = mp > 64 ? mp / 64 : 1;
    return (size_t)chunks * P * N * S * 3;
}

bool grad_supported(int H, int S) {
    return S <= GR_MAXS && (H + GR_CK - 1) / GR_CK <= GR_MAXSEG;
}

hipError_t launch_wind_transpose(int prec, const void* W, int M, int G, int B, void* Wt,
                                 hipStream_t st) {
    if (M <= 0 || G <= 0) return hipSuccess;
    if (B <= 0) return hipErrorInvalidValue;
    const dim3 tg((unsigned)((G + 31) / 32), (unsigned)((M + 31) / 32));
    if (prec == 0)
        hipLaunchKernelGGL(k_wind_transpose<double>, tg, dim3(256), 0, st, (const double2*)W, M, G, B,
                           (double2*)Wt);
    else
        hipLaunchKernelGGL(k_wind_transpose<float>, tg, dim3(256), 0, st, (const float2*)W, M, G, B,
                           (float2*)Wt);
    return hipGetLastError();
}

hipError_t launch_rollout_grad(int prec, const RolloutParams& rp, const void* u, const void* W,
                               const double* states, const int32_t* k_active, const double* acpar,
                               const double* targets, const int8_t* kind, void* Wt, double* partial,
                               double* grad_out, hipStream_t st) {
    if (!grad_supported(rp.H, rp.S)) return hipErrorInvalidValue;
    {
        // one block of all M samples: the plain [G][M] interleaving
        const hipError_t e = launch_wind_transpose(prec, W, rp.M, rp.G, rp.M, Wt, st);
        if (e != hipSuccess) return e;
    }
    GradParams gp;
    gp.rp = rp;
    gp.Mp = grad_lanes_per_group(rp.M);
    gp.chunks = gp.Mp > 64 ? gp.Mp / 64 : 1;
    const int64_t lanes = (int64_t)rp.P * rp.N * gp.Mp;
    const unsigned blocks = (unsigned)((lanes + GR_BLOCK - 1) / GR_BLOCK);
    double* dst = gp.chunks > 1 ? partial : grad_out;
    if (rp.M >= GS_MIN_M && rp.M <= 128 && rp.H <= GS_MAXH && rp.G < (1 << 24)) {
        // the sample-independent chain hoisted: one (particle, aircraft) per
        // two-wave workgroup from 65 to 128 samples, per wave from 33 to 64,
        // two per wave (32 lanes each) from 17 to 32; lanes past M idle (a
        // sum over each 64 lanes of the group, written by its first lane)
        GradParams gs = gp;
        gs.Mp = rp.M > 64 ? 128 : rp.M > 32 ? 64 : 32;
        gs.chunks = gs.Mp > 64 ? gs.Mp / 64 : 1;
        const int gpw = gs.Mp >= 64 ? 1 : 64 / gs.Mp;
        const int block = gs.Mp > 64 ? gs.Mp : 64;
        const size_t lds = (size_t)gpw * (rp.H + 1) * GS_REC * (prec == 0 ? 8 : 4);
        const int64_t groups = (int64_t)rp.P * rp.N;
        const unsigned blocks = (unsigned)((groups + gpw - 1) / gpw);
        double* gdst = gs.chunks > 1 ? partial : grad_out;
        if (prec == 0) {
            auto k = gs.Mp == 128 ? k_rollout_grad_split<double, 128>
                     : gs.Mp == 64 ? k_rollout_grad_split<double, 64> : k_rollout_grad_split<double, 32>;
            hipLaunchKernelGGL(k, dim3(blocks), dim3(block), lds, st, gs, (const double*)u,
                               (const double*)Wt, states, k_active, acpar, targets, kind, gdst);
        } else {
            auto k = gs.Mp == 128 ? k_rollout_grad_split<float, 128>
                     : gs.Mp == 64 ? k_rollout_grad_split<float, 64> : k_rollout_grad_split<float, 32>;
            hipLaunchKernelGGL(k, dim3(blocks), dim3(block), lds, st, gs, (const float*)u,
                               (const float*)Wt, states, k_active, acpar, targets, kind, gdst);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || gs.chunks == 1) return e;
        const int64_t n = (int64_t)rp.P * rp.N * rp.S * 3;
        hipLaunchKernelGGL(k_grad_chunks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                           gs.chunks, partial, grad_out);
        return hipGetLastError();
    }
    const int nseg = (rp.H + GR_CK - 1) / GR_CK;
    if (prec == 0) {
        hipLaunchKernelGGL((k_rollout_grad<double, GR_MAXSEG, false>), dim3(blocks),
                           dim3(GR_BLOCK), 0, st, gp, (const double*)u, (const double*)Wt, states,
                           k_active, acpar, targets, kind, dst);
    } else {
        // register checkpoints up to 6 segments (150 steps): 166 VGPRs, still
        // three waves per SIMD; longer horizons keep them in scratch memory
        auto k = nseg <= 6 ? k_rollout_grad<float, 6, true> : k_rollout_grad<float, GR_MAXSEG, false>;
        hipLaunchKernelGGL(k, dim3(blocks), dim3(GR_BLOCK), 0, st, gp, (const float*)u,
                           (const float*)Wt, states, k_active, acpar, targets, kind, dst);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || gp.chunks == 1) return e;
    const int64_t n = (int64_t)rp.P * rp.N * rp.S * 3;
    hipLaunchKernelGGL(k_grad_chunks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       gp.chunks, partial, grad_out);
    return hipGetLastError();
}

// ---- Langevin proposal and acceptance -----------------------------------------------

// u' = u + (eps^2 / 2) g + eps xi with g = -(beta / M) * grad_sum (the drift
// of the tempered fuel + time target), xi from the MALA stream.
template <typename R>
__global__ void k_mala_propose(int64_t count, const R* __restrict__ u, const double* __restrict__ gsum,
                               double coef, double eps, Stream s, R* __restrict__ up) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    mala_propose_at<R>(e, u, gsum, coef, eps, s, up);
}

template <typename R>
__global__ void k_mala_decide(int P, int N, int D, const R* __restrict__ u, const R* __restrict__ up,
                              const double* __restrict__ g, const double* __restrict__ gp_,
                              double coef, double eps, const double* __restrict__ logw,
                              const double* __restrict__ logw_prop, Stream s,
                              int32_t* __restrict__ flags) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    flags[p] = mala_decide_at<R>(p, N, D, u, up, g, gp_, coef, eps, logw, logw_prop, s);
}

hipError_t launch_mala_propose(int prec, int64_t count, const void* u, const double* gsum,
                               double coef, double eps, Stream s, void* up, hipStream_t st) {
    const unsigned blocks = (unsigned)((count + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_mala_propose<double>, dim3(blocks), dim3(256), 0, st, count,
                           (const double*)u, gsum, coef, eps, s, (double*)up);
    else
        hipLaunchKernelGGL(k_mala_propose<float>, dim3(blocks), dim3(256), 0, st, count,
                           (const float*)u, gsum, coef, eps, s, (float*)up);
    return hipGetLastError();
}

hipError_t launch_mala_decide(int prec, int P, int N, int D, const void* u, const void* up,
                              const double* g, const double* gprop, double coef, double eps,
                              const double* logw, const double* logw_prop, Stream s,
                              int32_t* flags, hipStream_t st) {
    const unsigned blocks = (unsigned)((P + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_mala_decide<double>, dim3(blocks), dim3(256), 0, st, P, N, D,
                           (const double*)u, (const double*)up, g, gprop, coef, eps, logw,
                           logw_prop, s, flags);
    else
        hipLaunchKernelGGL(k_mala_decide<float>, dim3(blocks), dim3(256), 0, st, P, N, D,
                           (const float*)u, (const float*)up, g, gprop, coef, eps, logw,
                           logw_prop, s, flags);
    return hipGetLastError();
}

}  // namespace smc
