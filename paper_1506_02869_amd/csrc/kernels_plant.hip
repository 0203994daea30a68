// The plant of the receding-horizon loop (Sec. "Model Predictive Control":
// only the first part of the optimised control sequence is applied, and the
// plant's disturbance differs from the optimiser's predictions; Sec.
// "Rolling Window": aircraft join at their pre-determined step and leave the
// problem when they finish).  One lane per aircraft: every aircraft that has
// joined flies the applied steps of its plan through one wind sample (one
// static field, or under the paper's time-correlated model that sample's
// field of each step, p.w_kstride reals apart) with the rollout's per-step
// arithmetic; an arrival stops when it meets the landing
// sector.  Written back: the states after the steps, the shifted activation
// steps and the events (1 landed, 2 left through the exit radius).
#include "rollout_math.h"

namespace smc {

template <typename R>
__global__ void __launch_bounds__(64)
k_plant(const RolloutParams p, const double* __restrict__ ctrl, const R* __restrict__ W,
        const double* __restrict__ states, const int32_t* __restrict__ k_active,
        const double* __restrict__ acpar, const double* __restrict__ targets,
        const int8_t* __restrict__ kind, int n_steps, double* __restrict__ states_out,
        int32_t* __restrict__ k_active_out, int32_t* __restrict__ event_out) {
    typedef typename V2<R>::t R2;
    typedef Ops<R> O;
    const int i = threadIdx.x;
    const int N = p.N, S = p.S, H = p.H;
    if (i >= N) return;

    const double* ac = acpar + i * 9;
    const R Sw = (R)ac[0], cd0 = (R)ac[1], cd2 = (R)ac[2], cf1 = (R)ac[3];
    const R inv_cf2 = (R)(1.0 / ac[4]);
    const bool is_arr = kind[i] == 0;
    const int k0 = k_active[i];
    const bool active = k0 >= 0 && k0 < H;
    const double* st = states + i * 6;
    R x = (R)st[0], y = (R)st[1], z = (R)st[2], v = (R)st[3], chi = (R)st[4];
    const R m0 = (R)st[5];
    R burn = 0, burn_c = 0;

    const R dt = (R)p.dt, inv_dt = (R)(1.0 / p.dt), g0 = (R)kG0, inv_g = (R)(1.0 / kG0);
    const R half_wx = (R)p.half_wx, half_wy = (R)p.half_wy;
    const R inv_hx = (R)p.inv_hx, inv_hy = (R)p.inv_hy, inv_hz = (R)p.inv_hz;
    const R fnx1 = (R)(p.nx - 1), fny1 = (R)(p.ny - 1), fnz1 = (R)(p.nz - 1);
    const int nyz = p.ny * p.nz, nzz = p.nz;
    const R p_run = (R)p.p_run, p_beta = (R)p.p_beta, p_chi = (R)p.p_chi, p_vs = (R)p.p_vs;
    const R isa_c = (R)(kLapse / kT0), isa_e = (R)(kG0 / (kRair * kLapse) - 1.0);
    const R rho0 = (R)kRho0;
    const R2* W0 = (const R2*)W;                 // the plant's wind sample (step 0)

    bool landed = false;
    for (int k = 0; k < n_steps; ++k) {
        if (!active || k < k0 || landed) continue;
        const int s = (k * S) / H;
        const int k_end = ((s + 1) * H + S - 1) / S;
        const R chidot = (R)ctrl[(i * S + s) * 3 + 0];
        const R vc = (R)ctrl[(i * S + s) * 3 + 1];
        const R zdot = (R)ctrl[(i * S + s) * 3 + 2];
        const R inv_rem = O::rcp((R)(k_end - k));

        // trilinear wind of step k at the current position (coordinates clamped)
        const R2* Wm = (const R2*)((const R*)W0 + (int64_t)k * p.w_kstride);
        const R fx = clampr((x + half_wx) * inv_hx, (R)0, fnx1);
        const R fy = clampr((y + half_wy) * inv_hy, (R)0, fny1);
        const R fz = clampr(z * inv_hz, (R)0, fnz1);
        const int ix = min((int)fx, p.nx - 2), iy = min((int)fy, p.ny - 2),
                  iz = min((int)fz, p.nz - 2);
        const R tx = fx - (R)ix, ty = fy - (R)iy, tz = fz - (R)iz;
        const int g = (ix * p.ny + iy) * nzz + iz;
        const R2 c000 = Wm[g], c001 = Wm[g + 1], c010 = Wm[g + nzz], c011 = Wm[g + nzz + 1];
        const R2 c100 = Wm[g + nyz], c101 = Wm[g + nyz + 1], c110 = Wm[g + nyz + nzz],
                 c111 = Wm[g + nyz + nzz + 1];
        const R a00x = c000.x + tz * (c001.x - c000.x), a00y = c000.y + tz * (c001.y - c000.y);
        const R a01x = c010.x + tz * (c011.x - c010.x), a01y = c010.y + tz * (c011.y - c010.y);
        const R a10x = c100.x + tz * (c101.x - c100.x), a10y = c100.y + tz * (c101.y - c100.y);
        const R a11x = c110.x + tz * (c111.x - c110.x), a11y = c110.y + tz * (c111.y - c110.y);
        const R b0x = a00x + ty * (a01x - a00x), b0y = a00y + ty * (a01y - a00y);
        const R b1x = a10x + ty * (a11x - a10x), b1y = a10y + ty * (a11y - a10y);
        const R wx = b0x + tx * (b1x - b0x);
        const R wy = b0y + tx * (b1y - b0y);

        // climb angle, bank, aerodynamics, thrust, fuel; Euler update
        const R sg = zdot * O::rcp(v);
        const R cg = O::sqrt((R)1 - sg * sg);
        const R tphi = v * chidot * inv_g;
        const R inv_cphi = O::sqrt((R)1 + tphi * tphi);
        const R zc = clampr(z, (R)0, (R)11000);
        const R rho = rho0 * O::pow_pos((R)1 - isa_c * zc, isa_e);
        const R qd = (R)0.5 * rho * v * v;
        const R mass = m0 - burn;
        const R CL = O::div(mass * g0 * inv_cphi, qd * Sw);
        const R D = qd * Sw * (cd0 + cd2 * CL * CL);
        const R vn = v + (vc - v) * inv_rem;
        const R T = mass * (vn - v) * inv_dt + D + mass * g0 * sg;
        const R eta = cf1 * ((R)1 + v * inv_cf2);
        const R fuel = dt * eta * m_max(T, (R)0);
        R sc, cc;
        O::sincos(chi, &sc, &cc);
        x = x + dt * (v * cc * cg + wx);
        y = y + dt * (v * sc * cg + wy);
        z = z + dt * (v * sg);
        chi = chi + dt * chidot;
        v = vn;
        kahan_add(burn, burn_c, fuel);

        if (is_arr) {   // landing sector (eq. TO_init) on the new state
            const R r = O::sqrt(x * x + y * y);
            const R tha = m_abs(O::atan2(y, x));
            const R ratio = tha > (R)1e-4 ? tha * O::rcp(m_max(O::sin(tha), (R)1e-6))
                                          : (R)1 + tha * tha * (R)(1.0 / 6.0);
            const R beta = O::atan2(z, r * ratio);
            landed = r <= p_run && beta <= p_beta && tha <= p_chi &&
                     m_abs(wrap_angle<R>(chi - Consts<R>::pi)) <= p_chi && v <= p_vs;
        }
    }

    double* so = states_out + i * 6;
    so[0] = (double)x; so[1] = (double)y; so[2] = (double)z; so[3] = (double)v;
    so[4] = (double)chi; so[5] = (double)(m0 - burn);
    const bool joined = active && k0 < n_steps;
    const double r = sqrt((double)x * (double)x + (double)y * (double)y);
    const bool exited = joined && !is_arr && r >= targets[i * 4 + 3];
    const int ev = landed ? 1 : (exited ? 2 : 0);
    event_out[i] = ev;
    k_active_out[i] = (k0 < 0 || ev > 0) ? -1 : max(k0 - n_steps, 0);
}

hipError_t launch_plant(int prec, const RolloutParams& p, const double* ctrl, const void* W,
                        const double* states, const int32_t* k_active, const double* acpar,
                        const double* targets, const int8_t* kind, int n_steps,
                        double* states_out, int32_t* k_active_out, int32_t* event_out,
                        hipStream_t st) {
    if (p.N < 1 || p.N > 64 || n_steps < 1 || n_steps > p.H) return hipErrorInvalidValue;
    if (prec == 0)
        hipLaunchKernelGGL(k_plant<double>, dim3(1), dim3(64), 0, st, p, ctrl, (const double*)W,
                           states, k_active, acpar, targets, kind, n_steps, states_out,
                           k_active_out, event_out);
    else
        hipLaunchKernelGGL(k_plant<float>, dim3(1), dim3(64), 0, st, p, ctrl, (const float*)W,
                           states, k_active, acpar, targets, kind, n_steps, states_out,
                           k_active_out, event_out);
    return hipGetLastError();
}

}  // namespace smc
