// Rollout, world-per-lane layout: one lane integrates all N aircraft of one
// (particle, wind sample) world, with every aircraft's state in registers
// (N is a compile-time bucket NMAX >= N).
//
// The per-step arithmetic is the one of the aircraft-per-lane kernel (paper,
// Sec. "Trajectory Planning", eq. hor; Sec. "Constraint Handling"; eq.
// TO_init; Sec. "Particle Costing", "Noise Pollution Reduction"; eq.
// avoidance).  What the layout changes on the hardware:
//   * aircraft i is processed by all lanes at once, so its kind, activation
//     step and parameters are wave-uniform: scalar loads and uniform branches,
//     no arrival/departure divergence;
//   * the N (N - 1) / 2 separation tests of a step are lane-local register
//     arithmetic with compile-time pair masks, no LDS exchange;
//   * the lanes of a wave are consecutive particles under the same wind
//     sample, so the trilinear gathers of a wave hit one field.
// A segment's controls are staged in LDS ([aircraft][control][lane], each
// lane reads only its own column) to keep them out of the register budget.
#include "rollout_math.h"

namespace smc {

// Occupancy target per bucket: the state takes about 8 VGPRs per aircraft.
template <typename R, int NMAX>
constexpr int wm_waves() { return sizeof(R) == 4 ? (NMAX <= 4 ? 4 : (NMAX <= 10 ? 3 : 2)) : 1; }

template <typename R, int NMAX>
__global__ void __launch_bounds__(256, (wm_waves<R, NMAX>()))
k_rollout_wm(const RolloutParams p, const RolloutArrays a, const R* __restrict__ acR) {
    typedef typename V2<R>::t R2;
    typedef Ops<R> O;
    extern __shared__ unsigned char smem_raw[];
    R* uc = reinterpret_cast<R*>(smem_raw);   // [N][3][blockDim.x]

    const int tid = threadIdx.x;
    const int bd = blockDim.x;
    const int N = p.N, S = p.S, H = p.H;
    const int64_t world = (int64_t)blockIdx.x * bd + tid;
    const int64_t nworld = (int64_t)p.P * p.M;
    const bool valid = world < nworld;
    const int l = valid ? (int)(world % p.P) : 0;
    const int m = valid ? (int)(world / p.P) : 0;

    // uniform scalars
    const R dt = (R)p.dt, inv_dt = (R)(1.0 / p.dt), g0 = (R)kG0, inv_g = (R)(1.0 / kG0);
    const R half_wx = (R)p.half_wx, half_wy = (R)p.half_wy;
    const R inv_hx = (R)p.inv_hx, inv_hy = (R)p.inv_hy, inv_hz = (R)p.inv_hz;
    const R fnx1 = (R)(p.nx - 1), fny1 = (R)(p.ny - 1), fnz1 = (R)(p.nz - 1);
    const int nyz = p.ny * p.nz, nzz = p.nz;
    const R sep_h2 = (R)p.sep_h2, sep_v = (R)p.sep_v;
    const R zmin = (R)p.zmin, zmax = (R)p.zmax, vmin = (R)p.vmin, vmax = (R)p.vmax;
    const R p_run = (R)p.p_run, p_beta = (R)p.p_beta, p_chi = (R)p.p_chi, p_vs = (R)p.p_vs;
    const R beta_f = (R)p.beta_f;
    const R mix = (R)(1.0 - p.w[7] - p.w[8]);
    const R w_hdg = (R)p.w[0], w_gl = (R)p.w[1], w_brg = (R)p.w[3], w_alt = (R)p.w[5],
            w_spd = (R)p.w[6], a_time = (R)p.w[7], a_noise = (R)p.w[8];
    const R inv_tnorm = (R)(1.0 / p.time_norm);
    const R zdm_dt = (R)(p.zdot_max * p.dt);
    const R inv_Ac = (R)(1.0 / p.noise_alt);
    const R isa_c = (R)(kLapse / kT0), isa_e = (R)(kG0 / (kRair * kLapse) - 1.0);
    const R rho0 = (R)kRho0;

    R x[NMAX], y[NMAX], z[NMAX], v[NMAX], chi[NMAX], burn[NMAX], acc[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        if (i < N) {
            const double* st = a.states + 6 * i;
            x[i] = (R)st[0]; y[i] = (R)st[1]; z[i] = (R)st[2]; v[i] = (R)st[3]; chi[i] = (R)st[4];
        } else {
            x[i] = y[i] = z[i] = chi[i] = (R)0; v[i] = (R)1;
        }
        burn[i] = (R)0;
        acc[i] = (R)0;
    }
    uint32_t done = 0u, bad = 0u, sepbad = 0u;
    int nsim = 0, npair = 0;

    const R* ub = (const R*)a.u + (int64_t)l * N * S * 3;
    const R2* Wm = (const R2*)a.W + (int64_t)m * p.G;
    int s_cur = -1, k_end = 0;

    for (int k = 0; k < H; ++k) {
        const int s = (k * S) / H;
        if (s != s_cur) {  // uniform: stage the segment's physical controls
            s_cur = s;
            k_end = ((s + 1) * H + S - 1) / S;
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    uc[(i * 3 + c) * bd + tid] =
                        (R)p.ctrl_lo[c] + ub[(i * S + s) * 3 + c] * (R)p.ctrl_span[c];
        }
        const R inv_rem = O::rcp((R)(k_end - k));
        uint32_t pres = 0u;

#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i >= N) continue;
            const int k0 = a.k_active[i];
            if (k0 < 0 || k0 >= H || k < k0) continue;   // wave-uniform
            if ((done >> i) & 1u) continue;               // landed in this world
            pres |= 1u << i;
            ++nsim;
            const R* c_i = acR + 16 * i;                  // uniform parameters
            const R chidot = uc[(i * 3 + 0) * bd + tid];
            const R vc = uc[(i * 3 + 1) * bd + tid];
            const R zdot = uc[(i * 3 + 2) * bd + tid];
            const R xi = x[i], yi = y[i], zi = z[i], vi = v[i], chii = chi[i];

            // trilinear wind (coordinates clamped to the grid)
            const R fx = clampr((xi + half_wx) * inv_hx, (R)0, fnx1);
            const R fy = clampr((yi + half_wy) * inv_hy, (R)0, fny1);
            const R fz = clampr(zi * inv_hz, (R)0, fnz1);
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

            // climb angle, bank, aerodynamics, thrust, fuel
            const R sg = zdot * O::rcp(vi);
            const R cg = O::sqrt((R)1 - sg * sg);
            const R tphi = vi * chidot * inv_g;
            const R inv_cphi = O::sqrt((R)1 + tphi * tphi);
            const R zc = clampr(zi, (R)0, (R)11000);
            const R rho = rho0 * O::pow_pos((R)1 - isa_c * zc, isa_e);
            const R qd = (R)0.5 * rho * vi * vi;
            const R m0 = (R)a.states[6 * i + 5];
            const R mass = m0 - burn[i];
            const R Sw = c_i[0];
            const R CL = O::div(mass * g0 * inv_cphi, qd * Sw);
            const R D = qd * Sw * (c_i[1] + c_i[2] * CL * CL);
            const R vn = vi + (vc - vi) * inv_rem;
            const R T = mass * (vn - vi) * inv_dt + D + mass * g0 * sg;
            const R eta = c_i[3] * ((R)1 + vi * c_i[4]);
            const R fuel = dt * eta * m_max(T, (R)0);
            R sc, cc;
            O::sincos(chii, &sc, &cc);
            const R xn = xi + dt * (vi * cc * cg + wx);
            const R yn = yi + dt * (vi * sc * cg + wy);
            const R zn = zi + dt * (vi * sg);
            const R chin = chii + dt * chidot;
            const R burn_n = burn[i] + fuel;
            const R mn = m0 - burn_n;
            const bool viol = (T > c_i[5]) || (m_abs(tphi) >= c_i[7]) || (m_abs(sg) > c_i[8]) ||
                              (zn < zmin) || (zn > zmax) || (vn < vmin) || (vn > vmax) ||
                              (mn < c_i[6]);
            if (viol) bad |= 1u << i;
            x[i] = xn; y[i] = yn; z[i] = zn; v[i] = vn; chi[i] = chin; burn[i] = burn_n;

            // geometry at the new state
            const R r = O::sqrt(xn * xn + yn * yn);
            const R theta = O::atan2(yn, xn);
            const R tha = m_abs(theta);
            const R inv_vv = O::rcp(m_max(vn, vmin));
            R cst;
            if (c_i[14] == (R)0) {   // arrival (uniform)
                const R ratio = tha > (R)1e-4 ? tha * O::rcp(m_max(O::sin(tha), (R)1e-6))
                                              : (R)1 + tha * tha * (R)(1.0 / 6.0);
                const R s_arc = r * ratio;
                const R beta = O::atan2(zn, s_arc);
                const bool landed = r <= p_run && beta <= p_beta && tha <= p_chi &&
                                    m_abs(wrap_angle<R>(chin - Consts<R>::pi)) <= p_chi &&
                                    vn <= p_vs;
                if (landed) done |= 1u << i;
                const R hdg = m_abs(wrap_angle<R>(chin - (Consts<R>::pi + (R)2 * theta))) *
                              (R)(1.0 / Consts<double>::pi);
                const R glide = m_abs(beta - beta_f) * (R)(1.0 / Consts<double>::half_pi);
                const R tt = m_min(s_arc * inv_vv * inv_tnorm, (R)1);
                cst = landed ? (R)0 : mix * (w_hdg * hdg + w_gl * glide) + a_time * tt;
            } else {                 // departure
                const R brg = m_abs(wrap_angle<R>(theta - c_i[9])) * (R)(1.0 / Consts<double>::pi);
                const R d0 = m_abs(c_i[10] - (R)a.states[6 * i + 2]);
                const R span = zdm_dt * (R)max(k + 1 - k0, 1);
                const R sup = d0 + span;
                const R inf = m_max(d0 - span, (R)0);
                const R alt = clampr(O::div(m_abs(c_i[10] - zn) - inf, sup - inf), (R)0, (R)1);
                const R spd = m_abs(vn - c_i[11]) * c_i[13];
                const R tt = m_min(m_max(c_i[12] - r, (R)0) * inv_vv * inv_tnorm, (R)1);
                cst = mix * (w_brg * brg + w_alt * alt + w_spd * spd) + a_time * tt;
            }
            if (p.use_noise) {
                const R fpx = clampr((xn + half_wx) * (R)p.pop_inv_hx, (R)0, (R)(p.pop_nx - 1));
                const R fpy = clampr((yn + half_wy) * (R)p.pop_inv_hy, (R)0, (R)(p.pop_ny - 1));
                const int px = min((int)fpx, p.pop_nx - 2), py = min((int)fpy, p.pop_ny - 2);
                const R ux = fpx - (R)px, uy = fpy - (R)py;
                const float* pr = a.pop + (int64_t)py * p.pop_nx + px;
                const R p00 = (R)pr[0], p01 = (R)pr[1], p10 = (R)pr[p.pop_nx],
                        p11 = (R)pr[p.pop_nx + 1];
                const R pd = ((R)1 - ux) * ((R)1 - uy) * p00 + ux * ((R)1 - uy) * p01 +
                             ((R)1 - ux) * uy * p10 + ux * uy * p11;
                const R za = zn * inv_Ac;
                if (!((done >> i) & 1u)) cst += a_noise * (m_max((R)1 - za * za, (R)0) * pd);
            }
            acc[i] += cst;
        }

        {   // pair tests with both aircraft present (work count)
            const int np = __popc(pres);
            npair += np * (np - 1) / 2;
        }
        // separation at the new state among the aircraft simulated this step
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
#pragma unroll
            for (int j = i + 1; j < NMAX; ++j) {
                if (j >= N) continue;
                const R dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                const bool both = ((pres >> i) & (pres >> j) & 1u) != 0u;
                if (both && dx * dx + dy * dy < sep_h2 && m_abs(dz) < sep_v)
                    sepbad |= (1u << i) | (1u << j);
            }
        }
    }

    if (valid) {
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i >= N) continue;
            const int k0 = a.k_active[i];
            double cost = 0.0;
            if (k0 >= 0 && k0 < H) {
                const double* ac = a.acpar + 9 * i;
                const int nsteps = H - k0;
                const double wf = a.kind[i] == 0 ? p.w[2] : p.w[4];
                const double denom = p.dt * (double)nsteps * ac[5] * (ac[3] * (1.0 + p.vmax / ac[4]));
                cost = (1.0 - p.w[7] - p.w[8]) * wf * ((double)burn[i] / denom) +
                       (double)acc[i] / (double)nsteps;
            }
            const int64_t o = ((int64_t)m * p.P + l) * N + i;
            a.cost[o] = cost;
            a.feas[o] = (((bad | sepbad) >> i) & 1u) ? 0 : 1;
        }
    }
    if (a.steps) {
        int cnt = valid ? nsim : 0;
        int cp = valid ? npair : 0;
        for (int off = 32; off > 0; off >>= 1) {
            cnt += __shfl_xor(cnt, off);
            cp += __shfl_xor(cp, off);
        }
        if ((tid & 63) == 0) {
            if (cnt) atomicAdd(&a.steps[blockIdx.x & (kStepSlots - 1)], (unsigned long long)cnt);
            if (cp)
                atomicAdd(&a.steps[kStepSlots + (blockIdx.x & (kStepSlots - 1))],
                          (unsigned long long)cp);
        }
    }
}

// 256 lanes per block in FP32, 128 in FP64: the staged controls take
// N * 3 * block * sizeof(R) bytes of LDS (48 KB at N = 16 either way).
template <typename R, int NMAX>
static hipError_t launch_wm_n(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              hipStream_t st) {
    const int block = sizeof(R) == 4 ? 256 : 128;
    const int64_t nworld = (int64_t)p.P * p.M;
    const unsigned blocks = (unsigned)((nworld + block - 1) / block);
    const size_t lds = (size_t)p.N * 3 * block * sizeof(R);
    hipLaunchKernelGGL((k_rollout_wm<R, NMAX>), dim3(blocks), dim3(block), lds, st, p, a,
                       (const R*)acR);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_wm_t(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              hipStream_t st) {
    if (p.N <= 2) return launch_wm_n<R, 2>(p, a, acR, st);
    if (p.N <= 4) return launch_wm_n<R, 4>(p, a, acR, st);
    if (p.N <= 6) return launch_wm_n<R, 6>(p, a, acR, st);
    if (p.N <= 8) return launch_wm_n<R, 8>(p, a, acR, st);
    if (p.N <= 10) return launch_wm_n<R, 10>(p, a, acR, st);
    if (p.N <= 12) return launch_wm_n<R, 12>(p, a, acR, st);
    return launch_wm_n<R, 16>(p, a, acR, st);
}

bool rollout_wm_supported(int N) { return N >= 1 && N <= kWorldLaneMaxN; }

hipError_t launch_rollout_wm(int prec, const RolloutParams& p, const RolloutArrays& a,
                             const void* acR, hipStream_t st) {
    if (!rollout_wm_supported(p.N)) return hipErrorInvalidValue;
    if (p.P <= 0 || p.M <= 0) return hipSuccess;
    return prec == 0 ? launch_wm_t<double>(p, a, acR, st) : launch_wm_t<float>(p, a, acR, st);
}

}  // namespace smc
