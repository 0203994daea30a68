// Rollout of every (particle, wind sample, aircraft): one lane per aircraft,
// the N aircraft of one (particle, wind sample) "world" in consecutive lanes
// of one wavefront, aircraft state in registers for the whole horizon.
//
// Per step and lane (paper, Sec. "Trajectory Planning", eq. hor, with the
// per-segment kinematic controls mapped onto thrust / climb / bank through
// the inverse relations of Sec. "Fuel Estimate 1" and "Fuel Estimate 2"):
//   trilinear wind -> climb angle from climb rate -> bank from heading rate
//   -> ISA density, lift = weight in the turn, parabolic drag -> thrust that
//   realises the airspeed change -> fuel flow eta(v) -> Euler update ->
//   unary checks (Sec. "Constraint Handling") -> landing sector test
//   (eq. TO_init) -> per-step cost elements (Sec. "Particle Costing",
//   "Noise Pollution Reduction") -> pairwise separation (eq. avoidance)
//   through an LDS exchange of the new positions inside the workgroup.
// Up to 32 aircraft (or 64), each wavefront holds whole worlds and the
// double-buffered position exchange needs only the wavefront's order.  For
// 33 .. 63 aircraft, where one world per wavefront would leave many lanes
// idle, the worlds of a workgroup sit back to back in its lanes (a world may
// straddle two wavefronts; e.g. 8 worlds of 40 aircraft in 320 lanes) and
// one workgroup barrier per step orders the exchange.
// Pairs are split evenly over the world's lanes (lane i tests i against
// i+1 .. i+(N-1)/2 modulo N, plus i+N/2 for i < N/2 when N is even); a hit
// sets the bits of both aircraft in a per-lane violation mask that is
// OR-reduced over the world once, after the last step.  The pair tests with
// both aircraft present are counted per world and step from the wavefronts'
// presence ballots.
#include "rollout_math.h"

namespace smc {

template <typename R, bool PACKED>
__global__ void __launch_bounds__(sizeof(R) == 4 ? kRolloutMaxBlock32 : kRolloutMaxBlock64)
k_rollout(const RolloutParams p, const RolloutArrays a, int wpb) {
    typedef typename V2<R>::t R2;
    extern __shared__ unsigned char smem_raw[];
    const int nb = blockDim.x;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int N = p.N, S = p.S, H = p.H;
    int wib, i;        // world within the workgroup, aircraft
    bool inblk;        // the lane holds an aircraft of one of the workgroup's worlds
    if constexpr (PACKED) {
        wib = tid / N;
        i = tid - wib * N;
        inblk = wib < wpb;
    } else {           // whole worlds in each wavefront
        const int wpw = 64 / N;
        const int wiw = lane / N;
        i = lane - wiw * N;
        wib = (tid >> 6) * wpw + wiw;
        inblk = wiw < wpw;
    }
    const int lbase = tid - i;                     // lane of the world's aircraft 0
    const int64_t world = (int64_t)blockIdx.x * wpb + wib;
    const int64_t nworld = (int64_t)p.P * p.M;
    const bool valid = inblk && (world < nworld);
    const int pidx = valid ? (int)(world % p.P) : 0;
    const int m = valid ? (int)(world / p.P) : 0;
    const int base = wib * N;
    // Positions as two arrays of pairs, (x, y) and (z, present), each world
    // stored twice in a row (2N entries): the partner i + d of lane i needs no
    // wrap, and its address is the lane's own plus a constant.
    const int nslot = 2 * wpb * N;                // entries per buffer
    R2* pxy = reinterpret_cast<R2*>(smem_raw);    // [2][nslot]
    R2* pzw = pxy + 2 * nslot;                    // [2][nslot]

    // per-aircraft constants
    const double* ac = a.acpar + i * 9;
    const R Sw = (R)ac[0], cd0 = (R)ac[1], cd2 = (R)ac[2], cf1 = (R)ac[3];
    const R tmax = (R)ac[5], m_empty = (R)ac[6];
    const R tan_phimax = (R)tan(ac[7]);
    const R sin_gmax = (R)sin(ac[8]);
    const bool is_arr = a.kind[i] == 0;
    const double* tg = a.targets + i * 4;
    const R thF = (R)tg[0], Zt = (R)tg[1], vD = (R)tg[2], dtma = (R)tg[3];
    const R inv_spd_den = (R)(1.0 / fmax(p.vmax - tg[2], tg[2] - p.vmin));
    const R inv_cf2 = (R)(1.0 / ac[4]);
    const int k0 = a.k_active[i];
    const bool active = valid && k0 >= 0 && k0 < H;
    const double* st = a.states + i * 6;
    R x = (R)st[0], y = (R)st[1], z = (R)st[2], v = (R)st[3], chi = (R)st[4];
    const R m0 = (R)st[5];
    const R d0 = m_abs(Zt - (R)st[2]);

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
    const R sent_x = (R)(1e9 + 1e7 * i);

    const R* ubase = (const R*)a.u + ((int64_t)pidx * N + i) * (int64_t)(S * 3);
    const R2* Wm = (const R2*)a.W + (int64_t)m * p.G;

    R burn = 0, burn_c = 0, acc = 0, acc_c = 0;
    bool feas_unary = true, done = false;
    // separation hits relative to the lane: bit d of relmask is set once the
    // pair (i, i + d mod N) violated, d = 1 .. (N - 1) / 2; halfhit for the
    // pair (i, i + N / 2) of an even N (lanes i < N / 2)
    uint32_t relmask = 0u;
    bool halfhit = false;
    int nsim = 0, npair = 0;
    R chidot = 0, vc = 0, zdot = 0;
    int s_cur = -1, k_end = 0;
    R inv_rem = 0;

    for (int k = 0; k < H; ++k) {
        const int s = (k * S) / H;
        if (s != s_cur) {  // uniform branch: depends on k only
            s_cur = s;
            chidot = (R)p.ctrl_lo[0] + ubase[s * 3 + 0] * (R)p.ctrl_span[0];
            vc = (R)p.ctrl_lo[1] + ubase[s * 3 + 1] * (R)p.ctrl_span[1];
            zdot = (R)p.ctrl_lo[2] + ubase[s * 3 + 2] * (R)p.ctrl_span[2];
            k_end = ((s + 1) * H + S - 1) / S;
            // FP32: heading back into [-pi, pi) at each segment start (its
            // rounding stays that of an angle near pi)
            if constexpr (sizeof(R) == 4) chi = wrap_angle<R>(chi);
        }
        // airspeed ramps to vc by the segment's end: 1 / (steps remaining)
        inv_rem = Ops<R>::rcp((R)(k_end - k));
        const bool present = active && k >= k0 && !done;

        // trilinear wind at the current position (coordinates clamped)
        R fx = clampr((x + half_wx) * inv_hx, (R)0, fnx1);
        R fy = clampr((y + half_wy) * inv_hy, (R)0, fny1);
        R fz = clampr(z * inv_hz, (R)0, fnz1);
        const int ix = min((int)fx, p.nx - 2), iy = min((int)fy, p.ny - 2),
                  iz = min((int)fz, p.nz - 2);
        const R tx = fx - (R)ix, ty = fy - (R)iy, tz = fz - (R)iz;
        const int g = (ix * p.ny + iy) * nzz + iz;
        const R2 c000 = Wm[g], c001 = Wm[g + 1], c010 = Wm[g + nzz], c011 = Wm[g + nzz + 1];
        const R2 c100 = Wm[g + nyz], c101 = Wm[g + nyz + 1], c110 = Wm[g + nyz + nzz],
                 c111 = Wm[g + nyz + nzz + 1];
        R2 w;
        {
            const R a00x = c000.x + tz * (c001.x - c000.x), a00y = c000.y + tz * (c001.y - c000.y);
            const R a01x = c010.x + tz * (c011.x - c010.x), a01y = c010.y + tz * (c011.y - c010.y);
            const R a10x = c100.x + tz * (c101.x - c100.x), a10y = c100.y + tz * (c101.y - c100.y);
            const R a11x = c110.x + tz * (c111.x - c110.x), a11y = c110.y + tz * (c111.y - c110.y);
            const R b0x = a00x + ty * (a01x - a00x), b0y = a00y + ty * (a01y - a00y);
            const R b1x = a10x + ty * (a11x - a10x), b1y = a10y + ty * (a11y - a10y);
            w.x = b0x + tx * (b1x - b0x);
            w.y = b0y + tx * (b1y - b0y);
        }

        // climb angle, bank, aerodynamics, thrust, fuel
        typedef Ops<R> O;
        const R inv_v = O::rcp(v);
        const R sg = zdot * inv_v;
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
        const R xn = x + dt * (v * cc * cg + w.x);
        const R yn = y + dt * (v * sc * cg + w.y);
        const R zn = z + dt * (v * sg);
        const R chin = chi + dt * chidot;
        R burn_n = burn, burn_cn = burn_c;
        kahan_add(burn_n, burn_cn, fuel);
        const R mn = m0 - burn_n;
        const bool viol = (T > tmax) || (m_abs(tphi) >= tan_phimax) || (m_abs(sg) > sin_gmax) ||
                          (zn < zmin) || (zn > zmax) || (vn < vmin) || (vn > vmax) ||
                          (mn < m_empty);
        if (present) {
            if (viol) feas_unary = false;
            x = xn; y = yn; z = zn; v = vn; chi = chin;
            burn = burn_n; burn_c = burn_cn;
            ++nsim;
        }

        // geometry at the new state, shared by the landing test and the cost
        // elements of both kinds (one wrap, one time-to-go)
        const R r = O::sqrt(x * x + y * y);
        const R theta = O::atan2(y, x);
        const R tha = m_abs(theta);
        const R ratio = tha > (R)1e-4 ? tha * O::rcp(m_max(O::sin(tha), (R)1e-6))
                                      : (R)1 + tha * tha * (R)(1.0 / 6.0);
        const R s_arc = r * ratio;
        const R inv_vv = O::rcp(m_max(v, vmin));
        // arrivals: heading off the flow field chi_hat = pi + 2 theta;
        // departures: bearing off the target bearing
        const R ang = is_arr ? chi - (Consts<R>::pi + (R)2 * theta) : theta - thF;
        const R e_ang = m_abs(wrap_angle<R>(ang)) * (R)(1.0 / Consts<double>::pi);
        const R tnum = is_arr ? s_arc : m_max(dtma - r, (R)0);
        const R tt = m_min(tnum * inv_vv * inv_tnorm, (R)1);
        R c;
        bool landed = false;
        if (is_arr) {
            const R beta = O::atan2(z, s_arc);
            landed = present && r <= p_run && beta <= p_beta && tha <= p_chi &&
                     m_abs(wrap_angle<R>(chi - Consts<R>::pi)) <= p_chi && v <= p_vs;
            const R glide = m_abs(beta - beta_f) * (R)(1.0 / Consts<double>::half_pi);
            c = mix * (w_hdg * e_ang + w_gl * glide) + a_time * tt;
        } else {
            const R span = zdm_dt * (R)max(k + 1 - k0, 1);
            const R sup = d0 + span;
            const R inf = m_max(d0 - span, (R)0);
            const R alt = clampr(O::div(m_abs(Zt - z) - inf, sup - inf), (R)0, (R)1);
            const R spd = m_abs(v - vD) * inv_spd_den;
            c = mix * (w_brg * e_ang + w_alt * alt + w_spd * spd) + a_time * tt;
        }
        if (p.use_noise) {
            R fpx = clampr((x + half_wx) * (R)p.pop_inv_hx, (R)0, (R)(p.pop_nx - 1));
            R fpy = clampr((y + half_wy) * (R)p.pop_inv_hy, (R)0, (R)(p.pop_ny - 1));
            const int px = min((int)fpx, p.pop_nx - 2), py = min((int)fpy, p.pop_ny - 2);
            const R ux = fpx - (R)px, uy = fpy - (R)py;
            const float* pr = a.pop + (int64_t)py * p.pop_nx + px;
            const R p00 = (R)pr[0], p01 = (R)pr[1], p10 = (R)pr[p.pop_nx], p11 = (R)pr[p.pop_nx + 1];
            const R pd = ((R)1 - ux) * ((R)1 - uy) * p00 + ux * ((R)1 - uy) * p01 +
                         ((R)1 - ux) * uy * p10 + ux * uy * p11;
            const R za = z * inv_Ac;
            c += a_noise * (m_max((R)1 - za * za, (R)0) * pd);
        }
        if (present && !landed) kahan_add(acc, acc_c, c);
        if (landed) done = true;

        // separation at the new state among aircraft simulated this step.
        // Double buffering: a lane writes buffer k & 1 only after every lane
        // passed the barrier of step k - 1, i.e. finished reading it at k - 2.
        const int buf = k & 1;
        const R px_ = present ? x : sent_x;
        const R py_ = present ? y : (R)0;
        const R pz_ = present ? z : (R)0;
        R2 mxy, mzw;
        mxy.x = px_; mxy.y = py_;
        mzw.x = pz_; mzw.y = present ? (R)1 : (R)0;
        if (inblk) {
            const int o = buf * nslot + 2 * base + i;
            pxy[o] = mxy; pxy[o + N] = mxy;
            pzw[o] = mzw; pzw[o + N] = mzw;
        }
        // a world's lanes in one wavefront need only the wavefront's order;
        // one barrier per step orders the workgroup otherwise
        if constexpr (PACKED) __syncthreads(); else wave_sync();
        if (valid) {
            const R2* qxy = pxy + buf * nslot + 2 * base + i;   // partner d at [d]
            const R2* qzw = pzw + buf * nslot + 2 * base + i;
            R qsum = (R)0;
            const int half = (N - 1) >> 1;
            for (int d = 1; d <= half; ++d) {
                const R2 a2 = qxy[d], b2 = qzw[d];
                qsum += b2.y;
                const R dx = px_ - a2.x, dy = py_ - a2.y, dz = pz_ - b2.x;
                const bool hit = (dx * dx + dy * dy < sep_h2) & (m_abs(dz) < sep_v);
                relmask |= hit ? (1u << d) : 0u;
            }
            if (((N & 1) == 0) && i < (N >> 1)) {
                const int d = N >> 1;
                const R2 a2 = qxy[d], b2 = qzw[d];
                qsum += b2.y;
                const R dx = px_ - a2.x, dy = py_ - a2.y, dz = pz_ - b2.x;
                halfhit |= (dx * dx + dy * dy < sep_h2) & (m_abs(dz) < sep_v);
            }
            if (present) npair += (int)qsum;
        }
    }

    // an aircraft violated separation if its own tests hit, or if the lane
    // that tested it as partner i + d recorded bit d
    __syncthreads();
    uint32_t* rm = reinterpret_cast<uint32_t*>(smem_raw);   // [nb] relmask, [nb] halfhit
    rm[tid] = relmask;
    rm[nb + tid] = halfhit ? 1u : 0u;
    __syncthreads();
    bool sepbad = relmask != 0u || halfhit;
    if (valid) {
        const int half = (N - 1) >> 1;
        for (int d = 1; d <= half; ++d) {
            int src = i - d;
            if (src < 0) src += N;
            if ((rm[lbase + src] >> d) & 1u) sepbad = true;
        }
        if (((N & 1) == 0) && i >= (N >> 1) && rm[nb + lbase + i - (N >> 1)]) sepbad = true;
    }

    if (valid) {
        double cost = 0.0;
        if (active) {
            const int nsteps = H - k0;
            const double wf = is_arr ? p.w[2] : p.w[4];
            const double denom = p.dt * (double)nsteps * ac[5] * (ac[3] * (1.0 + p.vmax / ac[4]));
            const double fuel_term = (double)burn / denom;
            cost = (1.0 - p.w[7] - p.w[8]) * wf * fuel_term + (double)acc / (double)nsteps;
        }
        const bool ok = feas_unary && !sepbad;
        const int64_t o = ((int64_t)m * p.P + pidx) * N + i;
        a.cost[o] = cost;
        a.feas[o] = ok ? 1 : 0;
    }

    if (a.steps) {
        int cnt = valid ? nsim : 0;
        int cp = valid ? npair : 0;
        for (int off = 32; off > 0; off >>= 1) {
            cnt += __shfl_xor(cnt, off);
            cp += __shfl_xor(cp, off);
        }
        if (lane == 0) {
            if (cnt) atomicAdd(&a.steps[blockIdx.x & (kStepSlots - 1)], (unsigned long long)cnt);
            if (cp)
                atomicAdd(&a.steps[kStepSlots + (blockIdx.x & (kStepSlots - 1))],
                          (unsigned long long)cp);
        }
    }
}

// Packed layout: worlds across wavefronts (see above).
bool rollout_packed(int N) { return N > 32 && N < 64; }

// Worlds per workgroup.  Packed: the count whose lanes (N per world, rounded
// up to whole wavefronts) are the busiest, the smaller workgroup on ties;
// otherwise four wavefronts of 64 / N worlds.
int rollout_worlds_per_block(int N, int prec) {
    if (!rollout_packed(N)) return 4 * (64 / N);
    const int maxb = prec == 0 ? kRolloutMaxBlock64 : kRolloutMaxBlock32;
    int best_k = 1;
    double best_u = -1.0;
    for (int k = 1; k * N <= maxb; ++k) {
        const int lanes = k * N;
        const int threads = (lanes + 63) / 64 * 64;
        const double u = (double)lanes / threads;
        if (u > best_u + 1e-12) { best_u = u; best_k = k; }
    }
    return best_k;
}

hipError_t launch_rollout(int prec, const RolloutParams& p, const RolloutArrays& a,
                          hipStream_t st) {
    if (p.N < 1 || p.N > 64) return hipErrorInvalidValue;
    const bool packed = rollout_packed(p.N);
    const int wpb = rollout_worlds_per_block(p.N, prec);
    const int threads = packed ? (wpb * p.N + 63) / 64 * 64 : 256;
    const int64_t nworld = (int64_t)p.P * p.M;
    const int64_t nblock = (nworld + wpb - 1) / wpb;
    if (nblock <= 0) return hipSuccess;
    const size_t rsz = prec == 0 ? sizeof(double) : sizeof(float);
    // two arrays of pairs, two buffers, each world twice
    const size_t lds = (size_t)2 * 2 * (2 * wpb * p.N) * 2 * rsz;
    if (prec == 0) {
        if (packed)
            hipLaunchKernelGGL((k_rollout<double, true>), dim3((unsigned)nblock), dim3(threads), lds,
                               st, p, a, wpb);
        else
            hipLaunchKernelGGL((k_rollout<double, false>), dim3((unsigned)nblock), dim3(threads),
                               lds, st, p, a, wpb);
    } else {
        if (packed)
            hipLaunchKernelGGL((k_rollout<float, true>), dim3((unsigned)nblock), dim3(threads), lds,
                               st, p, a, wpb);
        else
            hipLaunchKernelGGL((k_rollout<float, false>), dim3((unsigned)nblock), dim3(threads),
                               lds, st, p, a, wpb);
    }
    return hipGetLastError();
}

}  // namespace smc
