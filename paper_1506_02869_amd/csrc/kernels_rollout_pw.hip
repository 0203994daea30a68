// Rollout, particle-per-wave layout (FP32, 21 .. 64 aircraft): the 64 lanes
// of a wavefront are 64 wind samples of ONE particle, so every lane flies
// the same control sequences through its own wind field.
//
// The per-step arithmetic is that of the other layouts (paper, Sec.
// "Trajectory Planning", eq. hor; Sec. "Constraint Handling"; eq. TO_init;
// Sec. "Particle Costing", "Noise Pollution Reduction"; eq. avoidance).
// What the layout exploits: in the model the wind moves an aircraft only
// horizontally (x, y); its airspeed ramp, climb, heading, bank, density,
// drag, thrust, fuel flow and mass, and with them every unary constraint,
// the altitude-dependent cost elements and the altitude itself, are the
// same in all wind samples of a particle until the aircraft lands in one of
// them.  So each step has two phases:
//   1. lanes i < N each compute aircraft i's wind-independent step once for
//      the particle and store a small record in LDS (one wavefront's slice);
//   2. every lane (one world = one wind sample) runs the aircraft in turn,
//      reading the record by a broadcast LDS load: trilinear wind at its own
//      position, horizontal Euler update, landing test and the horizontal
//      cost elements.
// Separation (eq. avoidance) needs |dz| < sep_v AND dh < sep_h.  The
// altitudes are wave-uniform, so the vertical test of every pair is one
// ballot per aircraft over the phase-1 lanes; only pairs inside sep_v (a
// uniform bit mask) get the horizontal test, which reads the partner's
// position from registers by a uniform dynamic index (two vector halves of
// at most 32, indexed through the GPR index mode).  Skipping the other pairs
// is exact: their |dz| is at least sep_v in the same FP32 arithmetic.
// An aircraft that has landed in a world is parked far away (x = kGoneX +
// i kGoneDX) from the next step on, so the horizontal test needs no
// presence check.
// The fuel element is folded into the per-step sum: each simulated step adds
// (1 - alpha_time - alpha_noise) w_fuel fuel_k / (dt T_max eta(v_max)), so
// the element sum over the steps divided by their number is the fuel
// element plus the mean of the other elements.
#include "rollout_pw_common.h"

namespace smc {

// One aircraft of phase 2 in every world of the wave (aircraft i, index ii
// = i - 32 HI into the upper halves).  x, y: this half's vectors; xlo,
// ylo: the lower halves (pair partners below 32); masks per half; accl:
// this lane's cost sums in LDS, aircraft i at accl[i * 64].
// The vectors are written once each, unconditionally, at a uniform index
// (values chosen by selects), so that no vector is carried through a
// divergent branch.
template <bool HI, typename VX>
__device__ __forceinline__ void pw_aircraft(
    const RolloutParams& p, const RolloutArrays& a, const float* __restrict__ par,
    const float* __restrict__ rec, const PwTap& w, int i, uint64_t actk, float zn_lane, VX& x,
    VX& y, float* __restrict__ accl, const v32f& xlo, const v32f& ylo, uint32_t done0,
    uint32_t& done, uint32_t& bad, uint32_t& sepbad, uint32_t& sepbad_lo, int& nhor,
    PwNoise& noise) {
    typedef Ops<float> O;
    const RollConst<float>& q = p.cf;
    const int ii = HI ? i - 32 : i;
    const uint32_t bit = 1u << ii;
    const float4* r4 = reinterpret_cast<const float4*>(rec + i * kPwRec);
    const float4 ra = r4[0], rb = r4[1], rc = r4[2];
    // wave-uniform parts of the record moved to scalar registers: the
    // arrival / departure choice and the noise weight are uniform branches
    const uint32_t flags = __builtin_amdgcn_readfirstlane(__float_as_uint(rc.z));
    const float na = uniform_real(rc.x);
    const bool wasdone = (done0 & bit) != 0u;
    const float xi = w.xi, yi = w.yi, tx = w.tx, ty = w.ty, tz = w.tz;

    // trilinear wind of this world's sample at (x, y, z)
    const F2 c000 = w.c[0], c001 = w.c[1], c010 = w.c[2], c011 = w.c[3];
    const F2 c100 = w.c[4], c101 = w.c[5], c110 = w.c[6], c111 = w.c[7];
    const float a00x = c000.x + tz * (c001.x - c000.x), a00y = c000.y + tz * (c001.y - c000.y);
    const float a01x = c010.x + tz * (c011.x - c010.x), a01y = c010.y + tz * (c011.y - c010.y);
    const float a10x = c100.x + tz * (c101.x - c100.x), a10y = c100.y + tz * (c101.y - c100.y);
    const float a11x = c110.x + tz * (c111.x - c110.x), a11y = c110.y + tz * (c111.y - c110.y);
    const float b0x = a00x + ty * (a01x - a00x), b0y = a00y + ty * (a01y - a00y);
    const float b1x = a10x + ty * (a11x - a10x), b1y = a10y + ty * (a11y - a10y);
    const float wx = b0x + tx * (b1x - b0x);
    const float wy = b0y + tx * (b1y - b0y);

    const float xn = m_fma(q.dt, ra.x + wx, xi);
    const float yn = m_fma(q.dt, ra.y + wy, yi);
    const float zn = ra.z, chin = ra.w;
    // geometry at the new state
    const float r = O::sqrt(xn * xn + yn * yn);
    const float theta = O::atan2(yn, xn);
    const float tha = m_abs(theta);
    float cst;
    bool landed = false;
    if (!(flags & F_DEP)) {   // arrival (uniform)
        // both forms, then a select: no divergent branch
        // sin|theta| = |y| / r: the ratio |theta| / sin|theta| without the sine
        const float r_arc = tha * r * O::rcp(m_max(m_abs(yn), 1e-6f * r));
        const float r_small = 1.f + tha * tha * (1.f / 6.f);
        const float ratio = tha > 1e-4f ? r_arc : r_small;
        const float s_arc = r * ratio;
        const float beta = O::atan2(zn, s_arc);
        landed = !wasdone & (r <= q.p_run) & (beta <= q.p_beta) & (tha <= q.p_chi) &
                 ((flags & F_LANDOK) != 0u);
        const float hdg = m_abs(wrap_angle<float>(chin - (Consts<float>::pi + 2.f * theta)));
        const float tt = m_min(s_arc * rb.w, 1.f);
        cst = landed ? 0.f : q.c_hdg * hdg + q.c_gl * m_abs(beta - q.beta_f) + q.a_time * tt;
    } else {                  // departure
        const float* pi_ = par + i * kPwPar;
        const float brg = m_abs(wrap_angle<float>(theta - pi_[A_THF]));
        const float tt = m_min(m_max(pi_[A_DTMA] - r, 0.f) * rb.w, 1.f);
        cst = q.c_brg * brg + rb.z + q.a_time * tt;
    }
    noise.i = -1;
    if (p.use_noise && na != 0.f) {   // uniform: below the noise altitude
        const float fpx = clampr(m_fma(xn, q.pop_inv_hx, q.pop_ox), 0.f, q.fpnx1);
        const float fpy = clampr(m_fma(yn, q.pop_inv_hy, q.pop_oy), 0.f, q.fpny1);
        const int px = min((int)fpx, p.pop_nx - 2), py = min((int)fpy, p.pop_ny - 2);
        noise.ux = fpx - (float)px;
        noise.uy = fpy - (float)py;
        const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)a.pop, (short)0, p.pop_nx * p.pop_ny * 4, 0x00020000);
        const int po = (py * p.pop_nx + px) * 4;
        noise.p0 = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(prs, po, 0, 0));
        noise.p1 = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(prs, po, p.pop_nx * 4, 0));
        noise.w = (landed | wasdone) ? 0.f : na;
        noise.i = i;
    }
    accl[i * 64] += wasdone ? 0.f : cst + rc.y;
    done |= landed ? bit : 0u;
    bad |= ((flags & F_VIOL) != 0u && !wasdone) ? bit : 0u;
    // parked from the step after landing on (far away in x, distinct per
    // aircraft; y keeps moving, finite and unused)
    const float xs = wasdone ? (float)kGoneX + (float)kGoneDX * (float)i : xn;
    const float ys = yn;
    x[ii] = xs;
    y[ii] = ys;

    // separation against the aircraft already moved this step whose altitude
    // is within sep_v (a uniform candidate mask)
    const uint64_t vclose = __ballot(m_abs(zn_lane - zn) < q.sep_v);
    const uint64_t cand = vclose & actk & ((1ull << i) - 1ull);
    nhor += __popcll(cand);   // uniform: horizontal tests of this aircraft
    uint32_t c_lo = (uint32_t)cand;
    while (c_lo) {
        const int jj = __builtin_ctz(c_lo);
        c_lo &= c_lo - 1u;
        const float dx = xs - xlo[jj], dy = ys - ylo[jj];
        const bool hit = dx * dx + dy * dy < q.sep_h2;
        if (__builtin_expect(__ballot(hit) != 0ull, 0)) {
            if (hit) { sepbad |= bit; sepbad_lo |= 1u << jj; }
        }
    }
    if (HI) {
        uint32_t c_hi = (uint32_t)(cand >> 32);
        while (c_hi) {
            const int jj = __builtin_ctz(c_hi);
            c_hi &= c_hi - 1u;
            const float dx = xs - x[jj], dy = ys - y[jj];
            const bool hit = dx * dx + dy * dy < q.sep_h2;
            if (__builtin_expect(__ballot(hit) != 0ull, 0)) {
                if (hit) sepbad |= bit | (1u << jj);
            }
        }
    }
}

// Phase 2 over the active aircraft of one half (bits of `todo`, aircraft
// index base + bit), the wind lookup of the next aircraft issued before
// this one's arithmetic.
template <bool HI, typename VX>
__device__ __forceinline__ void pw_half(
    const RolloutParams& p, const RolloutArrays& a, const float* __restrict__ par,
    const float* __restrict__ rec, const __amdgpu_buffer_rsrc_t wrs, int s_z, int s_y, int s_x,
    int vbase, int bw, uint32_t todo, uint64_t actk, float zn_lane, VX& x, VX& y,
    float* __restrict__ accl,
    const v32f& xlo, const v32f& ylo, uint32_t done0, uint32_t& done, uint32_t& bad,
    uint32_t& sepbad, uint32_t& sepbad_lo, int& nhor) {
    if (!todo) return;
    const int base = HI ? 32 : 0;
    int ii = __builtin_ctz(todo);
    // two lookups alternate (the loop body twice), so that no lookup in
    // flight is copied from register to register
    PwTap ta = pw_issue<kPwRec>(p.cf, rec, wrs, s_z, s_y, s_x, vbase, bw, base + ii, ii, x, y), tb;
    PwNoise pend;
    pend.i = -1;
    // one aircraft: first the previous aircraft's population lookup (issued
    // after this aircraft's wind lookup, so waiting for it waits for nothing
    // still needed later), then the next aircraft's wind lookup (after the
    // last aircraft a repeat of this one's, unused), issued unconditionally
    // so that it stays ahead of this aircraft's arithmetic
#define PW_ONE(CUR, NXT)                                                                    \
    {                                                                                       \
        todo &= todo - 1u;                                                                  \
        pw_noise_add(pend, accl);                                                           \
        const int inext = todo ? __builtin_ctz(todo) : ii;                                  \
        NXT = pw_issue<kPwRec>(p.cf, rec, wrs, s_z, s_y, s_x, vbase, bw, base + inext, inext, x, y); \
        pw_aircraft<HI>(p, a, par, rec, CUR, base + ii, actk, zn_lane, x, y, accl, xlo, ylo,  \
                        done0, done, bad, sepbad, sepbad_lo, nhor, pend);                   \
        if (!todo) break;                                                                   \
        ii = inext;                                                                         \
    }
    while (true) {                                                 // uniform
        PW_ONE(ta, tb)
        PW_ONE(tb, ta)
    }
#undef PW_ONE
    pw_noise_add(pend, accl);
}

template <int NMAX>
__global__ void __launch_bounds__(64 * kPwWaves, pw_waves<NMAX>())
k_rollout_pw(const RolloutParams p, const RolloutArrays a, const float* __restrict__ acR,
             const float* __restrict__ Wt) {
    typedef typename PwHalf<pw_nb<NMAX>()>::t vBf;
    __shared__ __attribute__((aligned(16))) float par[NMAX * kPwPar];
    __shared__ __attribute__((aligned(16))) float recs[kPwWaves * NMAX * kPwRec];
    // per-world cost sums [wave][aircraft][lane] (LDS, so that the sum of
    // the aircraft at a uniform index needs no register indexing)
    __shared__ float accs[kPwWaves * NMAX * 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int N = p.N, S = p.S, H = p.H, M = p.M;
    const int nmb = (M + 63) >> 6;                      // 64-sample blocks per particle
    // workgroup -> (sample block, particles): workgroups go to the eight
    // XCDs in turn, so when the blocks divide 8, every XCD keeps to one block
    // of samples and to one contiguous range of particles, which it works
    // through in order: the workgroups resident on an XCD at a time hold
    // neighbouring particles, which after resampling (ancestors in
    // non-decreasing order) fly similar tracks through the same cells of the
    // fields, so their wind lookups share the XCD's L2; otherwise waves run
    // in (particle, block) order
    int mb;
    int64_t l64;
    if ((kXcds % nmb) == 0) {
        const int xcd = (int)(blockIdx.x % kXcds);
        const int64_t slot = blockIdx.x / kXcds;
        const int64_t per_xcd = gridDim.x / kXcds;               // workgroups per XCD
        mb = xcd % nmb;
        l64 = (((int64_t)(xcd / nmb) * per_xcd + slot) * kPwWaves) + wv;
    } else {
        const int64_t wave = (int64_t)blockIdx.x * kPwWaves + wv;
        mb = (int)(wave % nmb);
        l64 = wave / nmb;
    }
    const int64_t wave = l64 * nmb + mb;                // counter slot
    const bool wvalid = l64 < p.P;
    const int l = wvalid ? (int)l64 : 0;
    const int m = (wvalid ? mb : 0) * 64 + lane;
    const bool valid = wvalid && m < M;
    const RollConst<float>& q = p.cf;

    // per-aircraft parameters for the workgroup
    pw_fill_par(p, a, acR, par, tid);
    __syncthreads();

    // phase-1 lane state: aircraft j = lane (j < N), wind-independent
    const int j = lane < N ? lane : N - 1;
    const float* pj = par + j * kPwPar;
    PwAc sj = {pj[A_Z0], pj[A_V0], pj[A_CHI0], 0.f, 0.f, 0.f, 0.f};
    const int k0j = __float_as_int(pj[A_K0]);
    const bool actj = lane < N && k0j >= 0 && k0j < H;
    const bool arrj = a.kind[j] == 0;
    const float* ubj = (const float*)a.u + ((int64_t)l * N + j) * S * 3;
    float* recw = recs + wv * NMAX * kPwRec;

    // phase-2 state: one world per lane, all aircraft; aircraft i < 32 in
    // the lower halves, i >= 32 in the upper ones
    v32f xa, ya;
    vBf xb, yb;
    float* accl = accs + wv * NMAX * 64 + lane;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) accl[i * 64] = 0.f;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int ic = i < N ? i : 0;
        xa[i] = (float)a.states[6 * ic];
        ya[i] = (float)a.states[6 * ic + 1];
    }
#pragma unroll
    for (int i = 0; i < pw_nb<NMAX>(); ++i) {
        const int ic = i + 32 < N ? i + 32 : 0;
        xb[i] = (float)a.states[6 * ic];
        yb[i] = (float)a.states[6 * ic + 1];
    }
    uint32_t done_lo = 0u, done_hi = 0u, bad_lo = 0u, bad_hi = 0u, sep_lo = 0u, sep_hi = 0u;
    int nsim = 0, npair = 0, nhor = 0;

    // field of this world's sample in blocks of 64 samples,
    // Wt[b][g][64][c]: the corner (ix, iy, iz) of lane t of block b sits at
    // byte ((b G + g) 64 + t) 8, the other corners at uniform offsets
    constexpr int B = kWtBlockPw;
    const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Wt, (short)0, (int)wt_elems(M, p.G, B) * 8, 0x00020000);
    const int s_z = B * 8, s_y = p.nz * B * 8, s_x = p.ny * p.nz * B * 8;
    // lanes past the last sample (M not a multiple of 64) read sample M - 1
    // and write nothing
    const int mc = m < M ? m : M - 1;
    const int vbase = ((mc / B) * p.G * B + mc % B) * 8;

    int s_cur = -1, k_end = 0;
    for (int k = 0; k < H; ++k) {
        if (k == k_end) {   // uniform: the next control segment
            const int s = ++s_cur;
            k_end = ((s + 1) * H + S - 1) / S;
            sj.chidot = q.lo[0] + ubj[s * 3 + 0] * q.span[0];
            sj.vc = q.lo[1] + ubj[s * 3 + 1] * q.span[1];
            sj.zdot = q.lo[2] + ubj[s * 3 + 2] * q.span[2];
        }
        // ---- phase 1: aircraft j's wind-independent step (lane j) ----
        const bool act = actj && k >= k0j;
        const uint64_t actk = __ballot(act);
        wave_sync();   // the previous step's records were read
        const float zn_lane = pw_phase1(p, pj, k, k0j, k_end, arrj, act, sj,
                                        recw + lane * kPwRec, lane < N);
        wave_sync();   // records visible to every lane

        // ---- phase 2: every world runs the active aircraft in turn, the
        // wind lookup of the next one issued before this one's arithmetic ----
        const uint32_t d0lo = done_lo, d0hi = done_hi;
        pw_half<false>(p, a, par, recw, wrs, s_z, s_y, s_x, vbase, B, (uint32_t)actk, actk,
                       zn_lane, xa, ya, accl, xa, ya, d0lo, done_lo, bad_lo, sep_lo, sep_lo, nhor);
        if (NMAX > 32)
            pw_half<true>(p, a, par, recw, wrs, s_z, s_y, s_x, vbase, B, (uint32_t)(actk >> 32),
                          actk, zn_lane, xb, yb, accl, xa, ya, d0hi, done_hi, bad_hi, sep_hi,
                          sep_lo, nhor);
        {   // aircraft simulated this step and pair tests with both present
            const uint64_t pres = actk & ~(((uint64_t)d0hi << 32) | d0lo);
            const int np = __popcll(pres);
            nsim += np;
            npair += np * (np - 1) / 2;
        }
    }

    if (valid) {
        const uint64_t badm = ((uint64_t)(bad_hi | sep_hi) << 32) | (bad_lo | sep_lo);
        for (int i = 0; i < N; ++i) {
            const int k0 = a.k_active[i];
            const float ai = accl[i * 64];
            const double cost = (k0 >= 0 && k0 < H) ? (double)ai / (double)(H - k0) : 0.0;
            const int64_t o = ((int64_t)m * p.P + l) * N + i;
            a.cost[o] = cost;
            a.feas[o] = ((badm >> i) & 1ull) ? 0 : 1;
        }
    }
    if (a.steps) {
        int cnt = valid ? nsim : 0;
        int cp = valid ? npair : 0;
        for (int off = 32; off > 0; off >>= 1) {
            cnt += __shfl_xor(cnt, off);
            cp += __shfl_xor(cp, off);
        }
        if (lane == 0) {
            const unsigned slot = (unsigned)(wave & (kStepSlots - 1));
            if (cnt) atomicAdd(&a.steps[slot], (unsigned long long)cnt);
            if (cp) atomicAdd(&a.steps[kStepSlots + slot], (unsigned long long)cp);
        }
    }
    if (a.steps_h) {   // nhor is wave-uniform: one count per valid lane (world)
        const unsigned long long nv = (unsigned long long)__popcll(__ballot(valid));
        if (lane == 0 && nhor && nv)
            atomicAdd(&a.steps_h[(unsigned)(wave & (kStepSlots - 1))],
                      (unsigned long long)nhor * nv);
    }
}

bool rollout_pw_supported(int N, int prec) { return prec == 1 && N >= 1 && N <= 64; }

template <int NMAX>
static hipError_t launch_pw_n(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              const void* Wt, hipStream_t st) {
    const int nmb = (p.M + 63) / 64;
    int64_t blocks;
    if ((kXcds % nmb) == 0) {
        // whole rounds of the eight XCDs: each holds ceil(P / (4 * 8 / nmb))
        // workgroups of 4 particles of its sample block
        const int64_t per_round = (int64_t)kPwWaves * (kXcds / nmb);
        blocks = (((int64_t)p.P + per_round - 1) / per_round) * kXcds;
    } else {
        blocks = ((int64_t)p.P * nmb + kPwWaves - 1) / kPwWaves;
    }
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_rollout_pw<NMAX>), dim3((unsigned)blocks), dim3(64 * kPwWaves), 0, st,
                       p, a, (const float*)acR, (const float*)Wt);
    return hipGetLastError();
}

// Wt: the fields in the sample-interleaved layout [G][M][2] (FP32).
hipError_t launch_rollout_pw(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                             const void* Wt, hipStream_t st) {
    if (!rollout_pw_supported(p.N, 1) || p.w_kstride != 0) return hipErrorInvalidValue;
    if (p.P <= 0 || p.M <= 0) return hipSuccess;
    if (wt_elems(p.M, p.G, kWtBlockPw) * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    if (p.N <= 32) return launch_pw_n<32>(p, a, acR, Wt, st);
    if (p.N <= 40) return launch_pw_n<40>(p, a, acR, Wt, st);
    if (p.N <= 48) return launch_pw_n<48>(p, a, acR, Wt, st);
    return launch_pw_n<64>(p, a, acR, Wt, st);
}

}  // namespace smc
