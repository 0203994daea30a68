// Rollout, particle-tile layout (FP32, up to 64 aircraft): a wavefront holds
// 4 particles x 16 wind samples, one world (particle, sample) per lane, and
// a workgroup consecutive particles of one block of 16 samples.
//
// The per-step arithmetic is that of the other layouts (paper, Sec.
// "Trajectory Planning", eq. hor; Sec. "Constraint Handling"; eq. TO_init;
// Sec. "Particle Costing", "Noise Pollution Reduction"; eq. avoidance).  As
// in the particle-per-wave layout, each aircraft's wind-independent step is
// computed once per particle (four passes of the wave's lanes, one per
// particle, lane j = aircraft j) and read by the particle's 16 sample lanes
// from LDS; only pairs inside the vertical separation get the horizontal
// test (exact: the altitudes do not depend on the wind).  What the tile
// changes: a workgroup (8 wavefronts up to 40 aircraft, 32 particles; 4
// above) reads the fields of 16 samples only, so with the blocks of samples
// dealt one per XCD the lookups of every workgroup on an XCD fall in one
// block of the fields, which its L2 holds (G x 16 x 8 bytes: 4.2 MB on a
// 64 x 64 x 8 grid), where 64 samples per wavefront (17 MB per block)
// missed the L2 on large grids.  The fields are stored block by block, so
// that a block is one contiguous range: interleaving all M samples per grid
// point would leave an XCD's lines at a stride of 8 M bytes, which crowds
// them into a fraction of the L2's sets and channels.
//
// Vertical candidates: after the four passes of a step, for every particle
// and aircraft i, the mask of aircraft j < i active at the step with
// |z_j - z_i| < sep_v (each lane compares its aircraft with every other),
// kept per particle and as the union over the wavefront's four particles
// (the uniform loop of the pair tests; each lane tests only its particle's
// candidates).
#include "rollout_pw_common.h"

namespace smc {

namespace {

constexpr int kPtP = 4;         // particles per wavefront
constexpr int kPtS = 16;        // wind samples per particle in a wavefront
static_assert(kPtS == kWtBlockPt, "the fields come in blocks of one wavefront's samples");

// waves per SIMD the register budget is set for (as the particle-per-wave
// layout: x and y of every aircraft in registers, cost sums in LDS)
template <int NMAX>
constexpr int pt_waves() { return NMAX <= 40 ? 2 : 1; }
// wavefronts per workgroup: a wavefront takes about NMAX x 480 bytes of LDS
// (records, candidate masks, cost sums), so up to 40 aircraft one
// workgroup of 8 wavefronts fills a CU (157 KB of 160), above that 4
template <int NMAX>
constexpr int pt_wgw() { return NMAX <= 40 ? 8 : 4; }

}  // namespace

// One aircraft of phase 2 in every world of the wave (aircraft i, index ii
// = i - 32 HI into the upper halves).  rec: the records of the lane's
// particle; dep: aircraft i is a departure (uniform); mine: the lane's
// particle's vertical candidates for i; cand: their union over the wave.
template <bool HI, typename VX>
__device__ __forceinline__ void pt_aircraft(
    const RolloutParams& p, const RolloutArrays& a, const float* __restrict__ par,
    const float* __restrict__ rec, const PwTap& w, int i, bool dep, uint64_t mine,
    uint64_t cand, VX& x, VX& y, float* __restrict__ accl, const v32f& xlo, const v32f& ylo,
    uint32_t done0, uint32_t& done, uint32_t& bad, uint32_t& sepbad, uint32_t& sepbad_lo,
    int& nhor, PwNoise& noise) {
    typedef Ops<float> O;
    const RollConst<float>& q = p.cf;
    const int ii = HI ? i - 32 : i;
    const uint32_t bit = 1u << ii;
    const float4* r4 = reinterpret_cast<const float4*>(rec + i * kPwRec);
    const float4 ra = r4[0], rb = r4[1], rc = r4[2];
    const uint32_t flags = __float_as_uint(rc.z);   // per particle: per lane
    const float na = rc.x;
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
    if (!dep) {               // arrival (uniform)
        // both forms, then a select: no divergent branch
        // sin|theta| = |y| / r: the ratio |theta| / sin|theta| without the sine
        const float r_arc = tha * r * O::rcp(m_max(m_abs(yn), 1e-6f * r));
        const float r_small = 1.f + tha * tha * (1.f / 6.f);
        const float ratio = tha > 1e-4f ? r_arc : r_small;
        const float s_arc = r * ratio;
        const float beta = O::atan2_xpos(zn, s_arc);                 // s_arc >= 0
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
    // uniform: some particle of the wave is below the noise altitude
    if (p.use_noise && __ballot(na != 0.f) != 0ull) {
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

    // separation against the aircraft already moved this step that are
    // vertical candidates of the lane's particle: every lane tests the
    // wave's union of candidates and keeps a mask of the horizontal
    // conflicts, restricted to its own particle's candidates at the end.
    // d2 < sep_h2 is read off the sign of the rounded difference, which
    // is negative exactly then (a difference of finite floats rounds to
    // zero only when they are equal, and keeps its sign otherwise).
    nhor += __popcll(mine);
    uint32_t c_lo = (uint32_t)cand, h_lo = 0u;
    while (c_lo) {                                                  // uniform
        const int jj = __builtin_ctz(c_lo);
        c_lo &= c_lo - 1u;
        const float dx = xs - xlo[jj], dy = ys - ylo[jj];
        h_lo |= (__float_as_uint(dx * dx + dy * dy - q.sep_h2) >> 31) << jj;
    }
    h_lo &= (uint32_t)mine;
    if (HI) {
        uint32_t c_hi = (uint32_t)(cand >> 32), h_hi = 0u;
        while (c_hi) {                                              // uniform
            const int jj = __builtin_ctz(c_hi);
            c_hi &= c_hi - 1u;
            const float dx = xs - x[jj], dy = ys - y[jj];
            h_hi |= (__float_as_uint(dx * dx + dy * dy - q.sep_h2) >> 31) << jj;
        }
        h_hi &= (uint32_t)(mine >> 32);
        sepbad |= (h_lo | h_hi) != 0u ? bit | h_hi : 0u;
    } else {
        sepbad |= h_lo != 0u ? bit : 0u;
    }
    sepbad_lo |= h_lo;
}

// Phase 2 over the active aircraft of one half (bits of `todo`, aircraft
// index base + bit), the wind lookup of the next aircraft issued before
// this one's arithmetic; cm: this lane's particle's candidate masks, cu:
// the wave's union masks (LDS).
template <bool HI, typename VX>
__device__ __forceinline__ void pt_half(
    const RolloutParams& p, const RolloutArrays& a, const float* __restrict__ par,
    const float* __restrict__ rec, const uint64_t* __restrict__ cm,
    const uint64_t* __restrict__ cu, uint64_t depm, const __amdgpu_buffer_rsrc_t wrs, int s_z,
    int s_y, int s_x, int vbase, int bw, uint32_t todo, VX& x, VX& y, float* __restrict__ accl,
    const v32f& xlo, const v32f& ylo, uint32_t done0, uint32_t& done, uint32_t& bad,
    uint32_t& sepbad, uint32_t& sepbad_lo, int& nhor) {
    if (!todo) return;
    const int base = HI ? 32 : 0;
    int ii = __builtin_ctz(todo);
    PwTap ta = pw_issue<kPwRec>(p.cf, rec, wrs, s_z, s_y, s_x, vbase, bw, base + ii, ii, x, y), tb;
    PwNoise pend;
    pend.i = -1;
#define PT_ONE(CUR, NXT)                                                                     \
    {                                                                                        \
        todo &= todo - 1u;                                                                   \
        pw_noise_add(pend, accl);                                                            \
        const int inext = todo ? __builtin_ctz(todo) : ii;                                   \
        NXT = pw_issue<kPwRec>(p.cf, rec, wrs, s_z, s_y, s_x, vbase, bw, base + inext, inext, x, y);  \
        const int i = base + ii;                                                             \
        const uint64_t un = __builtin_amdgcn_readfirstlane((uint32_t)cu[i]) |                \
                            ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(cu[i] >> 32)) << 32); \
        pt_aircraft<HI>(p, a, par, rec, CUR, i, ((depm >> i) & 1ull) != 0ull, cm[i], un, x, y, \
                        accl, xlo, ylo, done0, done, bad, sepbad, sepbad_lo, nhor, pend);    \
        if (!todo) break;                                                                    \
        ii = inext;                                                                          \
    }
    while (true) {                                                  // uniform
        PT_ONE(ta, tb)
        PT_ONE(tb, ta)
    }
#undef PT_ONE
    pw_noise_add(pend, accl);
}

template <int NMAX>
__global__ void __launch_bounds__(64 * pt_wgw<NMAX>(), pt_waves<NMAX>())
k_rollout_pt(const RolloutParams p, const RolloutArrays a, const float* __restrict__ acR,
             const float* __restrict__ Wt) {
    typedef typename PwHalf<pw_nb<NMAX>()>::t vBf;
    constexpr int kPtWaves = pt_wgw<NMAX>();
    constexpr int kPtPart = kPtP * kPtWaves;   // particles per workgroup
    __shared__ __attribute__((aligned(16))) float par[NMAX * kPwPar];
    // per-particle strides padded so that the four particles' records (and
    // masks) of one aircraft, read together by the wave, fall in distinct
    // LDS banks
    constexpr int kRecStride = NMAX * kPwRec + 4;       // floats
    constexpr int kMaskStride = NMAX + 1;                // 64-bit words
    __shared__ __attribute__((aligned(16))) float recs[kPtWaves * kPtP * kRecStride];
    __shared__ uint64_t cmask[kPtWaves * kPtP * kMaskStride];   // per particle
    __shared__ uint64_t cunion[kPtWaves * NMAX];         // union over the wave's particles
    __shared__ float accs[kPtWaves * NMAX * 64];         // [wave][aircraft][lane]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int pl = lane / kPtS, ms = lane % kPtS;
    const int N = p.N, S = p.S, H = p.H, M = p.M;
    const RollConst<float>& q = p.cf;
    const int nmb = (M + kPtS - 1) / kPtS;              // 16-sample blocks
    // workgroup -> (sample block, 16 particles): when the blocks divide the
    // eight XCDs (to which workgroups are dealt in turn), every XCD keeps to
    // one block and to one contiguous range of particles, worked through in
    // order; otherwise (block, particles) in launch order
    int mb;
    int64_t pg;
    if ((kXcds % nmb) == 0) {
        const int xcd = (int)(blockIdx.x % kXcds);
        const int64_t slot = blockIdx.x / kXcds;
        const int64_t per_xcd = gridDim.x / kXcds;
        mb = xcd % nmb;
        pg = (int64_t)(xcd / nmb) * per_xcd + slot;
    } else {
        mb = (int)(blockIdx.x % nmb);
        pg = blockIdx.x / nmb;
    }
    const int64_t l0 = pg * kPtPart + (int64_t)wv * kPtP;   // the wave's first particle
    const int64_t l64 = l0 + pl;
    const bool lvalid = l64 < p.P;
    const int l = lvalid ? (int)l64 : p.P - 1;
    const int m = mb * kPtS + ms;
    const bool valid = lvalid && m < M;

    pw_fill_par(p, a, acR, par, tid);
    __syncthreads();

    // phase-1 lanes: pass r computes the wave's particle r, lane j = aircraft j
    const int j = lane < N ? lane : N - 1;
    const float* pj = par + j * kPwPar;
    const int k0j = __float_as_int(pj[A_K0]);
    const bool actj = lane < N && k0j >= 0 && k0j < H;
    const bool arrj = a.kind[j] == 0;
    PwAc s1[kPtP];
    const float* ubr[kPtP];
#pragma unroll
    for (int r = 0; r < kPtP; ++r) {
        s1[r] = PwAc{pj[A_Z0], pj[A_V0], pj[A_CHI0], 0.f, 0.f, 0.f, 0.f};
        const int64_t lr = l0 + r < p.P ? l0 + r : p.P - 1;
        ubr[r] = (const float*)a.u + (lr * N + j) * S * 3;
    }
    // departures (uniform)
    uint64_t depm = 0ull;
    for (int i = 0; i < N; ++i)
        if (a.kind[i] != 0) depm |= 1ull << i;
    float* recw = recs + wv * kPtP * kRecStride;             // the wave's records
    const float* recl = recw + pl * kRecStride;              // the lane's particle's
    uint64_t* cmw = cmask + wv * kPtP * kMaskStride;
    const uint64_t* cml = cmw + pl * kMaskStride;
    uint64_t* cuw = cunion + wv * NMAX;

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

    // fields in blocks of kPtS samples, Wt[b][g][kPtS][c]: the corner
    // (ix, iy, iz) of sample m = b kPtS + t sits at byte ((b G + g) kPtS +
    // t) 8, the other corners at uniform offsets; lanes past the last
    // sample read sample M - 1 and write nothing
    const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Wt, (short)0, (int)wt_elems(M, p.G, kPtS) * 8, 0x00020000);
    const int s_z = kPtS * 8, s_y = p.nz * kPtS * 8, s_x = p.ny * p.nz * kPtS * 8;
    const int mc = m < M ? m : M - 1;
    const int vbase = ((mc / kPtS) * p.G * kPtS + mc % kPtS) * 8;

    int s_cur = -1, k_end = 0;
    for (int k = 0; k < H; ++k) {
        if (k == k_end) {   // uniform: the next control segment
            const int s = ++s_cur;
            k_end = ((s + 1) * H + S - 1) / S;
#pragma unroll
            for (int r = 0; r < kPtP; ++r) {
                s1[r].chidot = q.lo[0] + ubr[r][s * 3 + 0] * q.span[0];
                s1[r].vc = q.lo[1] + ubr[r][s * 3 + 1] * q.span[1];
                s1[r].zdot = q.lo[2] + ubr[r][s * 3 + 2] * q.span[2];
            }
        }
        // ---- phase 1: the wind-independent step of every (particle,
        // aircraft), then the vertical candidates ----
        const bool act = actj && k >= k0j;
        const uint64_t actk = __ballot(act);
        wave_sync();   // the previous step's records and masks were read
        uint64_t un = 0ull;
#pragma unroll
        for (int r = 0; r < kPtP; ++r) {
            const float zr = pw_phase1(p, pj, k, k0j, k_end, arrj, act, s1[r],
                                       recw + r * kRecStride + lane * kPwRec, lane < N);
            // lane i's mask of aircraft j < i, active at this step, with
            // |z_j - z_i| < sep_v: every lane compares its altitude with
            // aircraft i's in turn and sets bit i (|z_j - z_i| is symmetric)
            uint32_t mlo = 0u, mhi = 0u;
            uint64_t todo = actk;
            while (todo) {                                          // uniform
                const int i = __builtin_ctzll(todo);
                todo &= todo - 1ull;
                const float zi = __builtin_bit_cast(
                    float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, zr), i));
                // |z_j - z_i| < sep_v from the sign of the difference
                const uint32_t close = __float_as_uint(m_abs(zr - zi) - q.sep_v) >> 31;
                if (i < 32) mlo |= close << i;                      // uniform
                else mhi |= close << (i - 32);
            }
            const uint64_t mr = act ? (((uint64_t)mhi << 32) | mlo) & actk &
                                          ((1ull << lane) - 1ull)
                                    : 0ull;
            un |= mr;
            if (lane < N) cmw[r * kMaskStride + lane] = mr;
        }
        if (lane < N) cuw[lane] = un;
        wave_sync();   // records and masks visible to every lane

        // ---- phase 2: every world runs the active aircraft in turn ----
        const uint32_t d0lo = done_lo, d0hi = done_hi;
        pt_half<false>(p, a, par, recl, cml, cuw, depm, wrs, s_z, s_y, s_x, vbase, kPtS,
                       (uint32_t)actk, xa, ya, accl, xa, ya, d0lo, done_lo, bad_lo, sep_lo, sep_lo,
                       nhor);
        if (NMAX > 32)
            pt_half<true>(p, a, par, recl, cml, cuw, depm, wrs, s_z, s_y, s_x, vbase, kPtS,
                          (uint32_t)(actk >> 32), xb, yb, accl, xa, ya, d0hi, done_hi, bad_hi,
                          sep_hi, sep_lo, nhor);
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
    const unsigned slot = blockIdx.x & (kStepSlots - 1);
    if (a.steps) {
        int cnt = valid ? nsim : 0;
        int cp = valid ? npair : 0;
        for (int off = 32; off > 0; off >>= 1) {
            cnt += __shfl_xor(cnt, off);
            cp += __shfl_xor(cp, off);
        }
        if (lane == 0) {
            if (cnt) atomicAdd(&a.steps[slot], (unsigned long long)cnt);
            if (cp) atomicAdd(&a.steps[kStepSlots + slot], (unsigned long long)cp);
        }
    }
    if (a.steps_h) {   // horizontal tests of the lane's world
        int nh = valid ? nhor : 0;
        for (int off = 32; off > 0; off >>= 1) nh += __shfl_xor(nh, off);
        if (lane == 0 && nh) atomicAdd(&a.steps_h[slot], (unsigned long long)nh);
    }
}

bool rollout_pt_supported(int N, int prec) { return prec == 1 && N >= 1 && N <= 64; }

template <int NMAX>
static hipError_t launch_pt_n(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              const void* Wt, hipStream_t st) {
    constexpr int kPtPart = kPtP * pt_wgw<NMAX>();
    const int nmb = (p.M + kPtS - 1) / kPtS;
    const int64_t groups = ((int64_t)p.P + kPtPart - 1) / kPtPart;
    int64_t blocks;
    if ((kXcds % nmb) == 0) {
        // whole rounds of the eight XCDs: each takes one block of samples and
        // ceil(groups / (8 / nmb)) groups of 16 particles
        const int64_t per = kXcds / nmb;
        blocks = ((groups + per - 1) / per) * kXcds;
    } else {
        blocks = groups * nmb;
    }
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_rollout_pt<NMAX>), dim3((unsigned)blocks), dim3(64 * pt_wgw<NMAX>()), 0, st,
                       p, a, (const float*)acR, (const float*)Wt);
    return hipGetLastError();
}

// Wt: the fields in the sample-interleaved layout [G][M][2] (FP32).
hipError_t launch_rollout_pt(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                             const void* Wt, hipStream_t st) {
    if (!rollout_pt_supported(p.N, 1) || p.w_kstride != 0) return hipErrorInvalidValue;
    if (p.P <= 0 || p.M <= 0) return hipSuccess;
    if (wt_elems(p.M, p.G, kPtS) * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    if (p.N <= 32) return launch_pt_n<32>(p, a, acR, Wt, st);
    if (p.N <= 40) return launch_pt_n<40>(p, a, acR, Wt, st);
    if (p.N <= 48) return launch_pt_n<48>(p, a, acR, Wt, st);
    return launch_pt_n<64>(p, a, acR, Wt, st);
}

}  // namespace smc
