// Pieces shared by the two rollout layouts whose lanes are wind samples of
// the same particles (particle-per-wave: 64 samples of one particle;
// particle tile: 16 samples of each of 4 particles): the per-aircraft
// parameter rows, the wind-independent part of a step (computed once per
// particle and aircraft), its record, and the wind lookup of one aircraft.
//
// In the model the wind moves an aircraft only horizontally (x, y): its
// airspeed ramp, climb, heading, bank, density, drag, thrust, fuel flow and
// mass, with them every unary constraint, the altitude-dependent cost
// elements and the altitude itself are the same in all wind samples of a
// particle until the aircraft lands in one of them (paper, Sec.
// "Trajectory Planning", eq. hor; Sec. "Constraint Handling"; eq. TO_init;
// Sec. "Particle Costing", "Noise Pollution Reduction").
#pragma once

#include "rollout_math.h"

namespace smc {

namespace {

// one float per aircraft of the world, in two register vectors of at most
// 32 (aircraft 0..31 and 32..NMAX-1), each indexed at a uniform index
typedef float v32f __attribute__((ext_vector_type(32)));
template <int NB> struct PwHalf { typedef float t __attribute__((ext_vector_type(NB))); };
template <int NMAX>
constexpr int pw_nb() { return NMAX <= 32 ? 8 : NMAX - 32; }

constexpr int kPwWaves = 4;     // wavefronts per workgroup (independent)
constexpr int kXcds = 8;        // accelerator complex dies; workgroups are dealt to them in turn
constexpr int kPwRec = 12;      // floats of an aircraft-step record
constexpr int kPwPar = 24;      // floats of an aircraft parameter row

// record fields (phase 1 -> phase 2)
enum : int {
    R_VX = 0, R_VY, R_ZN, R_CHIN, R_GZ, R_TZ, R_UDEP, R_IVT, R_NA, R_FUEL, R_FLAGS
};
// parameter row fields (LDS, whole workgroup)
enum : int {
    A_SW = 0, A_CD0, A_CD2, A_CF, A_CFV, A_TMAX, A_MEMP, A_TPHI, A_SGAM, A_THF, A_ZT, A_VD,
    A_DTMA, A_CSPD, A_CFUEL, A_M0, A_D0, A_Z0, A_V0, A_CHI0, A_K0
};
constexpr uint32_t F_VIOL = 1u, F_LANDOK = 2u, F_DEP = 4u;

// waves per SIMD the register budget is set for: the world state takes
// 2 NMAX VGPRs (x and y of every aircraft), the cost sums NMAX x 64 floats
// of LDS per wave
template <int NMAX>
constexpr int pw_waves() { return NMAX <= 48 ? 2 : 1; }

}  // namespace

typedef float F2 __attribute__((ext_vector_type(2)));

// The wind lookup of one aircraft in every world of the wave, issued one
// aircraft ahead of its use so that the loads overlap the previous
// aircraft's arithmetic: the position, the cell fractions and the eight
// corners (x, y components) of this lane's sample.
struct PwTap {
    float xi, yi, tx, ty, tz;
    F2 c[8];
};

// A population lookup in flight: its two rows, the cell fractions, the
// weight it enters the cost with (0 when the aircraft is above the noise
// altitude, has landed or had landed) and the aircraft (-1: none).  It is
// consumed one aircraft later, so that waiting for it never waits for the
// wind lookup issued after it.
struct PwNoise {
    F2 p0, p1;
    float ux, uy, w;
    int i;
};

__device__ __forceinline__ void pw_noise_add(const PwNoise& n, float* __restrict__ accl) {
    if (n.i < 0) return;                                            // uniform
    const float pd = (1.f - n.ux) * (1.f - n.uy) * n.p0.x + n.ux * (1.f - n.uy) * n.p0.y +
                     (1.f - n.ux) * n.uy * n.p1.x + n.ux * n.uy * n.p1.y;
    accl[n.i * 64] += n.w * pd;
}

// Issue the lookup of aircraft i (its position before this step's update;
// the altitude cell and fraction come from its phase-1 record); x, y: the
// half holding aircraft i, at index ii; bw: the samples per block of the
// fields (grid point g of the lane's block starts at byte vbase + 8 g bw);
// RS: floats between consecutive aircraft's records.
template <int RS, typename V>
__device__ __forceinline__ PwTap pw_issue(const RollConst<float>& q, const float* __restrict__ rec,
                                          const __amdgpu_buffer_rsrc_t wrs, int s_z, int s_y,
                                          int s_x, int vbase, int bw, int i, int ii, const V& x,
                                          const V& y) {
    PwTap t;
    t.xi = x[ii];
    t.yi = y[ii];
    const float2 zc = *reinterpret_cast<const float2*>(rec + i * RS + R_GZ);   // cell, fraction
    const float fx = clampr(m_fma(t.xi, q.inv_hx, q.ox), 0.f, q.fnx1);
    const float fy = clampr(m_fma(t.yi, q.inv_hy, q.oy), 0.f, q.fny1);
    const float flx = m_floor(clampr(fx, 0.f, q.fnx2));
    const float fly = m_floor(clampr(fy, 0.f, q.fny2));
    t.tx = fx - flx;
    t.ty = fy - fly;
    t.tz = zc.y;
    const int g = (int)m_fma(m_fma(flx, q.fny, fly), q.fnz, zc.x);
    // (a 24-bit multiply: g < 2^24 and 8 bw < 2^24, the product is a byte
    // offset inside the fields, below 2^31)
    const int vo = (int)__umul24((unsigned)g, (unsigned)(bw * 8)) + vbase;
    const int off[8] = {0, s_z, s_y, s_y + s_z, s_x, s_x + s_z, s_x + s_y, s_x + s_y + s_z};
#pragma unroll
    for (int c = 0; c < 8; ++c)
        t.c[c] = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(wrs, vo, off[c], 0));
    return t;
}


// Per-aircraft parameter rows of a workgroup (host constants from acR, the
// initial state, the fuel element's per-step coefficient); thread tid < N
// writes row tid.
__device__ __forceinline__ void pw_fill_par(const RolloutParams& p, const RolloutArrays& a,
                                            const float* __restrict__ acR, float* par, int tid) {
    const int N = p.N;
    if (tid >= N) return;
    const int i = tid;
    const float* c = acR + kAcR * i;
    float* r = par + i * kPwPar;
#pragma unroll
    for (int f = 0; f < 14; ++f) r[f] = c[f];
    const double* ac = a.acpar + 9 * i;
    const double wf = a.kind[i] == 0 ? p.w[2] : p.w[4];
    r[A_CFUEL] = (float)((1.0 - p.w[7] - p.w[8]) * wf /
                         (p.dt * ac[5] * (ac[3] * (1.0 + p.vmax / ac[4]))));
    const double* st = a.states + 6 * i;
    r[A_M0] = (float)st[5];
    r[A_D0] = fabsf(c[10] - (float)st[2]);
    r[A_Z0] = (float)st[2];
    r[A_V0] = (float)st[3];
    r[A_CHI0] = (float)st[4];
    r[A_K0] = __int_as_float(a.k_active[i]);
}

// The wind-independent state of one (particle, aircraft) and its segment
// controls.
struct PwAc {
    float z, v, chi, burn, chidot, vc, zdot;
};

// The wind-independent step k of one (particle, aircraft): writes the
// record read by every sample's lane (velocity over ground without wind,
// new altitude and heading, the altitude cell and fraction of the wind
// lookup, the departure altitude and speed elements, 1 / (v t_norm), the
// noise altitude factor, the fuel element's share, the flags), returns the
// new altitude, and advances the state when the aircraft is active.
__device__ __forceinline__ float pw_phase1(const RolloutParams& p, const float* __restrict__ pj,
                                           int k, int k0j, int k_end, bool arrj, bool act,
                                           PwAc& s, float* __restrict__ rec_out, bool write) {
    typedef Ops<float> O;
    const RollConst<float>& q = p.cf;
    const float chidot = s.chidot, vc = s.vc, zdot = s.zdot;
    const float zj = s.z, vj = s.v, chij = s.chi, burnj = s.burn;
    const float inv_rem = O::rcp((float)(k_end - k));
    const float sg = zdot * O::rcp(vj);
    const float cg = O::sqrt(1.f - sg * sg);
    const float tphi = vj * chidot * q.inv_g;
    const float zc = clampr(zj, 0.f, 11000.f);
    const float rho = q.rho0 * O::pow_pos(1.f - q.isa_c * zc, q.isa_e);
    const float qS = 0.5f * rho * vj * vj * pj[A_SW];
    const float mass = pj[A_M0] - burnj;
    // only C_L^2 = (m g / (q S))^2 (1 + tan^2 phi) enters the drag
    const float wq = O::div(mass * q.g0, qS);
    const float D = qS * (pj[A_CD0] + pj[A_CD2] * (wq * wq * (1.f + tphi * tphi)));
    const float dv = (vc - vj) * inv_rem;
    const float vn = vj + dv;
    const float T = mass * (dv * q.inv_dt + q.g0 * sg) + D;
    const float fuel = m_fma(vj, pj[A_CFV], pj[A_CF]) * m_max(T, 0.f);
    float sc, cc;
    O::sincos(chij, &sc, &cc);
    const float vcg = vj * cg;
    const float zn = m_fma(q.dt, zdot, zj);
    const float chin = m_fma(q.dt, chidot, chij);
    const float mn = mass - fuel;
    const bool viol = (T > pj[A_TMAX]) | (m_abs(tphi) >= pj[A_TPHI]) |
                      (m_abs(sg) > pj[A_SGAM]) | (zn < q.zmin) | (zn > q.zmax) |
                      (vn < q.vmin) | (vn > q.vmax) | (mn < pj[A_MEMP]);
    // wind cell along z at the current altitude (shared by the worlds)
    const float fz = clampr(zj * q.inv_hz, 0.f, q.fnz1);
    const float flz = m_floor(clampr(fz, 0.f, q.fnz2));
    const float ivt = q.inv_tnorm * O::rcp(maxr(vn, q.vmin));
    float udep = 0.f;
    bool landok = false;
    if (arrj) {
        landok = (m_abs(wrap_angle<float>(chin - Consts<float>::pi)) <= q.p_chi) &
                 (vn <= q.p_vs);
    } else {
        const float span = q.zdm_dt * (float)max(k + 1 - k0j, 1);
        const float sup = pj[A_D0] + span;
        const float inf = m_max(pj[A_D0] - span, 0.f);
        const float alt = clampr(O::div(m_abs(pj[A_ZT] - zn) - inf, sup - inf), 0.f, 1.f);
        udep = q.c_alt * alt + pj[A_CSPD] * m_abs(vn - pj[A_VD]);
    }
    float na = 0.f;
    if (p.use_noise) {
        const float za = zn * q.inv_Ac;
        na = q.a_noise * m_max(1.f - za * za, 0.f);
    }
    const uint32_t fl = (viol ? F_VIOL : 0u) | (landok ? F_LANDOK : 0u) |
                        (arrj ? 0u : F_DEP);
    if (write) {
        float4* r4 = reinterpret_cast<float4*>(rec_out);
        r4[0] = make_float4(vcg * cc, vcg * sc, zn, chin);
        r4[1] = make_float4(flz, fz - flz, udep, ivt);
        r4[2] = make_float4(na, pj[A_CFUEL] * fuel, __uint_as_float(fl), 0.f);
    }
    // the heading is kept in [-pi, pi) (it enters only through sin, cos and
    // wrapped differences), so its rounding stays that of an angle near pi
    // however far the aircraft turns
    if (act) { s.z = zn; s.v = vn; s.chi = wrap_angle<float>(chin); s.burn = burnj + fuel; }
    return zn;
}

}  // namespace smc
