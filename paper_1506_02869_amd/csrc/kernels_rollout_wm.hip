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

// PC: the paper's per-step thrust / flight-path angle / bank controls (Sec.
// "Trajectory Planning and Disturbance Realisations", eq. hor) in place of
// the kinematic segment controls.
template <typename R, int NMAX, bool PC>
__global__ void __launch_bounds__(256, (wm_waves<R, NMAX>()))
k_rollout_wm(const RolloutParams p, const RolloutArrays a, const R* __restrict__ acR) {
    constexpr bool kTV = false;
    constexpr bool kPC = PC;
    extern __shared__ unsigned char smem_raw[];
    R* uc = reinterpret_cast<R*>(smem_raw);   // [N][3][blockDim.x]
    const int tid = threadIdx.x;
    const int bd = blockDim.x;
    const int64_t world = (int64_t)blockIdx.x * bd + tid;
    const unsigned slot = blockIdx.x;
#include "rollout_wm_body.inc"
}

// 256 lanes per block in FP32, 128 in FP64: the staged controls take
// NMAX * 3 * block * sizeof(R) bytes of LDS (one NMAX x 3 x 64 slice per
// wave; 60 KB at NMAX = 20 either way).
template <typename R, int NMAX>
static hipError_t launch_wm_n(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              hipStream_t st) {
    const int block = sizeof(R) == 4 ? 256 : 128;
    const int64_t nworld = (int64_t)p.P * p.M;
    const unsigned blocks = (unsigned)((nworld + block - 1) / block);
    const size_t lds = (size_t)NMAX * 3 * block * sizeof(R);
    if (p.control_model == 1)
        hipLaunchKernelGGL((k_rollout_wm<R, NMAX, true>), dim3(blocks), dim3(block), lds, st, p,
                           a, (const R*)acR);
    else
        hipLaunchKernelGGL((k_rollout_wm<R, NMAX, false>), dim3(blocks), dim3(block), lds, st, p,
                           a, (const R*)acR);
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
    if (p.N <= 16) return launch_wm_n<R, 16>(p, a, acR, st);
    return launch_wm_n<R, 20>(p, a, acR, st);
}

bool rollout_wm_supported(int N) { return N >= 1 && N <= kWorldLaneMaxN; }

hipError_t launch_rollout_wm(int prec, const RolloutParams& p, const RolloutArrays& a,
                             const void* acR, hipStream_t st) {
    if (!rollout_wm_supported(p.N)) return hipErrorInvalidValue;
    if (p.P <= 0 || p.M <= 0) return hipSuccess;
    return prec == 0 ? launch_wm_t<double>(p, a, acR, st) : launch_wm_t<float>(p, a, acR, st);
}

}  // namespace smc
