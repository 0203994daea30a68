// World-per-lane rollout under the paper's time-correlated wind (Sec. "Wind
// Model": one field per step of the horizon from the linear Gaussian
// model).  The per-step arithmetic is the world-per-lane body of the static
// model; only the field a step reads changes: step k reads the fields that
// start k * p.w_kstride reals into W ([H][M][G][2]).  A separate kernel
// family, so that the static kernels carry no per-step field offset.
#include "rollout_math.h"

namespace smc {

template <typename R, int NMAX>
__global__ void __launch_bounds__(256, (wm_waves<R, NMAX>()))
k_rollout_wm_tv(const RolloutParams p, const RolloutArrays a, const R* __restrict__ acR) {
    constexpr bool kTV = true;
    constexpr bool kPC = false;
    extern __shared__ unsigned char smem_raw[];
    R* uc = reinterpret_cast<R*>(smem_raw);   // [N][3][blockDim.x]
    const int tid = threadIdx.x;
    const int bd = blockDim.x;
    // Workgroups are dispatched round-robin over the 8 XCDs, each with its
    // own L2; every step reads fresh fields, so each XCD takes a contiguous
    // range of worlds (whole wind samples) and a step's field of a sample is
    // fetched into one L2.  Block b runs on XCD b % 8 as its (b / 8)-th
    // block; the map onto logical blocks is a bijection for any grid size.
    const unsigned lb = [] {
        const unsigned nb = gridDim.x, b = blockIdx.x;
        const unsigned q = nb / 8, r = nb % 8, xcd = b % 8;
        return xcd * q + min(xcd, r) + b / 8;
    }();
    const int64_t world = (int64_t)lb * bd + tid;
    const unsigned slot = blockIdx.x;
#include "rollout_wm_body.inc"
}

// Launch shape as the static kernel: 256 lanes per block in FP32, 128 in
// FP64, the staged controls in NMAX x 3 x block reals of LDS.
template <typename R, int NMAX>
static hipError_t launch_tv_n(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              hipStream_t st) {
    const int block = sizeof(R) == 4 ? 256 : 128;
    const int64_t nworld = (int64_t)p.P * p.M;
    const unsigned blocks = (unsigned)((nworld + block - 1) / block);
    const size_t lds = (size_t)NMAX * 3 * block * sizeof(R);
    hipLaunchKernelGGL((k_rollout_wm_tv<R, NMAX>), dim3(blocks), dim3(block), lds, st, p, a,
                       (const R*)acR);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_tv_t(const RolloutParams& p, const RolloutArrays& a, const void* acR,
                              hipStream_t st) {
    if (p.N <= 2) return launch_tv_n<R, 2>(p, a, acR, st);
    if (p.N <= 4) return launch_tv_n<R, 4>(p, a, acR, st);
    if (p.N <= 6) return launch_tv_n<R, 6>(p, a, acR, st);
    if (p.N <= 8) return launch_tv_n<R, 8>(p, a, acR, st);
    if (p.N <= 10) return launch_tv_n<R, 10>(p, a, acR, st);
    if (p.N <= 12) return launch_tv_n<R, 12>(p, a, acR, st);
    if (p.N <= 16) return launch_tv_n<R, 16>(p, a, acR, st);
    return launch_tv_n<R, 20>(p, a, acR, st);
}

hipError_t launch_rollout_wm_tv(int prec, const RolloutParams& p, const RolloutArrays& a,
                                const void* acR, hipStream_t st) {
    if (!rollout_wm_supported(p.N) || p.w_kstride <= 0) return hipErrorInvalidValue;
    if (p.P <= 0 || p.M <= 0) return hipSuccess;
    return prec == 0 ? launch_tv_t<double>(p, a, acR, st) : launch_tv_t<float>(p, a, acR, st);
}

}  // namespace smc
