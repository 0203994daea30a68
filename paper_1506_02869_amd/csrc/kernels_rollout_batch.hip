// Persistent world-per-lane rollout of a batch of scenarios.
//
// The work of one rollout pass over a batch is a list of items, each a run of
// kItemWorlds consecutive worlds (particle, wind sample) of one scenario; the
// host orders the items of a bucket by decreasing N^2 H so that the longest
// items start first and short ones fill the tail.  A grid sized to the
// resident capacity of the chip loops: each wave takes the next item from an
// atomic counter, loads that scenario's scalars and arrays from the table
// (wave-uniform: scalar loads) and integrates its 64 worlds with the same
// per-step arithmetic as the single-scenario kernel (one shared body), so a
// scenario's costs are bit-identical in both launch styles.  Every wave
// leaves once the counter passes the item count, so the grid drains.
#include "rollout_math.h"

namespace smc {

template <typename R, int NMAX>
__global__ void __launch_bounds__(256, (wm_waves<R, NMAX>()))
k_rollout_wm_batch(const BatchScen* __restrict__ tab, const BatchItem* __restrict__ items,
                   int n_items, uint32_t* __restrict__ queue, const void* __restrict__ u_base,
                   unsigned long long* __restrict__ steps) {
    extern __shared__ unsigned char smem_raw[];
    R* uc = reinterpret_cast<R*>(smem_raw);   // [NMAX][3][blockDim.x]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // Item fetch without a branch: every lane takes part in the atomic, lane 0
    // adding 1 and the others 0, so lane 0's returned value is the wave's
    // ticket whatever order the lanes' operations take.  (A fetch guarded by
    // "lane == 0" sits next to the lane-0 counter update at the end of the
    // body; the compiler merged the two across the loop's back edge and turned
    // the uniform item loop into a divergent one in which lanes 1..63 re-read
    // a stale ticket forever.)
    const uint32_t inc = lane == 0 ? 1u : 0u;
    for (;;) {
        const uint32_t got = atomicAdd(queue, inc);
        const int it = __builtin_amdgcn_readfirstlane((int)got);
        if (it >= n_items) break;
        // table and items are read-only for the whole launch: constant
        // address space, so their scalar loads can be re-issued instead of
        // holding every scenario scalar in registers
        typedef const __attribute__((address_space(4))) BatchItem CItem;
        typedef const __attribute__((address_space(4))) BatchScen CScen;
        CItem* item = (CItem*)items + it;
        CScen* sc = (CScen*)tab + item->scen;
        const auto& p = sc->rp;   // fields loaded where used, as from kernel arguments
        RolloutArrays a;
        a.u = (const R*)u_base + sc->off_u;
        a.W = sc->ra.W;
        a.states = sc->ra.states;
        a.k_active = sc->ra.k_active;
        a.acpar = sc->ra.acpar;
        a.targets = sc->ra.targets;
        a.kind = sc->ra.kind;
        a.pop = sc->ra.pop;
        a.cost = sc->ra.cost;
        a.feas = sc->ra.feas;
        a.steps = steps;
        const R* __restrict__ acR = (const R*)sc->acR;
        const int64_t world = (int64_t)item->world0 + lane;
        const unsigned slot = (unsigned)it;
        constexpr bool kTV = false;
        constexpr bool kPC = false;
#include "rollout_wm_body.inc"
    }
}

// Dynamic LDS of one workgroup: the segment's controls of its lanes, kept
// within 64 KB.
constexpr size_t kMaxRolloutLds = 65536;

template <typename R, int NMAX>
static hipError_t launch_nb(const BatchScen* tab, const BatchItem* items, int n_items,
                            uint32_t* queue, const void* u, unsigned long long* steps, int block,
                            int grid, hipStream_t st) {
    const size_t lds = (size_t)NMAX * 3 * block * sizeof(R);
    if (lds > kMaxRolloutLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_rollout_wm_batch<R, NMAX>), dim3(grid), dim3(block), lds, st, tab,
                       items, n_items, queue, u, steps);
    return hipGetLastError();
}

template <typename R, int NMAX>
static int resident_nb(int block) {
    const size_t lds = (size_t)NMAX * 3 * block * sizeof(R);
    if (lds > kMaxRolloutLds) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&k_rollout_wm_batch<R, NMAX>), block, lds) !=
        hipSuccess)
        return 0;
    return nb;
}

#define SMC_BUCKET_SWITCH(R, CALL)          \
    switch (bucket) {                       \
    case 0: return CALL(R, 2);              \
    case 1: return CALL(R, 4);              \
    case 2: return CALL(R, 6);              \
    case 3: return CALL(R, 8);              \
    case 4: return CALL(R, 10);             \
    case 5: return CALL(R, 12);             \
    case 6: return CALL(R, 16);             \
    default: return CALL(R, 20);            \
    }

#define SMC_LAUNCH_NB(R, NM) launch_nb<R, NM>(tab, items, n_items, queue, u, steps, block, grid, st)
#define SMC_RESIDENT_NB(R, NM) resident_nb<R, NM>(block)

static_assert(kNumBuckets == 8, "bucket switch covers 8 buckets");

hipError_t launch_b_rollout(int prec, int bucket, const BatchScen* tab, const BatchItem* items,
                            int n_items, uint32_t* queue, const void* u,
                            unsigned long long* steps, int block, int grid, hipStream_t st) {
    if (bucket < 0 || bucket >= kNumBuckets) return hipErrorInvalidValue;
    if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
    if (n_items <= 0) return hipSuccess;
    if (grid < 1) return hipErrorInvalidValue;
    if (prec == 0) {
        SMC_BUCKET_SWITCH(double, SMC_LAUNCH_NB)
    } else {
        SMC_BUCKET_SWITCH(float, SMC_LAUNCH_NB)
    }
}

int b_rollout_resident(int prec, int bucket, int block) {
    if (bucket < 0 || bucket >= kNumBuckets) return 0;
    if (prec == 0) {
        SMC_BUCKET_SWITCH(double, SMC_RESIDENT_NB)
    } else {
        SMC_BUCKET_SWITCH(float, SMC_RESIDENT_NB)
    }
}

}  // namespace smc
