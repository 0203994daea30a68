// Wind field generation (Sec. "Wind Model"): the dense lower-triangular
// factor L = sigma Lx (x) Ly (x) Lz is expanded once per context; each SMC
// iteration forms W = wbar + L Z for all 2M Gaussian columns with an MFMA
// GEMM (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 on gfx950).
#include "engine.h"

namespace smc {

// L[g][h] = sigma * Lx[ix][jx] * Ly[iy][jy] * Lz[iz][jz] (computed in FP64).
template <typename T>
__global__ void k_kron_expand(const double* __restrict__ Lx, const double* __restrict__ Ly,
                              const double* __restrict__ Lz, int nx, int ny, int nz,
                              double sigma, T* __restrict__ Lf) {
    const int64_t G = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G * G) return;
    const int64_t g = t / G, h = t % G;
    const int iz = (int)(g % nz), iy = (int)((g / nz) % ny), ix = (int)(g / ((int64_t)ny * nz));
    const int jz = (int)(h % nz), jy = (int)((h / nz) % ny), jx = (int)(h / ((int64_t)ny * nz));
    const double v = sigma * ((Lx[ix * nx + jx] * Ly[iy * ny + jy]) * Lz[iz * nz + jz]);
    Lf[t] = (T)v;
}

template <typename T> struct Mfma;
// Operands of both instructions: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result register r of lane l holds D[row][l % 16] with
// row = 4 (l / 16) + r for f32 (groups of 4 consecutive rows) and
// row = 4 r + l / 16 for f64 (4 groups of one row).
template <> struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

// Block tile 32 (grid points) x 64 (columns), K stage 32; 4 waves as 2 x 2,
// each wave 16 x 32 = two 16x16 MFMA tiles.  The factor is lower triangular,
// so row block rb only needs k < (rb + 1) * 32.
// Stages are double-buffered in LDS with the next stage's global loads in
// flight in registers while the current one feeds the MFMAs (one barrier per
// stage).  LDS tiles are k-major: As[k][row], Bs[k][col], so the fragment
// reads A[l % 16][l / 16] and B[l / 16][l % 16] of the 64 lanes hit
// consecutive addresses.
constexpr int GB_M = 32, GB_N = 64, GB_K = 32;
constexpr int GA_LD = GB_M + 4;
constexpr int GBB_LD = GB_N + 4;

template <typename T>
struct GemmStage {
    T a[4];      // A[row][k4 .. k4+3] of this thread
    T b[2][4];   // B[k][c4 .. c4+3], two chunks
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 t; };
template <> struct Vec4<double> { typedef double4 t; };

// Four consecutive elements; one vector load when they are in bounds and the
// offset is a multiple of 4 elements (row pitch divisible by 4).
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ src, int64_t off, bool full,
                                      int nvalid, T (&out)[4]) {
    if (full && (off & 3) == 0) {
        const typename Vec4<T>::t v = *reinterpret_cast<const typename Vec4<T>::t*>(src + off);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else if (full) {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = src[off + e];
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = e < nvalid ? src[off + e] : (T)0;
    }
}

template <typename T>
__device__ __forceinline__ void gemm_fetch(const T* __restrict__ A, const T* __restrict__ Z,
                                           int G, int NC, int row0, int col0, int k0,
                                           GemmStage<T>& st) {
    const int tid = threadIdx.x;
    {   // A: 32 rows x 32 k, one 4-vector per thread
        const int r = tid >> 3, kq = (tid & 7) * 4;
        const int gr = row0 + r, gk = k0 + kq;
        const bool ok = gr < G && gk < G;
        load4(A, (int64_t)gr * G + gk, ok && gk + 4 <= G, ok ? G - gk : 0, st.a);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // B: 32 k x 64 cols, two 4-vectors per thread
        const int e = tid + h * 256;
        const int r = e >> 4, cq = (e & 15) * 4;
        const int gk = k0 + r, gc = col0 + cq;
        const bool ok = gk < G && gc < NC;
        load4(Z, (int64_t)gk * NC + gc, ok && gc + 4 <= NC, ok ? NC - gc : 0, st.b[h]);
    }
}

template <typename T>
__device__ __forceinline__ void gemm_store(const GemmStage<T>& st, T* As, T* Bs) {
    const int tid = threadIdx.x;
    {
        const int r = tid >> 3, kq = (tid & 7) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) As[(kq + e) * GA_LD + r] = st.a[e];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e0 = tid + h * 256;
        const int r = e0 >> 4, cq = (e0 & 15) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) Bs[r * GBB_LD + cq + e] = st.b[h][e];
    }
}

// Product of the tile's rows with the K range [kbeg, kend) (whole stages),
// accumulated from zero: acc0 / acc1 hold the wave's two 16 x 16 tiles.
template <typename T>
__device__ __forceinline__ void gemm_range(const T* __restrict__ A, const T* __restrict__ Z,
                                           int G, int NC, int row0, int col0, int kbeg, int kend,
                                           T* As, T* Bs, typename Mfma<T>::acc_t& acc0,
                                           typename Mfma<T>::acc_t& acc1) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 16;         // wave row offset in tile
    const int wc = (wave & 1) * 32;          // wave col offset in tile
    const int nst = (kend - kbeg + GB_K - 1) / GB_K;
    acc0 = {0, 0, 0, 0};
    acc1 = {0, 0, 0, 0};
    GemmStage<T> st;
    gemm_fetch<T>(A, Z, G, NC, row0, col0, kbeg, st);
    gemm_store<T>(st, As, Bs);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        const int cur = s & 1;
        const T* Ac = As + cur * (GB_K * GA_LD);
        const T* Bc = Bs + cur * (GB_K * GBB_LD);
        if (s + 1 < nst) gemm_fetch<T>(A, Z, G, NC, row0, col0, kbeg + (s + 1) * GB_K, st);
#pragma unroll
        for (int kk = 0; kk < GB_K; kk += 4) {
            const int kr = kk + (lane >> 4);
            const T a = Ac[kr * GA_LD + wr + (lane & 15)];
            const T b0 = Bc[kr * GBB_LD + wc + (lane & 15)];
            const T b1 = Bc[kr * GBB_LD + wc + 16 + (lane & 15)];
            acc0 = Mfma<T>::op(a, b0, acc0);
            acc1 = Mfma<T>::op(a, b1, acc1);
        }
        if (s + 1 < nst) gemm_store<T>(st, As + (cur ^ 1) * (GB_K * GA_LD),
                                       Bs + (cur ^ 1) * (GB_K * GBB_LD));
        __syncthreads();
    }
}

// W element (g, col) with col = 2 m + c: the mean (wm0, wm1), or
// wmean[2 (m / mper) + c] per group of mper samples, plus the product.
// Column col of row g is (field column jj, level iz) = (col / nzo, col % nzo),
// jj = 2 m + c, and lands at W[m][g nzo + iz][c]: nzo = 1 for the dense
// factor's product; nzo = nz when the rows are horizontal nodes and each
// field column carries its nz levels (the horizontal factor's product).
template <typename T>
__device__ __forceinline__ void gemm_put(int G, int g, int col, int nzo, double wm0, double wm1,
                                         const double* __restrict__ wmean, int mper, T v,
                                         T* __restrict__ W) {
    const int jj = nzo == 1 ? col : col / nzo, iz = col - jj * nzo;   // nzo is uniform
    const int m = jj >> 1, c = jj & 1;
    const double base = wmean ? wmean[2 * (m / mper) + c] : (c ? wm1 : wm0);
    W[(((int64_t)m * G + g) * nzo + iz) * 2 + c] = (T)(base + (double)v);
}

// The K extent of row block rb is split into chunks of GK_CHUNK (the factor
// is lower triangular: k < (rb + 1) 32), each accumulated from zero; the
// chunk products are summed in chunk order.  Both launch forms below do
// exactly these additions, so a field does not depend on how many columns
// share the launch.
constexpr int GK_CHUNK = 1024;

__host__ __device__ inline int gemm_kmax(int G, int rb) { return min(G, (rb + 1) * GB_M); }
__host__ __device__ inline int gemm_nchunks(int G, int rb) {
    return (gemm_kmax(G, rb) + GK_CHUNK - 1) / GK_CHUNK;
}

// One row block: one pipelined pass over its K extent, the accumulators
// folded into the running sum at every chunk boundary (the same additions as
// the per-chunk form), then the epilogue.
template <typename T>
__device__ __forceinline__ void gemm_rowblock(const T* __restrict__ A, const T* __restrict__ Z,
                                              int G, int NC, int nzo, int rb, int cb, double wm0,
                                              double wm1, const double* __restrict__ wmean,
                                              int mper, T* __restrict__ W, T* As, T* Bs) {
    typedef typename Mfma<T>::acc_t acc_t;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 16, wc = (wave & 1) * 32;
    const int row0 = rb * GB_M, col0 = cb * GB_N;
    const int kmax = gemm_kmax(G, rb);
    const int nst = (kmax + GB_K - 1) / GB_K;
    constexpr int kChunkStages = GK_CHUNK / GB_K;
    acc_t tot0 = {0, 0, 0, 0}, tot1 = {0, 0, 0, 0};
    acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    GemmStage<T> st;
    gemm_fetch<T>(A, Z, G, NC, row0, col0, 0, st);
    gemm_store<T>(st, As, Bs);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        const int cur = s & 1;
        const T* Ac = As + cur * (GB_K * GA_LD);
        const T* Bc = Bs + cur * (GB_K * GBB_LD);
        if (s + 1 < nst) gemm_fetch<T>(A, Z, G, NC, row0, col0, (s + 1) * GB_K, st);
#pragma unroll
        for (int kk = 0; kk < GB_K; kk += 4) {
            const int kr = kk + (lane >> 4);
            const T a = Ac[kr * GA_LD + wr + (lane & 15)];
            const T b0 = Bc[kr * GBB_LD + wc + (lane & 15)];
            const T b1 = Bc[kr * GBB_LD + wc + 16 + (lane & 15)];
            acc0 = Mfma<T>::op(a, b0, acc0);
            acc1 = Mfma<T>::op(a, b1, acc1);
        }
        if (s + 1 == nst || (s + 1) % kChunkStages == 0) {   // end of a chunk
#pragma unroll
            for (int r = 0; r < 4; ++r) { tot0[r] += acc0[r]; tot1[r] += acc1[r]; }
            acc0 = {0, 0, 0, 0};
            acc1 = {0, 0, 0, 0};
        }
        if (s + 1 < nst) gemm_store<T>(st, As + (cur ^ 1) * (GB_K * GA_LD),
                                       Bs + (cur ^ 1) * (GB_K * GBB_LD));
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int g = row0 + wr + Mfma<T>::row(lane, r);
        if (g >= G) continue;
        const int c0 = col0 + wc + (lane & 15), c1 = c0 + 16;
        if (c0 < NC) gemm_put<T>(G, g, c0, nzo, wm0, wm1, wmean, mper, tot0[r], W);
        if (c1 < NC) gemm_put<T>(G, g, c1, nzo, wm0, wm1, wmean, mper, tot1[r], W);
    }
}

// Whole row blocks per workgroup (enough tiles to fill the chip): row blocks
// R - 1 - rb and rb, so that all workgroups do the same work.
template <typename T>
__global__ void __launch_bounds__(256) k_wind_gemm(const T* __restrict__ A,
                                                   const T* __restrict__ Z, int G, int NC,
                                                   int nzo, double wm0, double wm1,
                                                   const double* __restrict__ wmean, int mper,
                                                   T* __restrict__ W) {
    __shared__ T As[2 * GB_K * GA_LD];
    __shared__ T Bs[2 * GB_K * GBB_LD];
    const int R = (G + GB_M - 1) / GB_M;
    const int rb = blockIdx.x;
    const int rb2 = R - 1 - rb;
    const int cb = blockIdx.y;
    gemm_rowblock<T>(A, Z, G, NC, nzo, rb2, cb, wm0, wm1, wmean, mper, W, As, Bs);   // heavy first
    if (rb2 != rb) {
        __syncthreads();
        gemm_rowblock<T>(A, Z, G, NC, nzo, rb, cb, wm0, wm1, wmean, mper, W, As, Bs);
    }
}

// One (row block, column block, chunk) per workgroup (few tiles: the chunks
// give the chip enough workgroups); the chunk product goes to
// part[chunk][g][col].  Workgroups past a row block's last chunk exit.
template <typename T>
__global__ void __launch_bounds__(256) k_wind_gemm_part(const T* __restrict__ A,
                                                        const T* __restrict__ Z, int G, int NC,
                                                        T* __restrict__ part) {
    __shared__ T As[2 * GB_K * GA_LD];
    __shared__ T Bs[2 * GB_K * GBB_LD];
    typedef typename Mfma<T>::acc_t acc_t;
    const int rb = blockIdx.x, cb = blockIdx.y, j = blockIdx.z;
    if (j >= gemm_nchunks(G, rb)) return;       // uniform over the workgroup
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 16, wc = (wave & 1) * 32;
    const int row0 = rb * GB_M, col0 = cb * GB_N;
    const int kmax = gemm_kmax(G, rb);
    acc_t a0, a1;
    gemm_range<T>(A, Z, G, NC, row0, col0, j * GK_CHUNK, min(kmax, (j + 1) * GK_CHUNK), As, Bs,
                  a0, a1);
    T* pj = part + (int64_t)j * G * NC;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int g = row0 + wr + Mfma<T>::row(lane, r);
        if (g >= G) continue;
        const int c0 = col0 + wc + (lane & 15), c1 = c0 + 16;
        if (c0 < NC) pj[(int64_t)g * NC + c0] = a0[r];
        if (c1 < NC) pj[(int64_t)g * NC + c1] = a1[r];
    }
}

// Sum of a row's chunk products in chunk order, then the epilogue.
template <typename T>
__global__ void __launch_bounds__(256) k_wind_gemm_sum(const T* __restrict__ part, int G, int NC,
                                                       int nzo, double wm0, double wm1,
                                                       const double* __restrict__ wmean,
                                                       int mper, T* __restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)G * NC) return;
    const int g = (int)(e / NC), col = (int)(e % NC);
    const int nch = gemm_nchunks(G, g / GB_M);
    T tot = 0;
    for (int j = 0; j < nch; ++j) tot += part[(int64_t)j * G * NC + e];
    gemm_put<T>(G, g, col, nzo, wm0, wm1, wmean, mper, tot, W);
}

// Levels of the time-correlated wind: the vertical factor of Qhat = sigma
// L_h (x) L_z applied along the nz levels of each horizontal node, and the
// columns regrouped level-fastest for the horizontal factor's product:
// Y[h][col][iz] = sum_{j <= iz} Lz[iz][j] U[h nz + j][col] (FP64 sums).
// Thread per (h, col); the reads of consecutive columns and the writes of a
// thread's nz levels are contiguous.
template <typename T>
__global__ void k_wind_levels(const T* __restrict__ U, const double* __restrict__ Lz, int nh,
                              int nz, int NC, T* __restrict__ Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nh * NC) return;
    const int h = (int)(t / NC), col = (int)(t % NC);
    const T* u = U + (int64_t)h * nz * NC + col;
    double uv[kMaxWindLevels];
#pragma unroll
    for (int j = 0; j < kMaxWindLevels; ++j) uv[j] = j < nz ? (double)u[(int64_t)j * NC] : 0.0;
    T* y = Y + ((int64_t)h * NC + col) * nz;
    for (int iz = 0; iz < nz; ++iz) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kMaxWindLevels; ++j)
            if (j <= iz) acc += Lz[iz * nz + j] * uv[j];
        y[iz] = (T)acc;
    }
}

hipError_t launch_kron_expand(int prec, const double* Lx, const double* Ly,
                              const double* Lz, int nx, int ny, int nz,
                              double sigma, void* Lfac, hipStream_t st) {
    const int64_t G = (int64_t)nx * ny * nz;
    const int64_t n = G * G;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_kron_expand<double>, dim3(blocks), dim3(256), 0, st, Lx, Ly,
                           Lz, nx, ny, nz, sigma, (double*)Lfac);
    else
        hipLaunchKernelGGL(k_kron_expand<float>, dim3(blocks), dim3(256), 0, st, Lx, Ly,
                           Lz, nx, ny, nz, sigma, (float*)Lfac);
    return hipGetLastError();
}

size_t wind_gemm_part_elems(int G, int M) {
    const int NC = 2 * M;
    const int R = (G + GB_M - 1) / GB_M;
    const int ncb = (NC + GB_N - 1) / GB_N;
    if ((int64_t)((R + 1) / 2) * ncb >= kWindGemmSplitBelow) return 0;   // whole row blocks
    return (size_t)gemm_nchunks(G, R - 1) * G * NC;
}

static hipError_t wind_gemm(int prec, const void* Lfac, const void* Z, double wm0, double wm1,
                            const double* wmean, int mper, int G, int M, int nzo, void* W,
                            void* part, hipStream_t st) {
    const int NC = 2 * M;
    const int R = (G + GB_M - 1) / GB_M;
    const int ncb = (NC + GB_N - 1) / GB_N;
    if (wind_gemm_part_elems(G, M) > 0) {   // few tiles: one workgroup per chunk
        if (!part) return hipErrorInvalidValue;
        const dim3 grid((unsigned)R, (unsigned)ncb, (unsigned)gemm_nchunks(G, R - 1));
        const int64_t n = (int64_t)G * NC;
        const unsigned sblocks = (unsigned)((n + 255) / 256);
        if (prec == 0) {
            hipLaunchKernelGGL(k_wind_gemm_part<double>, grid, dim3(256), 0, st,
                               (const double*)Lfac, (const double*)Z, G, NC, (double*)part);
            hipLaunchKernelGGL(k_wind_gemm_sum<double>, dim3(sblocks), dim3(256), 0, st,
                               (const double*)part, G, NC, nzo, wm0, wm1, wmean, mper,
                               (double*)W);
        } else {
            hipLaunchKernelGGL(k_wind_gemm_part<float>, grid, dim3(256), 0, st,
                               (const float*)Lfac, (const float*)Z, G, NC, (float*)part);
            hipLaunchKernelGGL(k_wind_gemm_sum<float>, dim3(sblocks), dim3(256), 0, st,
                               (const float*)part, G, NC, nzo, wm0, wm1, wmean, mper,
                               (float*)W);
        }
        return hipGetLastError();
    }
    dim3 grid((unsigned)((R + 1) / 2), (unsigned)ncb);
    if (prec == 0)
        hipLaunchKernelGGL(k_wind_gemm<double>, grid, dim3(256), 0, st,
                           (const double*)Lfac, (const double*)Z, G, NC, nzo, wm0, wm1, wmean,
                           mper, (double*)W);
    else
        hipLaunchKernelGGL(k_wind_gemm<float>, grid, dim3(256), 0, st, (const float*)Lfac,
                           (const float*)Z, G, NC, nzo, wm0, wm1, wmean, mper, (float*)W);
    return hipGetLastError();
}

hipError_t launch_wind_gemm(int prec, const void* Lfac, const void* Z, double wm0,
                            double wm1, int G, int M, void* W, void* part, hipStream_t st) {
    return wind_gemm(prec, Lfac, Z, wm0, wm1, nullptr, 1, G, M, 1, W, part, st);
}

hipError_t launch_wind_levels(int prec, const void* U, const double* Lz, int nh, int nz, int M,
                              void* Y, hipStream_t st) {
    if (nz < 1 || nz > kMaxWindLevels) return hipErrorInvalidValue;
    const int NC = 2 * M;
    const int64_t n = (int64_t)nh * NC;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (prec == 0)
        hipLaunchKernelGGL(k_wind_levels<double>, dim3(blocks), dim3(256), 0, st,
                           (const double*)U, Lz, nh, nz, NC, (double*)Y);
    else
        hipLaunchKernelGGL(k_wind_levels<float>, dim3(blocks), dim3(256), 0, st,
                           (const float*)U, Lz, nh, nz, NC, (float*)Y);
    return hipGetLastError();
}

hipError_t launch_wind_gemm_levels(int prec, const void* Lh, const void* Y, double wm0,
                                   double wm1, int nh, int nz, int M, void* W, void* part,
                                   hipStream_t st) {
    return wind_gemm(prec, Lh, Y, wm0, wm1, nullptr, 1, nh, M * nz, nz, W, part, st);
}

hipError_t launch_wind_gemm_levels_grouped(int prec, const void* Lh, const void* Y,
                                           const double* wmean, int mper, int nh, int nz, int M,
                                           void* W, void* part, hipStream_t st) {
    if (!wmean || mper < 1) return hipErrorInvalidValue;
    return wind_gemm(prec, Lh, Y, 0.0, 0.0, wmean, mper, nh, M * nz, nz, W, part, st);
}

hipError_t launch_wind_gemm_grouped(int prec, const void* Lfac, const void* Z,
                                    const double* wmean, int mper, int G, int M, void* W,
                                    void* part, hipStream_t st) {
    if (!wmean || mper < 1) return hipErrorInvalidValue;
    return wind_gemm(prec, Lfac, Z, 0.0, 0.0, wmean, mper, G, M, 1, W, part, st);
}

}  // namespace smc
