// Photometric and depth L1 terms of the mapping objective (Eq. 7-9):
//   L = lambda_rgb mean_{p,c} |I^_pc - I_pc| + lambda_d mean_{p: Z_p > 0} |Z^_p - Z_p|
// (observed depth Z_p <= 0 marks a pixel without a measurement), and its
// gradient with respect to the rendered colour I^ and depth Z^ (sign, zero at
// a tie).  Deterministic: fixed per-block partial sums, then one block adds
// them in order.
#include "common.h"
#include "kernels.h"

namespace lam {

constexpr int kL1Threads = 256;
constexpr int kL1MaxBlocks = 1024;

static int l1_blocks(int n) { return std::max(1, std::min(kL1MaxBlocks, (n + kL1Threads - 1) / kL1Threads)); }

__device__ inline float sgn(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

// Block sum of one value through LDS (wave sums, then the first wave).
__device__ inline float block_sum(float v, float* sh)
{
    v = wave_allsum(v);
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (lane == 0) sh[w] = v;
    __syncthreads();
    float t = 0.0f;
    if (threadIdx.x == 0)
        for (int k = 0; k < kL1Threads / kWave; ++k) t += sh[k];
    __syncthreads();
    return t;
}

// part[b] = (sum |dI|, sum over valid pixels |dZ|, valid count) of block b's
// contiguous pixel range.
__global__ __launch_bounds__(kL1Threads) void k_l1_partials(const float* __restrict__ rgb,
                                                          const float* __restrict__ rgb_obs,
                                                          const float* __restrict__ depth,
                                                          const float* __restrict__ depth_obs, int n,
                                                          float* __restrict__ part)
{
    __shared__ float sh[kL1Threads / kWave];
    const int per = (n + gridDim.x - 1) / gridDim.x;
    const int p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    float si = 0.0f, sz = 0.0f, cnt = 0.0f;
    for (int p = p0 + threadIdx.x; p < p1; p += kL1Threads) {
        si += fabsf(rgb[3 * (size_t)p] - rgb_obs[3 * (size_t)p]) +
              fabsf(rgb[3 * (size_t)p + 1] - rgb_obs[3 * (size_t)p + 1]) +
              fabsf(rgb[3 * (size_t)p + 2] - rgb_obs[3 * (size_t)p + 2]);
        if (depth_obs[p] > 0.0f) {
            sz += fabsf(depth[p] - depth_obs[p]);
            cnt += 1.0f;
        }
    }
    si = block_sum(si, sh);
    sz = block_sum(sz, sh);
    cnt = block_sum(cnt, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = si;
        part[3 * blockIdx.x + 1] = sz;
        part[3 * blockIdx.x + 2] = cnt;
    }
}

// loss[0] and stats[0] = the number of pixels with observed depth.
__global__ __launch_bounds__(kL1Threads) void k_l1_final(const float* __restrict__ part, int nblocks, int n,
                                                       float lam_rgb, float lam_d, float* __restrict__ loss,
                                                       float* __restrict__ stats)
{
    __shared__ float sh[kL1Threads / kWave];
    float si = 0.0f, sz = 0.0f, cnt = 0.0f;
    for (int b = threadIdx.x; b < nblocks; b += kL1Threads) {
        si += part[3 * b];
        sz += part[3 * b + 1];
        cnt += part[3 * b + 2];
    }
    si = block_sum(si, sh);
    sz = block_sum(sz, sh);
    cnt = block_sum(cnt, sh);
    if (threadIdx.x == 0) {
        const float li = n > 0 ? lam_rgb * si / (3.0f * (float)n) : 0.0f;
        const float lz = cnt > 0.0f ? lam_d * sz / cnt : 0.0f;
        loss[0] = li + lz;
        stats[0] = cnt;
    }
}

__global__ __launch_bounds__(kL1Threads) void k_l1_grad(const float* __restrict__ rgb,
                                                      const float* __restrict__ rgb_obs,
                                                      const float* __restrict__ depth,
                                                      const float* __restrict__ depth_obs, int n, float lam_rgb,
                                                      float lam_d, const float* __restrict__ stats,
                                                      float* __restrict__ d_rgb, float* __restrict__ d_depth)
{
    const float gi = lam_rgb / (3.0f * (float)max(n, 1));
    const float cnt = stats[0];
    const float gz = cnt > 0.0f ? lam_d / cnt : 0.0f;
    for (size_t p = blockIdx.x * (size_t)kL1Threads + threadIdx.x; p < (size_t)n;
         p += (size_t)gridDim.x * kL1Threads) {
#pragma unroll
        for (int c = 0; c < 3; ++c) d_rgb[3 * p + c] = gi * sgn(rgb[3 * p + c] - rgb_obs[3 * p + c]);
        d_depth[p] = depth_obs[p] > 0.0f ? gz * sgn(depth[p] - depth_obs[p]) : 0.0f;
    }
}

static size_t l1_ws_bytes(int n) { return (size_t)l1_blocks(n) * 3 * 4 + 256; }

}  // namespace lam

using namespace lam;

extern "C" {

lam_status lam_rgbd_l1_workspace_size(int n, uint64_t* bytes)
{
    if (!bytes || n < 0) return LAM_ERR_INVALID_ARG;
    *bytes = l1_ws_bytes(n);
    return LAM_OK;
}

lam_status lam_rgbd_l1_loss(const float* rgb, const float* rgb_obs, const float* depth, const float* depth_obs,
                            int n, float lambda_rgb, float lambda_depth, float* loss, float* d_rgb,
                            float* d_depth, void* ws, uint64_t ws_bytes, void* stream)
{
    if (n < 0 || !loss || !ws || ws_bytes < l1_ws_bytes(n)) return LAM_ERR_INVALID_ARG;
    if (n > 0 && (!rgb || !rgb_obs || !depth || !depth_obs || !d_rgb || !d_depth)) return LAM_ERR_INVALID_ARG;
    if (!(lambda_rgb >= 0.0f) || !(lambda_depth >= 0.0f)) return LAM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int nb = l1_blocks(n);
    float* part = static_cast<float*>(ws);
    float* stats = part + (size_t)nb * 3;
    ProfScope ps("rgbd_l1", st);
    if (n > 0) {
        hipLaunchKernelGGL(k_l1_partials, dim3(nb), dim3(kL1Threads), 0, st, rgb, rgb_obs, depth, depth_obs, n,
                           part);
    } else {
        hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(part), 3, 0u, st);
        if (e != hipSuccess) return LAM_ERR_HIP;
    }
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kL1Threads), 0, st, (const float*)part, n > 0 ? nb : 1, n,
                       lambda_rgb, lambda_depth, loss, stats);
    if (n > 0)
        hipLaunchKernelGGL(k_l1_grad, dim3(std::min(nb * 4, 4096)), dim3(kL1Threads), 0, st, rgb, rgb_obs, depth,
                           depth_obs, n, lambda_rgb, lambda_depth, (const float*)stats, d_rgb, d_depth);
    return hipGetLastError() == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

}  // extern "C"
