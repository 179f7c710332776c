// Photometric and depth L1 terms of the mapping objective (Eq. 7-9):
//   L = lambda_rgb mean_{p,c} |I^_pc - I_pc| + lambda_d mean_{p: Z_p > 0} |Z^_p - Z_p|
// (observed depth Z_p <= 0 marks a pixel without a measurement), and its
// gradient with respect to the rendered colour I^ and depth Z^ (sign, zero at
// a tie).  Deterministic: fixed per-block partial sums, then one block adds
// them in order.
#include <cmath>

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

// ------------------------------------------------------------- SSIM (Eq. 7)
//
// Structural similarity per colour channel with an 11 x 11 Gaussian window
// (sigma 1.5, normalised), C1 = 0.01^2, C2 = 0.03^2 and zero padding, each
// view its own image; L = lambda (1 - mean S).  One workgroup per 16 x 16
// tile: the tile and a 5-pixel halo of both images sit in LDS, the window is
// applied separably (rows, then columns) to x, y, x^2, y^2 and x y.  The
// forward writes, per pixel and channel, dL/dmu_x, dL/dE[x^2] and dL/dE[x y];
// the backward applies the (symmetric) window to those maps and forms
// dL/dx = W*dmu + 2 x W*dExx + y W*dExy.

constexpr int kSsT = 16, kSsR = 5, kSsH = kSsT + 2 * kSsR, kSsW = 2 * kSsR + 1;
constexpr float kSsC1 = 0.01f * 0.01f, kSsC2 = 0.03f * 0.03f;

struct SsimViews {
    int n, total_tiles;
    int w[LAM_MAX_CAMS], h[LAM_MAX_CAMS], tiles_x[LAM_MAX_CAMS], tile_base[LAM_MAX_CAMS + 1];
    long long pix_base[LAM_MAX_CAMS];
    float g[kSsW];
};

__device__ inline int ssim_view(const SsimViews& V, int tile)
{
    int v = 0;
    while (v + 1 < V.n && tile >= V.tile_base[v + 1]) ++v;
    return v;
}

__global__ __launch_bounds__(256) void k_ssim_fwd(SsimViews V, const float* __restrict__ x,
                                                  const float* __restrict__ y, float scale,
                                                  float* __restrict__ part, float* __restrict__ tsum)
{
    __shared__ float sx[kSsH][kSsH + 1], sy[kSsH][kSsH + 1];
    __shared__ float hq[5][kSsH][kSsT];
    __shared__ float red[256 / kWave];
    const int v = ssim_view(V, blockIdx.x);
    const int lt = blockIdx.x - V.tile_base[v];
    const int ty = lt / V.tiles_x[v], tx = lt - ty * V.tiles_x[v];
    const int W = V.w[v], H = V.h[v];
    const long long base = V.pix_base[v];
    const int lx = threadIdx.x & (kSsT - 1), ly = threadIdx.x / kSsT;
    const int px = tx * kSsT + lx, py = ty * kSsT + ly;
    const bool inside = px < W && py < H;
    const int x0 = tx * kSsT - kSsR, y0 = ty * kSsT - kSsR;
    const size_t p = (size_t)(base + (long long)py * W + px);
    float ssum = 0.0f;
    for (int c = 0; c < 3; ++c) {
        __syncthreads();
        for (int t = threadIdx.x; t < kSsH * kSsH; t += 256) {
            const int r = t / kSsH, q = t - r * kSsH;
            const int gx = x0 + q, gy = y0 + r;
            float a = 0.0f, b = 0.0f;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const size_t pp = (size_t)(base + (long long)gy * W + gx);
                a = x[3 * pp + c];
                b = y[3 * pp + c];
            }
            sx[r][q] = a;
            sy[r][q] = b;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < kSsH * kSsT; t += 256) {
            const int r = t / kSsT, j = t - r * kSsT;
            float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
            for (int k = 0; k < kSsW; ++k) {
                const float gk = V.g[k], a = sx[r][j + k], b = sy[r][j + k];
                m0 += gk * a;
                m1 += gk * b;
                m2 += gk * a * a;
                m3 += gk * b * b;
                m4 += gk * a * b;
            }
            hq[0][r][j] = m0; hq[1][r][j] = m1; hq[2][r][j] = m2; hq[3][r][j] = m3; hq[4][r][j] = m4;
        }
        __syncthreads();
        if (inside) {
            float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
            for (int k = 0; k < kSsW; ++k) {
                const float gk = V.g[k];
                mx += gk * hq[0][ly + k][lx];
                my += gk * hq[1][ly + k][lx];
                exx += gk * hq[2][ly + k][lx];
                eyy += gk * hq[3][ly + k][lx];
                exy += gk * hq[4][ly + k][lx];
            }
            const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
            const float a1 = 2.f * mx * my + kSsC1, a2 = 2.f * sxy + kSsC2;
            const float b1 = mx * mx + my * my + kSsC1, b2 = sxx + syy + kSsC2;
            const float ib = 1.0f / (b1 * b2);
            const float S = a1 * a2 * ib;
            ssum += S;
            // scale = dL/dS = -lambda / (3 P)
            part[9 * p + 3 * c] = scale * ((2.f * my * a2 - 2.f * my * a1) * ib - S * (2.f * mx / b1 - 2.f * mx / b2));
            part[9 * p + 3 * c + 1] = scale * (-S / b2);
            part[9 * p + 3 * c + 2] = scale * (2.f * a1 * ib);
        }
    }
    const float wsum = wave_allsum(ssum);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = wsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < 256 / kWave; ++k) t += red[k];
        tsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(SsimViews V, const float* __restrict__ x,
                                                  const float* __restrict__ y, const float* __restrict__ part,
                                                  float* __restrict__ d_rgb, int accumulate)
{
    __shared__ float sp[3][kSsH][kSsH + 1];
    __shared__ float hq[3][kSsH][kSsT];
    const int v = ssim_view(V, blockIdx.x);
    const int lt = blockIdx.x - V.tile_base[v];
    const int ty = lt / V.tiles_x[v], tx = lt - ty * V.tiles_x[v];
    const int W = V.w[v], H = V.h[v];
    const long long base = V.pix_base[v];
    const int lx = threadIdx.x & (kSsT - 1), ly = threadIdx.x / kSsT;
    const int px = tx * kSsT + lx, py = ty * kSsT + ly;
    const bool inside = px < W && py < H;
    const int x0 = tx * kSsT - kSsR, y0 = ty * kSsT - kSsR;
    const size_t p = (size_t)(base + (long long)py * W + px);
    for (int c = 0; c < 3; ++c) {
        __syncthreads();
        for (int t = threadIdx.x; t < kSsH * kSsH; t += 256) {
            const int r = t / kSsH, q = t - r * kSsH;
            const int gx = x0 + q, gy = y0 + r;
            float a = 0.f, b = 0.f, d = 0.f;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const size_t pp = (size_t)(base + (long long)gy * W + gx);
                a = part[9 * pp + 3 * c];
                b = part[9 * pp + 3 * c + 1];
                d = part[9 * pp + 3 * c + 2];
            }
            sp[0][r][q] = a;
            sp[1][r][q] = b;
            sp[2][r][q] = d;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < kSsH * kSsT; t += 256) {
            const int r = t / kSsT, j = t - r * kSsT;
            float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
            for (int k = 0; k < kSsW; ++k) {
                const float gk = V.g[k];
                m0 += gk * sp[0][r][j + k];
                m1 += gk * sp[1][r][j + k];
                m2 += gk * sp[2][r][j + k];
            }
            hq[0][r][j] = m0; hq[1][r][j] = m1; hq[2][r][j] = m2;
        }
        __syncthreads();
        if (inside) {
            float b0 = 0.f, b1 = 0.f, b2 = 0.f;
#pragma unroll
            for (int k = 0; k < kSsW; ++k) {
                const float gk = V.g[k];
                b0 += gk * hq[0][ly + k][lx];
                b1 += gk * hq[1][ly + k][lx];
                b2 += gk * hq[2][ly + k][lx];
            }
            const float gr = b0 + 2.f * x[3 * p + c] * b1 + y[3 * p + c] * b2;
            d_rgb[3 * p + c] = accumulate ? d_rgb[3 * p + c] + gr : gr;
        }
    }
}

__global__ __launch_bounds__(256) void k_ssim_final(const float* __restrict__ tsum, int ntiles, float lam,
                                                    float inv_total, float* __restrict__ loss)
{
    __shared__ float red[256 / kWave];
    float s = 0.f;
    for (int t = threadIdx.x; t < ntiles; t += 256) s += tsum[t];
    s = wave_allsum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < 256 / kWave; ++k) t += red[k];
        loss[0] = lam * (1.0f - t * inv_total);
    }
}

// Views from camera rows (only width and height are read).
static bool ssim_views(const float* cams, int n_cams, SsimViews* V, long long* pixels)
{
    if (!cams || n_cams < 1 || n_cams > LAM_MAX_CAMS) return false;
    *V = SsimViews{};
    V->n = n_cams;
    long long pix = 0;
    int tiles = 0;
    for (int c = 0; c < n_cams; ++c) {
        const float fw = cams[c * LAM_CAM_FLOATS], fh = cams[c * LAM_CAM_FLOATS + 1];
        if (!(fw >= 1.f && fw <= 8192.f && fh >= 1.f && fh <= 8192.f)) return false;
        const int w = (int)fw, h = (int)fh;
        if ((float)w != fw || (float)h != fh) return false;
        V->w[c] = w;
        V->h[c] = h;
        V->tiles_x[c] = (w + kSsT - 1) / kSsT;
        V->tile_base[c] = tiles;
        V->pix_base[c] = pix;
        tiles += V->tiles_x[c] * ((h + kSsT - 1) / kSsT);
        pix += (long long)w * h;
    }
    V->tile_base[n_cams] = tiles;
    V->total_tiles = tiles;
    double g[kSsW], s = 0.0;
    for (int k = 0; k < kSsW; ++k) {
        const double d = (double)(k - kSsR);
        g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        s += g[k];
    }
    for (int k = 0; k < kSsW; ++k) V->g[k] = (float)(g[k] / s);
    *pixels = pix;
    return true;
}

static size_t ssim_ws_bytes(long long pixels, int tiles)
{
    return ((size_t)pixels * 9 * 4 + 255) / 256 * 256 + (size_t)tiles * 4 + 256;
}

}  // namespace lam

using namespace lam;

extern "C" {

lam_status lam_rgbd_l1_workspace_size(const lam_ctx* ctx, int n, uint64_t* bytes)
{
    if (!bytes || n < 0) return LAM_ERR_INVALID_ARG;
    *bytes = l1_ws_bytes(n);
    return LAM_OK;
}

lam_status lam_rgbd_l1_loss(lam_ctx* ctx, const float* rgb, const float* rgb_obs, const float* depth, const float* depth_obs,
                            int n, float lambda_rgb, float lambda_depth, float* loss, float* d_rgb,
                            float* d_depth, void* ws, uint64_t ws_bytes, void* stream)
{
    if (!ctx_ok(ctx) || n < 0 || !loss || !ws || ws_bytes < l1_ws_bytes(n)) return LAM_ERR_INVALID_ARG;
    if (n > 0 && (!rgb || !rgb_obs || !depth || !depth_obs || !d_rgb || !d_depth)) return LAM_ERR_INVALID_ARG;
    if (!(lambda_rgb >= 0.0f) || !(lambda_depth >= 0.0f)) return LAM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int nb = l1_blocks(n);
    float* part = static_cast<float*>(ws);
    float* stats = part + (size_t)nb * 3;
    ProfScope ps(ctx, "rgbd_l1", st);
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

extern "C" {

lam_status lam_ssim_workspace_size(const lam_ctx* ctx, const float* cams, int n_cams, uint64_t* bytes)
{
    SsimViews V;
    long long pixels = 0;
    if (!bytes || !ssim_views(cams, n_cams, &V, &pixels)) return LAM_ERR_INVALID_ARG;
    *bytes = ssim_ws_bytes(pixels, V.total_tiles);
    return LAM_OK;
}

lam_status lam_ssim_loss(lam_ctx* ctx, const float* rgb, const float* rgb_obs, const float* cams, int n_cams, float lambda,
                         float* loss, float* d_rgb, int accumulate, void* ws, uint64_t ws_bytes, void* stream)
{
    SsimViews V;
    long long pixels = 0;
    if (!ctx_ok(ctx) || !ssim_views(cams, n_cams, &V, &pixels)) return LAM_ERR_INVALID_ARG;
    if (!rgb || !rgb_obs || !loss || !d_rgb || !ws || ws_bytes < ssim_ws_bytes(pixels, V.total_tiles))
        return LAM_ERR_INVALID_ARG;
    if (!(lambda >= 0.0f)) return LAM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    float* part = static_cast<float*>(ws);
    float* tsum = reinterpret_cast<float*>(static_cast<char*>(ws) + ((size_t)pixels * 9 * 4 + 255) / 256 * 256);
    const float inv_total = 1.0f / (3.0f * (float)pixels);
    ProfScope ps(ctx, "ssim", st);
    hipLaunchKernelGGL(k_ssim_fwd, dim3(V.total_tiles), dim3(256), 0, st, V, rgb, rgb_obs, -lambda * inv_total,
                       part, tsum);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, st, (const float*)tsum, V.total_tiles, lambda,
                       inv_total, loss);
    hipLaunchKernelGGL(k_ssim_bwd, dim3(V.total_tiles), dim3(256), 0, st, V, rgb, rgb_obs, (const float*)part,
                       d_rgb, accumulate ? 1 : 0);
    return hipGetLastError() == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

}  // extern "C"
