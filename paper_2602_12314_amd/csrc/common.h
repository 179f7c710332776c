// Shared device-side definitions of the gfx950 library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/latentam.h"

namespace lam {

// 3D Gaussian Splatting conventions for Eq. 2 / Eq. 4 (the paper defers the
// projection and blending details to 3DGS), as float32 values: the projection
// is computed in float32.
constexpr float kNear = 0.2f;          // cull when camera-space z <= kNear
constexpr float kDilation = 0.3f;      // added to the screen covariance diagonal
constexpr float kFovClamp = 1.3f;      // x/z, y/z clamp in the Jacobian, in tan(fov/2) units
constexpr float kEigFloor = 0.1f;      // floor under mid^2 - det
constexpr float kSigmas = 3.0f;        // footprint half-width in standard deviations
constexpr float kAlphaMax = 0.99f;     // alpha clamp
constexpr float kAlphaMin = 1.0f / 255.0f;  // pairs below are skipped
constexpr float kTStop = 1e-4f;        // stop before transmittance would drop below

constexpr int kWave = 64;

// One camera as the kernels see it (passed by value inside CamSet).
struct Cam {
    int w, h, tiles_x, tiles_y;
    float fx, fy, cx, cy;
    float vm[12];        // rows 0..2 of the world->camera matrix
    int tile_base;       // first global tile id of this view
    int pad_;
    long long pix_base;  // first pixel of this view in the concatenated pixel order
};

struct CamSet {
    int n;
    int tile_w, tile_h, tile_shift_x;  // tile_w = 1 << tile_shift_x
    int tile_shift_y, total_tiles, pad0, pad1;
    Cam c[LAM_MAX_CAMS];
};

// Camera owning a global tile id (uniform across a workgroup).
__device__ inline int cam_of_tile(const CamSet& cs, int tile)
{
    int c = 0;
    for (int k = 1; k < cs.n; ++k)
        if (tile >= cs.c[k].tile_base) c = k;
    return c;
}

// ---------------------------------------------------------------- wave sums
// DPP row shifts and row broadcasts; the total of the 64 lanes ends in lane 63.
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
__device__ inline float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK,
                                                      BANK_MASK, BOUND_ZERO));
}

__device__ inline float wave_sum_to_last(float v)
{
    v += dpp_f<0x111, 0xF, 0xF, true>(v);   // row_shr:1
    v += dpp_f<0x112, 0xF, 0xF, true>(v);   // row_shr:2
    v += dpp_f<0x114, 0xF, 0xE, false>(v);  // row_shr:4, banks 1..3
    v += dpp_f<0x118, 0xF, 0xC, false>(v);  // row_shr:8, banks 2..3
    v += dpp_f<0x142, 0xA, 0xF, false>(v);  // row_bcast:15 into rows 1, 3
    v += dpp_f<0x143, 0xC, 0xF, false>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

// Total over the 64 lanes, uniform (all lanes must be active).
__device__ inline float wave_sum(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_last(v)), 63));
}

__device__ inline float wave_max(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline float wave_allsum(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ inline unsigned lane_id() { return __lane_id(); }

}  // namespace lam
