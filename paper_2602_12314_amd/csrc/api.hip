// C ABI of the library (declared in include/latentam.h): argument validation
// on the host, workspace carve-up, and the launch sequences.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

using namespace lam;

namespace {

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int log2i(int v)
{
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

// Parses and validates the host camera rows.
lam_status make_camset(const float* cams, int n_cams, int tile_w, int tile_h, CamSet* cs,
                       uint64_t* pixels)
{
    if (!cams || !cs || n_cams < 1) return LAM_ERR_INVALID_ARG;
    if (n_cams > LAM_MAX_CAMS) return LAM_ERR_UNSUPPORTED;
    if (!is_pow2(tile_w) || !is_pow2(tile_h)) return LAM_ERR_UNSUPPORTED;
    const int area = tile_w * tile_h;
    if (area != 64 && area != 128 && area != 256) return LAM_ERR_UNSUPPORTED;
    memset(cs, 0, sizeof(*cs));
    cs->n = n_cams;
    cs->tile_w = tile_w;
    cs->tile_h = tile_h;
    cs->tile_shift_x = log2i(tile_w);
    cs->tile_shift_y = log2i(tile_h);
    int64_t tiles = 0, pix = 0;
    for (int c = 0; c < n_cams; ++c) {
        const float* row = cams + (size_t)c * LAM_CAM_FLOATS;
        const float wf = row[0], hf = row[1];
        if (!(wf >= 1.0f && wf <= 8192.0f && hf >= 1.0f && hf <= 8192.0f)) return LAM_ERR_INVALID_ARG;
        if (wf != floorf(wf) || hf != floorf(hf)) return LAM_ERR_INVALID_ARG;
        for (int k = 2; k < LAM_CAM_FLOATS; ++k)
            if (!isfinite(row[k])) return LAM_ERR_INVALID_ARG;
        if (!(row[2] > 0.0f) || !(row[3] > 0.0f)) return LAM_ERR_INVALID_ARG;
        Cam& cam = cs->c[c];
        cam.w = (int)wf;
        cam.h = (int)hf;
        cam.fx = row[2];
        cam.fy = row[3];
        cam.cx = row[4];
        cam.cy = row[5];
        for (int k = 0; k < 12; ++k) cam.vm[k] = row[6 + k];
        cam.tiles_x = (cam.w + tile_w - 1) / tile_w;
        cam.tiles_y = (cam.h + tile_h - 1) / tile_h;
        cam.tile_base = (int)tiles;
        cam.pix_base = pix;
        tiles += (int64_t)cam.tiles_x * cam.tiles_y;
        pix += (int64_t)cam.w * cam.h;
    }
    cs->total_tiles = (int)tiles;
    *pixels = (uint64_t)pix;
    return LAM_OK;
}

lam_status render_layout(int n_gauss, int d, const float* cams, int n_cams, int tile_w,
                         int tile_h, uint64_t capacity, void* base, RenderLayout* L)
{
    if (n_gauss < 0) return LAM_ERR_INVALID_ARG;
    if (d != 16 && d != 32) return LAM_ERR_UNSUPPORTED;
    uint64_t pixels = 0;
    lam_status s = make_camset(cams, n_cams, tile_w, tile_h, &L->cams, &pixels);
    if (s != LAM_OK) return s;
    const uint64_t R = (uint64_t)n_cams * (uint64_t)n_gauss;
    if (R >= (1ull << 30) || capacity >= (1ull << 30)) return LAM_ERR_UNSUPPORTED;
    L->records = R;
    L->capacity = capacity;
    L->pixels = pixels;
    const int tb = log2i(std::max(L->cams.total_tiles, 2));
    L->tile_bits = tb;
    L->tile_in_b = radix_passes(tb, (uint32_t)capacity) % 2 == 1;
    if (capacity == 0) L->tile_in_b = false;
    const size_t depth_words = radix_scratch_words(32, (uint32_t)R);
    const size_t scan_words = scan_scratch_words((uint32_t)R);
    const size_t tile_words = radix_scratch_words(tb, (uint32_t)capacity);
    char* p = (char*)base;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        char* q = p ? p + off : nullptr;
        off += align_up(bytes);
        return q;
    };
    L->counters = (uint32_t*)take(64);
    L->sort_scratch = (uint32_t*)take(depth_words * 4);
    L->scan_scratch = (uint32_t*)take(scan_words * 4);
    L->tile_scratch = (uint32_t*)take(tile_words * 4);
    L->zero_end = p ? (uint32_t*)(p + off) : nullptr;
    L->rec0 = (float4*)take(R * 16);
    L->rec1 = (float4*)take(R * 16);
    L->foot = (uint2*)take(R * 8);
    L->depth_key = (uint32_t*)take(R * 4);
    L->depth_a = (uint32_t*)take(R * 4);
    L->depth_b = (uint32_t*)take(R * 4);
    L->recs_a = (uint32_t*)take(R * 4);
    L->recs_b = (uint32_t*)take(R * 4);
    L->ntiles = (uint32_t*)take(R * 4);
    L->offsets = (uint32_t*)take(R * 4);
    L->ikeys_a = (uint32_t*)take(capacity * 4);
    L->ikeys_b = (uint32_t*)take(capacity * 4);
    L->ivals_a = (uint32_t*)take(capacity * 4);
    L->ivals_b = (uint32_t*)take(capacity * 4);
    L->ranges = (uint2*)take((uint64_t)L->cams.total_tiles * 8);
    L->n_contrib = (uint32_t*)take(pixels * 4);
    L->t_final = (float*)take(pixels * 4);
    L->rec_grad = (float*)take(R * 24);
    L->rec_dz = (float*)take(R * 4);
    L->bytes = off;
    return LAM_OK;
}

bool ptr_ok(const void* p, uint64_t count) { return count == 0 || p != nullptr; }

// Buffers accessed with 16-byte vector loads and stores.
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" {

const char* lam_status_string(int status)
{
    switch (status) {
        case LAM_OK: return "ok";
        case LAM_ERR_INVALID_ARG: return "invalid argument";
        case LAM_ERR_UNSUPPORTED: return "unsupported shape or option";
        case LAM_ERR_CAPACITY: return "tile instance capacity exceeded";
        case LAM_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

int lam_version(void) { return LAM_VERSION; }

lam_status lam_render_workspace_size(const lam_ctx* ctx, int n_gauss, int d, const float* cams, int n_cams,
                                     int tile_w, int tile_h, uint64_t instance_capacity,
                                     uint64_t* bytes)
{
    if (!bytes) return LAM_ERR_INVALID_ARG;
    RenderLayout L;
    lam_status s = render_layout(n_gauss, d, cams, n_cams, tile_w, tile_h, instance_capacity,
                                 nullptr, &L);
    if (s != LAM_OK) return s;
    *bytes = L.bytes;
    return LAM_OK;
}

static lam_status check_gauss(const float* means, const float* log_scales, const float* quats,
                              const float* logits, const float* queries, int n)
{
    if (n < 0) return LAM_ERR_INVALID_ARG;
    if (!ptr_ok(means, n) || !ptr_ok(log_scales, n) || !ptr_ok(quats, n) || !ptr_ok(logits, n) ||
        !ptr_ok(queries, n))
        return LAM_ERR_INVALID_ARG;
    return LAM_OK;
}

lam_status lam_render_forward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                              const float* opacity_logits, const float* queries, int n_gauss,
                              int d, const float* cams, int n_cams, int tile_w, int tile_h,
                              float* Q, float* T_final, void* ws, uint64_t ws_bytes,
                              uint64_t instance_capacity, void* stream)
{
    if (!ctx_ok(ctx)) return LAM_ERR_INVALID_ARG;
    lam_status s = check_gauss(means, log_scales, quats, opacity_logits, queries, n_gauss);
    if (s != LAM_OK) return s;
    RenderLayout L;
    s = render_layout(n_gauss, d, cams, n_cams, tile_w, tile_h, instance_capacity, ws, &L);
    if (s != LAM_OK) return s;
    if (!ws || ws_bytes < L.bytes) return LAM_ERR_INVALID_ARG;
    if (!ptr_ok(Q, L.pixels) || !ptr_ok(T_final, L.pixels)) return LAM_ERR_INVALID_ARG;
    if (!aligned16(Q) || !aligned16(queries)) return LAM_ERR_INVALID_ARG;
    RenderArgs A{};
    A.n = n_gauss;
    A.d = d;
    A.means = means;
    A.log_scales = log_scales;
    A.quats = quats;
    A.logits = opacity_logits;
    A.queries = queries;
    A.Q = Q;
    A.T_final = T_final;
    hipError_t e = render_forward_launch(ctx, A, L, (hipStream_t)stream);
    return e == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_render_backward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                               const float* opacity_logits, const float* queries, int n_gauss,
                               int d, const float* cams, int n_cams, int tile_w, int tile_h,
                               const float* dQ, float* d_means, float* d_log_scales,
                               float* d_quats, float* d_opacity_logits, float* d_queries,
                               void* ws, uint64_t ws_bytes, uint64_t instance_capacity,
                               void* stream)
{
    if (!ctx_ok(ctx)) return LAM_ERR_INVALID_ARG;
    lam_status s = check_gauss(means, log_scales, quats, opacity_logits, queries, n_gauss);
    if (s != LAM_OK) return s;
    if (!ptr_ok(d_means, n_gauss) || !ptr_ok(d_log_scales, n_gauss) || !ptr_ok(d_quats, n_gauss) ||
        !ptr_ok(d_opacity_logits, n_gauss) || !ptr_ok(d_queries, n_gauss))
        return LAM_ERR_INVALID_ARG;
    RenderLayout L;
    s = render_layout(n_gauss, d, cams, n_cams, tile_w, tile_h, instance_capacity, ws, &L);
    if (s != LAM_OK) return s;
    if (!ws || ws_bytes < L.bytes) return LAM_ERR_INVALID_ARG;
    if (!ptr_ok(dQ, L.pixels)) return LAM_ERR_INVALID_ARG;
    if (!aligned16(dQ) || !aligned16(queries)) return LAM_ERR_INVALID_ARG;
    RenderArgs A{};
    A.n = n_gauss;
    A.d = d;
    A.means = means;
    A.log_scales = log_scales;
    A.quats = quats;
    A.logits = opacity_logits;
    A.queries = queries;
    A.dQ = dQ;
    A.d_means = d_means;
    A.d_log_scales = d_log_scales;
    A.d_quats = d_quats;
    A.d_logits = d_opacity_logits;
    A.d_queries = d_queries;
    hipError_t e = render_backward_launch(ctx, A, L, (hipStream_t)stream);
    return e == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_render_rgbd_forward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                                   const float* opacity_logits, const float* queries, const float* colors,
                                   int n_gauss, int d, const float* cams, int n_cams, int tile_w, int tile_h,
                                   float* Q, float* rgb, float* depth, float* T_final, void* ws,
                                   uint64_t ws_bytes, uint64_t instance_capacity, void* stream)
{
    if (!ctx_ok(ctx)) return LAM_ERR_INVALID_ARG;
    lam_status s = check_gauss(means, log_scales, quats, opacity_logits, queries, n_gauss);
    if (s != LAM_OK) return s;
    if (!ptr_ok(colors, n_gauss)) return LAM_ERR_INVALID_ARG;
    RenderLayout L;
    s = render_layout(n_gauss, d, cams, n_cams, tile_w, tile_h, instance_capacity, ws, &L);
    if (s != LAM_OK) return s;
    if (!ws || ws_bytes < L.bytes) return LAM_ERR_INVALID_ARG;
    if (!ptr_ok(Q, L.pixels) || !ptr_ok(T_final, L.pixels) || !ptr_ok(rgb, L.pixels) ||
        !ptr_ok(depth, L.pixels))
        return LAM_ERR_INVALID_ARG;
    if (!aligned16(Q) || !aligned16(queries)) return LAM_ERR_INVALID_ARG;
    RenderArgs A{};
    A.n = n_gauss;
    A.d = d;
    A.means = means;
    A.log_scales = log_scales;
    A.quats = quats;
    A.logits = opacity_logits;
    A.queries = queries;
    A.Q = Q;
    A.T_final = T_final;
    A.rgbd = true;
    A.colors = colors;
    A.rgb = rgb;
    A.depth = depth;
    hipError_t e = render_forward_launch(ctx, A, L, (hipStream_t)stream);
    return e == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_render_rgbd_backward(lam_ctx* ctx, const float* means, const float* log_scales, const float* quats,
                                    const float* opacity_logits, const float* queries, const float* colors,
                                    int n_gauss, int d, const float* cams, int n_cams, int tile_w, int tile_h,
                                    const float* dQ, const float* d_rgb, const float* d_depth, float* d_means,
                                    float* d_log_scales, float* d_quats, float* d_opacity_logits,
                                    float* d_queries, float* d_colors, void* ws, uint64_t ws_bytes,
                                    uint64_t instance_capacity, void* stream)
{
    if (!ctx_ok(ctx)) return LAM_ERR_INVALID_ARG;
    lam_status s = check_gauss(means, log_scales, quats, opacity_logits, queries, n_gauss);
    if (s != LAM_OK) return s;
    if (!ptr_ok(colors, n_gauss) || !ptr_ok(d_colors, n_gauss)) return LAM_ERR_INVALID_ARG;
    if (!ptr_ok(d_means, n_gauss) || !ptr_ok(d_log_scales, n_gauss) || !ptr_ok(d_quats, n_gauss) ||
        !ptr_ok(d_opacity_logits, n_gauss) || !ptr_ok(d_queries, n_gauss))
        return LAM_ERR_INVALID_ARG;
    RenderLayout L;
    s = render_layout(n_gauss, d, cams, n_cams, tile_w, tile_h, instance_capacity, ws, &L);
    if (s != LAM_OK) return s;
    if (!ws || ws_bytes < L.bytes) return LAM_ERR_INVALID_ARG;
    if (!ptr_ok(dQ, L.pixels) || !ptr_ok(d_rgb, L.pixels) || !ptr_ok(d_depth, L.pixels))
        return LAM_ERR_INVALID_ARG;
    if (!aligned16(dQ) || !aligned16(queries)) return LAM_ERR_INVALID_ARG;
    RenderArgs A{};
    A.n = n_gauss;
    A.d = d;
    A.means = means;
    A.log_scales = log_scales;
    A.quats = quats;
    A.logits = opacity_logits;
    A.queries = queries;
    A.dQ = dQ;
    A.d_means = d_means;
    A.d_log_scales = d_log_scales;
    A.d_quats = d_quats;
    A.d_logits = d_opacity_logits;
    A.d_queries = d_queries;
    A.rgbd = true;
    A.colors = colors;
    A.d_rgb = d_rgb;
    A.d_depth = d_depth;
    A.d_colors = d_colors;
    hipError_t e = render_backward_launch(ctx, A, L, (hipStream_t)stream);
    return e == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_render_counters(lam_ctx* ctx, const void* ws, void* stream, uint64_t* instances_needed,
                               int* overflowed)
{
    if (!ctx_ok(ctx) || !ws || !instances_needed || !overflowed) return LAM_ERR_INVALID_ARG;
    uint32_t c[5] = {0, 0, 0, 0, 0};
    if (hipMemcpyAsync(c, ws, sizeof(c), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
        return LAM_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return LAM_ERR_HIP;
    *instances_needed = c[0];
    *overflowed = (int)c[1];
    if (c[4]) return LAM_ERR_HIP;  // a sort wait outlived its bound: the binning is not valid
    return c[1] ? LAM_ERR_CAPACITY : LAM_OK;
}

lam_status lam_render_debug_views(const lam_ctx* ctx, const void* ws, int n_gauss, int d, const float* cams,
                                  int n_cams, int tile_w, int tile_h, uint64_t instance_capacity,
                                  const uint32_t** tile_keys, const uint32_t** tile_recs,
                                  const uint32_t** ranges, const uint32_t** depth_keys,
                                  const uint32_t** footprints, const uint32_t** n_contrib)
{
    if (!ws) return LAM_ERR_INVALID_ARG;
    RenderLayout L;
    lam_status s = render_layout(n_gauss, d, cams, n_cams, tile_w, tile_h, instance_capacity,
                                 (void*)ws, &L);
    if (s != LAM_OK) return s;
    if (tile_keys) *tile_keys = L.tile_in_b ? L.ikeys_b : L.ikeys_a;
    if (tile_recs) *tile_recs = L.tile_in_b ? L.ivals_b : L.ivals_a;
    if (ranges) *ranges = (const uint32_t*)L.ranges;
    if (depth_keys) *depth_keys = L.depth_key;
    if (footprints) *footprints = (const uint32_t*)L.foot;
    if (n_contrib) *n_contrib = L.n_contrib;
    return LAM_OK;
}

}  // extern "C"
