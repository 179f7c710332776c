// Internal launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace lam {

// Launch timing of one kernel name: recorded (begin, end) event pairs and a
// pool of free events.
struct ProfSlot {
    std::string name;
    std::vector<hipEvent_t> begin, end;
    std::vector<hipEvent_t> pool;
};

}  // namespace lam

// The library context (opaque in the C ABI): the device it was made for, the
// launch choices an autotuner sets, and the per-device state the launches
// share (occupancy of the persistent kernels, kernels whose LDS limit was
// raised, the event that forks the dictionary gradients onto a second stream,
// the optional per-kernel timers).  The knobs are atomics and the caches sit
// behind ``mu``, so calls from several host threads on one context are safe.
struct lam_ctx {
    int device = 0;
    std::atomic<int> raster_schedule{2};  // 0 per tile, 1 persistent, 2 persistent for several views
    std::atomic<int> decode_shape{0};     // 0: 32 pixels x 4 waves, 1: 64 pixels x 8 waves where it fits
    std::atomic<int> decode_splits{0};    // pixel-range splits of the dictionary GEMMs; 0: sized to the device
    std::atomic<int> profile_on{0};
    hipEvent_t fork = nullptr;
    std::mutex mu;
    struct Occ {
        const void* kernel;
        int threads, blocks;
    };
    std::vector<Occ> occ;
    struct Lds {
        const void* kernel;
        size_t bytes;
    };
    std::vector<Lds> lds;
    std::vector<lam::ProfSlot> prof;
    int cus = 0;
    // this device's copy of the static scratch array of the allocation-free
    // decode entry point (device address, resolved when the context is made)
    void* static_scratch = nullptr;
    size_t static_scratch_bytes = 0;
};

namespace lam {

// True when ``ctx`` is usable from this thread: not null and made for the
// current HIP device.
bool ctx_ok(const lam_ctx* ctx);
// The options of ``ctx``, or the defaults when it is null (the host-only
// size queries accept a null context).
const lam_ctx* ctx_options(const lam_ctx* ctx);
// Workgroups of ``kernel`` with ``threads`` threads resident on the device at
// once (cached in the context).
int ctx_resident_blocks(lam_ctx* ctx, const void* kernel, int threads);
// Raises the dynamic LDS limit of ``kernel`` to at least ``bytes`` once per
// context (a function attribute of the device).
hipError_t ctx_ensure_lds(lam_ctx* ctx, const void* kernel, size_t bytes);

// ------------------------------------------------------------- sort / scan
// The scratch of a scan or a sort must be zero when it starts: the caller
// clears it (one fill may cover several scratch regions) or passes
// zero_scratch.  A look-back wait that outlives its bound (never expected)
// sets *err (a word of the scratch when err is null) and the result is wrong.
size_t scan_scratch_words(uint32_t n);
size_t radix_scratch_words(int bits, uint32_t n_cap);  // n_cap below 2^30
int radix_passes(int bits, uint32_t n_cap);  // passes launch_radix_sort makes for ``bits`` key bits
hipError_t launch_excl_scan(const uint32_t* in, const uint32_t* idx, uint32_t n, uint32_t* out,
                            uint32_t* total, uint32_t* over, uint32_t cap, uint32_t* scratch,
                            bool zero_scratch, uint32_t* err, hipStream_t st);
hipError_t launch_radix_sort(const uint32_t* keys_first, uint32_t* keys_a, uint32_t* vals_a,
                             uint32_t* keys_b, uint32_t* vals_b, bool iota_first,
                             const uint32_t* n_dev, uint32_t n_cap, int bits, uint32_t* scratch,
                             bool zero_scratch, uint32_t* err, bool* in_b, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);

// ------------------------------------------------------------- profiling
void prof_mark(lam_ctx* ctx, const char* name, bool is_begin, hipStream_t st);
struct ProfScope {
    lam_ctx* ctx;
    const char* name;
    hipStream_t st;
    ProfScope(lam_ctx* c, const char* n, hipStream_t s) : ctx(c), name(n), st(s) { prof_mark(ctx, name, true, st); }
    ~ProfScope() { prof_mark(ctx, name, false, st); }
};

// ------------------------------------------------------------- render
struct RenderArgs {
    int n, d;
    const float *means, *log_scales, *quats, *logits, *queries;
    float* Q;             // forward output
    float* T_final;       // forward output (caller copy)
    const float* dQ;      // backward input
    const float* T_final_in;  // backward: transmittance saved in the workspace
    float *d_means, *d_log_scales, *d_quats, *d_logits, *d_queries;
    // colour and depth (Sec. III-A), rendered when rgbd: colors [N, 3] in,
    // rgb [P, 3] and depth [P] out; d_rgb, d_depth in, d_colors out
    bool rgbd = false;
    const float* colors = nullptr;
    float *rgb = nullptr, *depth = nullptr;
    const float *d_rgb = nullptr, *d_depth = nullptr;
    float* d_colors = nullptr;
};

// Workspace carve-up (all pointers into the caller's buffer).
struct RenderLayout {
    CamSet cams;
    uint64_t records, capacity, pixels, bytes;
    int tile_bits;
    bool tile_in_b;  // where the sorted (tile, record) pairs end up
    // [0] pairs needed, [1] overflow flag, [2] / [3] work counters of the
    // persistent compositing forward / backward, [4] sort wait error
    uint32_t* counters;
    float4* rec0;
    float4* rec1;
    uint2* foot;
    uint32_t* depth_key;  // per-record depth key as projected (kept for inspection)
    uint32_t *depth_a, *depth_b, *recs_a, *recs_b;
    uint32_t* ntiles;
    uint32_t* offsets;
    // look-back scratch of the depth sort, the pair-count scan and the tile
    // sort, right after the counters: one fill clears [counters, zero_end)
    uint32_t *sort_scratch, *scan_scratch, *tile_scratch, *zero_end;
    uint32_t *ikeys_a, *ikeys_b, *ivals_a, *ivals_b;
    uint2* ranges;
    uint32_t* n_contrib;
    float* t_final;
    float* rec_grad;
    float* rec_dz;  // per-record gradient of the rendered depth
};

hipError_t render_forward_launch(lam_ctx* ctx, const RenderArgs& A, const RenderLayout& L, hipStream_t st);
hipError_t render_backward_launch(lam_ctx* ctx, const RenderArgs& A, const RenderLayout& L, hipStream_t st);

// ------------------------------------------------------------- decode
struct DecodeArgs {
    int prec, n, d, M, D;
    const float *Q, *K, *V, *target, *K0, *dF;
    float lambda_tr;
    float *loss, *dQ, *dK, *dV, *row_cos, *F;
    float lam_cos = 1.0f, lam_l2 = 0.0f;  // loss weights (1 - cos, |F - T|^2)
    float logit_scale = 0.0f;             // logits Q K^T * logit_scale; 0: 1 / sqrt(d)
};

struct DecodeLayout {
    int Mp;       // M rounded up to the atom tile
    int row_blocks;
    uint64_t bytes;
    void* base;
    // byte offsets inside the workspace, filled by decode_layout()
    size_t off_kb, off_vb, off_vt, off_kt, off_gf, off_m2, off_ds, off_qt, off_part, off_loss, off_sc;
    int splits, splits_k;
    bool wide;  // 64-pixel x 8-wave rows workgroups
};

// The decode block shape and split count come from the context.
bool decode_layout(const lam_ctx* ctx, int prec, int n, int d, int M, int D, DecodeLayout* L);
// With st_dict (not null and not st) the dictionary gradients and the loss run
// on st_dict after the rows kernel on st; the caller joins the two streams.
hipError_t decode_loss_launch(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, hipStream_t st,
                              hipStream_t st_dict = nullptr);
hipError_t decode_forward_launch(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, hipStream_t st);
hipError_t decode_backward_launch(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, hipStream_t st);

// ------------------------------------------------------------- tied decode
struct TiedArgs {
    int prec, n, ds, M, df;
    const float *Q, *W, *D, *target, *D0;
    float tau, lam_cos, lam_2, lam_D, delta;
    float *loss, *dQ, *dW, *dD;
};

struct TiedLayout {
    DecodeLayout dec;  // the decode call's workspace, at offset 0
    uint64_t bytes;
    size_t off_qs, off_gq, off_dqs, off_k, off_gd, off_g, off_dk, off_dv, off_apart, off_a, off_pen,
        off_loss;
};

bool tied_layout(const lam_ctx* ctx, int prec, int n, int ds, int M, int df, TiedLayout* L);
hipError_t tied_loss_launch(lam_ctx* ctx, const TiedArgs& T, const TiedLayout& L, void* base, hipStream_t st);

}  // namespace lam
