// Internal launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace lam {

// ------------------------------------------------------------- sort / scan
size_t scan_scratch_words(uint32_t n);
size_t radix_scratch_words(uint32_t n_cap);
int radix_passes(int bits, uint32_t n_cap);  // passes launch_radix_sort makes for ``bits`` key bits
hipError_t launch_excl_scan(const uint32_t* in, const uint32_t* idx, uint32_t n, uint32_t* out,
                            uint32_t* total, uint32_t* scratch, hipStream_t st);
hipError_t launch_radix_sort(const uint32_t* keys_first, uint32_t* keys_a, uint32_t* vals_a,
                             uint32_t* keys_b, uint32_t* vals_b, bool iota_first,
                             const uint32_t* n_dev, uint32_t n_cap, int bits, uint32_t* scratch,
                             bool* in_b, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);

// ------------------------------------------------------------- profiling
bool profiling();
void prof_mark(const char* name, bool is_begin, hipStream_t st);
struct ProfScope {
    const char* name;
    hipStream_t st;
    ProfScope(const char* n, hipStream_t s) : name(n), st(s) { prof_mark(name, true, st); }
    ~ProfScope() { prof_mark(name, false, st); }
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
    uint32_t* counters;  // [0] pairs needed, [1] overflow flag
    float4* rec0;
    float4* rec1;
    uint2* foot;
    uint32_t* depth_key;  // per-record depth key as projected (kept for inspection)
    uint32_t *depth_a, *depth_b, *recs_a, *recs_b;
    uint32_t* ntiles;
    uint32_t* offsets;
    uint32_t* sort_scratch;
    uint32_t *ikeys_a, *ikeys_b, *ivals_a, *ivals_b;
    uint2* ranges;
    uint32_t* n_contrib;
    float* t_final;
    float* rec_grad;
    float* rec_dz;  // per-record gradient of the rendered depth
};

hipError_t render_forward_launch(const RenderArgs& A, const RenderLayout& L, hipStream_t st);
hipError_t render_backward_launch(const RenderArgs& A, const RenderLayout& L, hipStream_t st);
void set_raster_schedule(int mode);

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
};

bool decode_layout(int prec, int n, int d, int M, int D, DecodeLayout* L);
void set_decode_shape(int mode);
// With st_dict (not null and not st) the dictionary gradients and the loss run
// on st_dict after the rows kernel on st; the caller joins the two streams.
hipError_t decode_loss_launch(const DecodeArgs& A, const DecodeLayout& L, hipStream_t st,
                              hipStream_t st_dict = nullptr);
hipError_t decode_forward_launch(const DecodeArgs& A, const DecodeLayout& L, hipStream_t st);
hipError_t decode_backward_launch(const DecodeArgs& A, const DecodeLayout& L, hipStream_t st);

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

bool tied_layout(int prec, int n, int ds, int M, int df, TiedLayout* L);
hipError_t tied_loss_launch(const TiedArgs& T, const TiedLayout& L, void* base, hipStream_t st);

}  // namespace lam
