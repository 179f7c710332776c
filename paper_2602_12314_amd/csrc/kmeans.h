// Host-side interface of the streaming K-means kernels (kmeans.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct lam_ctx;

namespace lam {
namespace km {

// Byte offsets of one Lloyd run's scratch inside a workspace, for up to npts
// points, k centres and dimension D.
struct KmLayout {
    size_t off_cf, off_cn, off_a, off_bv, off_ka, off_va, off_kb, off_vb, off_sort, off_start, off_end, off_head, off_tail,
        off_headw, off_tailw, off_c0, off_c1, off_w, off_n;
    size_t bytes;
    int npts, k, D;
};

// The streaming step: the Lloyd scratch (sized for both runs) at offset 0,
// then the seeds' rows, micro-centres and weights, the merged set and the
// initial global centres.
struct StreamKmLayout {
    KmLayout lloyd;
    size_t off_m0, off_mc, off_mw, off_p, off_pw, off_g0, off_seeds;
    size_t bytes;
};

bool kmeans_shape_ok(int prec, int D, int k);
KmLayout kmeans_layout(int prec, int npts, int D, int k);
StreamKmLayout stream_kmeans_layout(int prec, int n, int D, int Kp, int K, int m);
hipError_t kmeans_assign_launch(lam_ctx* ctx, int prec, const float* X, int n, int D, const float* C, int k, const KmLayout& L,
                                void* ws, uint32_t* a, float* d2, hipStream_t st);
hipError_t kmeans_lloyd_launch(lam_ctx* ctx, int prec, const float* X, const float* w, int n, int D, const float* C0, int k,
                               int iters, float* C, float* W, uint32_t* a_out, const KmLayout& L, void* ws,
                               hipStream_t st);
hipError_t stream_kmeans_launch(lam_ctx* ctx, int prec, const float* F, int n, int D, const float* Dprev, const float* wprev,
                                int Kp, int K, const int32_t* seeds_host, int m, int iters_local, int iters_global,
                                float* Dout, float* Wout, const StreamKmLayout& S, void* ws, hipStream_t st);

}  // namespace km
}  // namespace lam
