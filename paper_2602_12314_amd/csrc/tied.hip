// The paper's tied dictionary decode and full feature loss (Eq. 5-6):
//
//   C[p][j] = < x_p / |x_p|, D_j / |D_j| >,  x_p = Q_p W     (cosine logits)
//   F^ = softmax_j(C / tau) D
//   L = lambda_cos mean_p (1 - cos(F^_p, F_p)) + lambda_2 mean_p |F^_p - F_p|^2
//       + lambda_D sum_j ReLU(|D0_j - D_j| - delta)
//
// mapped onto the attention kernels of decode.hip: with Q'_p = Q_p / (tau |Q_p W|)
// and K = normalize_rows(D) W^T the logits are Q' K^T (logit scale 1) and the
// values are V = D, so one decode call gives the loss terms, dQ', dK and dV.
// The kernels here form Q' and K before it and chain the gradients after it:
//   dQ_p = dQ'_p / (tau |x_p|) - (dQ'_p . Q_p) (G Q_p) / (tau |x_p|^3),  G = W W^T
//   dW   = dK^T normalize_rows(D) + (sum_p c_p Q_p^T Q_p) W,  c_p = -(dQ'_p . Q_p) / (tau |x_p|^3)
//   dD   = dV + (dB - B <B, dB>) / |D_j| + lambda_D (D - D0) / |D - D0| outside delta,
//          with B = normalize_rows(D), dB = dK W
// |x_p|^2 = Q_p G Q_p^T uses the d x d Gram matrix instead of the D-wide x_p.
// Norms are guarded as max(|.|, 1e-12) (a zero row normalises to zero, and its
// derivative is 1 / 1e-12 there).  Everything outside the decode call is FP32
// VALU work of O(n d^2 + M d D).
#include "common.h"
#include "kernels.h"

namespace lam {

constexpr float kNormEps = 1e-12f;

// Workgroup r < M: K[r][a] = <D_r, W_a> / max(|D_r|, eps) for a < DS and
// gD[r] = max(|D_r|, eps); workgroup M + a: G[a][b] = <W_a, W_b>.  The 256
// threads stride over the features and their partial sums meet in LDS.
template <int DS>
__global__ __launch_bounds__(256) void k_tied_dict(const float* __restrict__ W, const float* __restrict__ D, int M,
                                                   int df, float* __restrict__ K, float* __restrict__ gD,
                                                   float* __restrict__ G)
{
    __shared__ float red[DS + 1][256];
    const int r = blockIdx.x;
    const bool atom = r < M;
    const float* x = atom ? D + (size_t)r * df : W + (size_t)(r - M) * df;
    float acc[DS + 1];
#pragma unroll
    for (int a = 0; a <= DS; ++a) acc[a] = 0.f;
    for (int f = threadIdx.x; f < df; f += 256) {
        const float v = x[f];
        acc[DS] += v * v;
#pragma unroll
        for (int a = 0; a < DS; ++a) acc[a] += v * W[(size_t)a * df + f];
    }
#pragma unroll
    for (int a = 0; a <= DS; ++a) red[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
#pragma unroll
            for (int a = 0; a <= DS; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (atom) {
        const float g = fmaxf(sqrtf(red[DS][0]), kNormEps);
        if ((int)threadIdx.x < DS) K[(size_t)r * DS + threadIdx.x] = red[threadIdx.x][0] / g;
        if (threadIdx.x == 0) gD[r] = g;
    } else if ((int)threadIdx.x < DS) {
        G[(size_t)(r - M) * DS + threadIdx.x] = red[threadIdx.x][0];
    }
}

// Q'_p = Q_p / (tau max(|x_p|, eps)) with |x_p|^2 = Q_p G Q_p^T; gq[p] = max(|x_p|, eps).
template <int DS>
__global__ __launch_bounds__(256) void k_tied_queries(const float* __restrict__ Q, int n, const float* __restrict__ G,
                                                      float tau, float* __restrict__ Qs, float* __restrict__ gq)
{
    __shared__ float sG[DS * DS];
    for (int e = threadIdx.x; e < DS * DS; e += 256) sG[e] = G[e];
    __syncthreads();
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    float q[DS];
#pragma unroll
    for (int a = 0; a < DS; a += 4) {
        const float4 v = *reinterpret_cast<const float4*>(Q + (size_t)p * DS + a);
        q[a] = v.x; q[a + 1] = v.y; q[a + 2] = v.z; q[a + 3] = v.w;
    }
    float x2 = 0.f;
#pragma unroll
    for (int a = 0; a < DS; ++a) {
        float r = 0.f;
#pragma unroll
        for (int b = 0; b < DS; ++b) r += sG[a * DS + b] * q[b];
        x2 += q[a] * r;
    }
    const float g = fmaxf(sqrtf(fmaxf(x2, 0.f)), kNormEps);
    gq[p] = g;
    const float s = 1.0f / (tau * g);
#pragma unroll
    for (int a = 0; a < DS; a += 4)
        *reinterpret_cast<float4*>(Qs + (size_t)p * DS + a) = make_float4(q[a] * s, q[a + 1] * s, q[a + 2] * s, q[a + 3] * s);
}

// dQ from dQ' through Q' = Q / (tau |Q W|) (c_p = the coefficient of G Q_p) and,
// per workgroup of 256 pixels, part[block][a][b] =
// sum over its pixels of c_p Q_p[a] Q_p[b] from the same loads (the pixels
// are staged in LDS; thread t owns pairs t, t + 256, ...).
template <int DS>
__global__ __launch_bounds__(256) void k_tied_dq_gram(const float* __restrict__ Q, const float* __restrict__ dQs,
                                                      int n, const float* __restrict__ G,
                                                      const float* __restrict__ gq, float tau,
                                                      float* __restrict__ dQ, float* __restrict__ part)
{
    constexpr int PAIRS = DS * DS, PER = (PAIRS + 255) / 256;
    __shared__ float sG[DS * DS];
    __shared__ float sq[256][DS + 1];
    __shared__ float sc[256];
    for (int e = threadIdx.x; e < DS * DS; e += 256) sG[e] = G[e];
    __syncthreads();
    const int p = blockIdx.x * 256 + threadIdx.x;
    float q[DS];
#pragma unroll
    for (int a = 0; a < DS; ++a) q[a] = 0.f;
    float c = 0.f;
    if (p < n) {
        float dq[DS];
#pragma unroll
        for (int a = 0; a < DS; a += 4) {
            const float4 v = *reinterpret_cast<const float4*>(Q + (size_t)p * DS + a);
            const float4 u = *reinterpret_cast<const float4*>(dQs + (size_t)p * DS + a);
            q[a] = v.x; q[a + 1] = v.y; q[a + 2] = v.z; q[a + 3] = v.w;
            dq[a] = u.x; dq[a + 1] = u.y; dq[a + 2] = u.z; dq[a + 3] = u.w;
        }
        const float g = gq[p];
        float t = 0.f;
#pragma unroll
        for (int a = 0; a < DS; ++a) t += dq[a] * q[a];
        const float inv = 1.0f / (tau * g);
        c = g > kNormEps ? -t * inv / (g * g) : 0.0f;
        if (dQ) {
#pragma unroll
            for (int a = 0; a < DS; ++a) {
                float gqa = 0.f;
#pragma unroll
                for (int b = 0; b < DS; ++b) gqa += sG[a * DS + b] * q[b];
                dQ[(size_t)p * DS + a] = dq[a] * inv + c * gqa;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < DS; ++a) sq[threadIdx.x][a] = q[a];
    sc[threadIdx.x] = c;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = (int)threadIdx.x + 256 * k;
        if (e < PAIRS) {
            const int a = e / DS, b = e % DS;
            float sum = 0.f;
            for (int i = 0; i < 256; ++i) sum += sc[i] * sq[i][a] * sq[i][b];
            part[(size_t)blockIdx.x * PAIRS + e] = sum;
        }
    }
}

// A[a][b] = sum over the splits of part[s][a][b].  One wave per entry: the
// lanes stride over the split partials, then a wave
// sum (fixed order, so the result is deterministic).
__global__ __launch_bounds__(256) void k_tied_areduce(const float* __restrict__ part, int splits, int pairs,
                                                      float* __restrict__ A)
{
    const int e = blockIdx.x * (256 / kWave) + (int)(threadIdx.x / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    if (e >= pairs) return;  // whole waves
    float s = 0.f;
    for (int k = lane; k < splits; k += kWave) s += part[(size_t)k * pairs + e];
    s = wave_allsum(s);
    if (lane == 0) A[e] = s;
}

// dW[a][f] = sum_j dK[j][a] D[j][f] / gD[j] + sum_b A[a][b] W[b][f].
// Workgroup (f block of 64, a): wave w sums atoms j = w, w + 4, ...; the four
// partial sums meet in LDS in wave order.
__global__ __launch_bounds__(256) void k_tied_dw(const float* __restrict__ dK, const float* __restrict__ D,
                                                 const float* __restrict__ gD, const float* __restrict__ A,
                                                 const float* __restrict__ W, int ds, int M, int df,
                                                 float* __restrict__ dW)
{
    __shared__ float red[256 / kWave][kWave];
    const int a = blockIdx.y, w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int f = blockIdx.x * kWave + lane;
    const bool ok = f < df;
    float s = 0.f;
    if (ok) {
#pragma unroll 4
        for (int j = w; j < M; j += 256 / kWave) s += dK[(size_t)j * ds + a] * (D[(size_t)j * df + f] / gD[j]);
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && ok) {
        float t = red[0][lane];
#pragma unroll
        for (int k = 1; k < 256 / kWave; ++k) t += red[k][lane];
        for (int b = 0; b < ds; ++b) t += A[a * ds + b] * W[(size_t)b * df + f];
        dW[(size_t)a * df + f] = t;
    }
}

// One workgroup per atom j: dB = dK_j W, B = D_j / gD_j,
// dD_j = dV_j + (dB - B <B, dB>) / gD_j (+ the hinge term), pen[j] = its penalty.
__global__ __launch_bounds__(256) void k_tied_dd(const float* __restrict__ dK, const float* __restrict__ dV,
                                                 const float* __restrict__ D, const float* __restrict__ D0,
                                                 const float* __restrict__ gD, const float* __restrict__ W,
                                                 int ds, int df, float lam_D, float delta, float* __restrict__ dD,
                                                 float* __restrict__ pen)
{
    extern __shared__ float sh[];  // dB [df], then two reduction slots [256] each
    float* sdb = sh;
    float* r0 = sh + df;
    float* r1 = r0 + 256;
    const int j = blockIdx.x;
    const float g = gD[j];
    const float* dj = D + (size_t)j * df;
    const float* d0 = D0 + (size_t)j * df;
    float dot = 0.f, dev2 = 0.f;
    for (int f = threadIdx.x; f < df; f += 256) {
        float b = 0.f;
        for (int a = 0; a < ds; ++a) b += dK[(size_t)j * ds + a] * W[(size_t)a * df + f];
        sdb[f] = b;
        dot += (dj[f] / g) * b;
        const float e = dj[f] - d0[f];
        dev2 += e * e;
    }
    r0[threadIdx.x] = dot;
    r1[threadIdx.x] = dev2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r0[threadIdx.x] += r0[threadIdx.x + o];
            r1[threadIdx.x] += r1[threadIdx.x + o];
        }
        __syncthreads();
    }
    const float proj = g > kNormEps ? r0[0] : 0.0f;
    const float dev = sqrtf(r1[0]);
    const float th = dev > delta ? lam_D / dev : 0.0f;
    for (int f = threadIdx.x; f < df; f += 256)
        dD[(size_t)j * df + f] = dV[(size_t)j * df + f] + (sdb[f] - (dj[f] / g) * proj) / g + th * (dj[f] - d0[f]);
    if (threadIdx.x == 0) pen[j] = lam_D * fmaxf(dev - delta, 0.0f);
}

// loss = decode loss + sum_j pen[j] (fixed order).
__global__ __launch_bounds__(256) void k_tied_loss(const float* __restrict__ dec_loss, const float* __restrict__ pen,
                                                   int M, float* __restrict__ loss)
{
    __shared__ float sh[256];
    float s = 0.f;
    for (int j = threadIdx.x; j < M; j += 256) s += pen[j];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = dec_loss[0] + sh[0];
}

// FP32 and BF16 only.  With cosine logits over a temperature of 0.1 the
// softmax puts its weight on a few atoms, so the E4M3 rounding of D reaches F
// without the averaging over many atoms that keeps the untied E4M3 decode
// within its bounds (dQ off by about 5 % against the FP64 loss).
bool tied_layout(const lam_ctx* ctx, int prec, int n, int ds, int M, int df, TiedLayout* L)
{
    if (prec != LAM_FP32 && prec != LAM_BF16) return false;
    if (!decode_layout(ctx, prec, n, ds, M, df, &L->dec)) return false;
    size_t off = (L->dec.bytes + 255) / 256 * 256;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L->off_qs = take((size_t)n * ds * 4);
    L->off_gq = take((size_t)n * 4);
    L->off_dqs = take((size_t)n * ds * 4);
    L->off_k = take((size_t)M * ds * 4);
    L->off_gd = take((size_t)M * 4);
    L->off_g = take((size_t)ds * ds * 4);
    L->off_dk = take((size_t)M * ds * 4);
    L->off_dv = take((size_t)M * df * 4);
    L->off_apart = take((size_t)std::max((n + 255) / 256, 1) * ds * ds * 4);
    L->off_a = take((size_t)ds * ds * 4);
    L->off_pen = take((size_t)M * 4);
    L->off_loss = take(4);
    L->bytes = off;
    return true;
}

hipError_t tied_loss_launch(lam_ctx* ctx, const TiedArgs& T, const TiedLayout& L, void* base_, hipStream_t st)
{
    char* base = reinterpret_cast<char*>(base_);
    float* Qs = reinterpret_cast<float*>(base + L.off_qs);
    float* gq = reinterpret_cast<float*>(base + L.off_gq);
    float* dQs = reinterpret_cast<float*>(base + L.off_dqs);
    float* K = reinterpret_cast<float*>(base + L.off_k);
    float* gD = reinterpret_cast<float*>(base + L.off_gd);
    float* G = reinterpret_cast<float*>(base + L.off_g);
    float* dK = reinterpret_cast<float*>(base + L.off_dk);
    float* dV = reinterpret_cast<float*>(base + L.off_dv);
    float* apart = reinterpret_cast<float*>(base + L.off_apart);
    float* Am = reinterpret_cast<float*>(base + L.off_a);
    float* pen = reinterpret_cast<float*>(base + L.off_pen);
    float* dloss = reinterpret_cast<float*>(base + L.off_loss);
    const int n = T.n, ds = T.ds, M = T.M, df = T.df;
    const int pblocks = (n + 255) / 256;
    {
        ProfScope ps(ctx, "tied_prep", st);
        if (ds == 16)
            hipLaunchKernelGGL(k_tied_dict<16>, dim3(M + ds), dim3(256), 0, st, T.W, T.D, M, df, K, gD, G);
        else
            hipLaunchKernelGGL(k_tied_dict<32>, dim3(M + ds), dim3(256), 0, st, T.W, T.D, M, df, K, gD, G);
        if (n > 0) {
            if (ds == 16)
                hipLaunchKernelGGL(k_tied_queries<16>, dim3(pblocks), dim3(256), 0, st, T.Q, n, (const float*)G,
                                   T.tau, Qs, gq);
            else
                hipLaunchKernelGGL(k_tied_queries<32>, dim3(pblocks), dim3(256), 0, st, T.Q, n, (const float*)G,
                                   T.tau, Qs, gq);
        }
    }
    DecodeArgs A{};
    A.prec = T.prec; A.n = n; A.d = ds; A.M = M; A.D = df;
    A.Q = Qs; A.K = K; A.V = T.D; A.target = T.target; A.K0 = nullptr; A.lambda_tr = 0.0f;
    A.loss = dloss; A.dQ = dQs; A.dK = dK; A.dV = dV; A.row_cos = nullptr;
    A.lam_cos = T.lam_cos; A.lam_l2 = T.lam_2; A.logit_scale = 1.0f;
    DecodeLayout DL = L.dec;
    DL.base = base_;
    hipError_t e = decode_loss_launch(ctx, A, DL, st);
    if (e != hipSuccess) return e;
    ProfScope ps(ctx, "tied_grads", st);
    const int splits = n > 0 ? pblocks : 0;  // one partial per workgroup of 256 pixels
    if (n > 0) {
        if (ds == 16)
            hipLaunchKernelGGL(k_tied_dq_gram<16>, dim3(pblocks), dim3(256), 0, st, T.Q, (const float*)dQs, n,
                               (const float*)G, (const float*)gq, T.tau, T.dQ, apart);
        else
            hipLaunchKernelGGL(k_tied_dq_gram<32>, dim3(pblocks), dim3(256), 0, st, T.Q, (const float*)dQs, n,
                               (const float*)G, (const float*)gq, T.tau, T.dQ, apart);
    }
    hipLaunchKernelGGL(k_tied_areduce, dim3((ds * ds + 3) / 4), dim3(256), 0, st, (const float*)apart, splits,
                       ds * ds, Am);
    hipLaunchKernelGGL(k_tied_dw, dim3((df + kWave - 1) / kWave, ds), dim3(256), 0, st, (const float*)dK, T.D,
                       (const float*)gD, (const float*)Am, T.W, ds, M, df, T.dW);
    hipLaunchKernelGGL(k_tied_dd, dim3(M), dim3(256), (size_t)(df + 512) * 4, st, (const float*)dK,
                       (const float*)dV, T.D, T.D0, (const float*)gD, T.W, ds, df, T.lam_D, T.delta, T.dD, pen);
    hipLaunchKernelGGL(k_tied_loss, dim3(1), dim3(256), 0, st, (const float*)dloss, (const float*)pen, M, T.loss);
    return hipGetLastError();
}

}  // namespace lam

// ------------------------------------------------------------ C ABI

using namespace lam;

static bool tied_aligned(const void* p) { return ((uintptr_t)p & 15u) == 0; }

extern "C" {

lam_status lam_decode_tied_workspace_size(const lam_ctx* ctx, int precision, int n, int ds, int M, int df,
                                          uint64_t* bytes)
{
    if (!bytes || n < 0) return LAM_ERR_INVALID_ARG;
    TiedLayout L{};
    if (!tied_layout(ctx_options(ctx), precision, n, ds, M, df, &L)) return LAM_ERR_UNSUPPORTED;
    *bytes = L.bytes;
    return LAM_OK;
}

lam_status lam_decode_tied_loss(lam_ctx* ctx, int precision, const float* Q, int n, int ds, const float* W, const float* D,
                                int M, int df, const float* target, const float* D0,
                                const lam_tied_params* params, float* loss, float* dQ, float* dW, float* dD,
                                void* ws, uint64_t ws_bytes, void* stream)
{
    if (!ctx_ok(ctx) || n < 0 || !params) return LAM_ERR_INVALID_ARG;
    TiedLayout L{};
    if (!tied_layout(ctx, precision, n, ds, M, df, &L)) return LAM_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < L.bytes) return LAM_ERR_INVALID_ARG;
    if (!W || !D || !D0 || !loss || !dW || !dD || (n > 0 && (!Q || !target))) return LAM_ERR_INVALID_ARG;
    if (!tied_aligned(Q) || !tied_aligned(target) || !tied_aligned(dQ)) return LAM_ERR_INVALID_ARG;
    const lam_tied_params& p = *params;
    if (!(p.tau > 0.0f) || !(p.delta >= 0.0f) || !(p.lambda_cos >= 0.0f) || !(p.lambda_2 >= 0.0f) ||
        !(p.lambda_D >= 0.0f))
        return LAM_ERR_INVALID_ARG;
    TiedArgs T{};
    T.prec = precision; T.n = n; T.ds = ds; T.M = M; T.df = df;
    T.Q = Q; T.W = W; T.D = D; T.target = target; T.D0 = D0;
    T.tau = p.tau; T.lam_cos = p.lambda_cos; T.lam_2 = p.lambda_2; T.lam_D = p.lambda_D; T.delta = p.delta;
    T.loss = loss; T.dQ = dQ; T.dW = dW; T.dD = dD;
    return tied_loss_launch(ctx, T, L, ws, (hipStream_t)stream) == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

}  // extern "C"
