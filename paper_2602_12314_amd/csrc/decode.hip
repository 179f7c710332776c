// Dictionary decode (paper Eq. 5) and feature loss (Eq. 6) on gfx950 MFMA.
//
//   S = Q K^T / sqrt(d),  P = softmax_atoms(S),  F = P V
//   L = mean_p (1 - cos(F_p, T_p)) + lambda ||K - K0||^2
//
// k_dec_rows handles 32 pixels per 256-thread workgroup (4 waves; or 64 pixels
// per 8 waves, each V fragment then feeding two pixel groups):
//   S^T tiles (32 atoms x 32 pixels) come from MFMA with the pixel as the
//   column, so the softmax statistics of a pixel stay inside one lane pair;
//   pass 1 takes the row max, pass 2 writes the unnormalised weights
//   P~ = exp(S - m) to LDS, F^T = V^T P~^T runs with each wave owning a share
//   of the D rows, and the epilogue forms 1 - cos and the cosine gradient
//   G = dL/dF / l (the softmax normaliser l folded in).  Then, per atom tile,
//   dP = G V^T (G staged in LDS), dS = P~ (dP - delta) and dQ^T += K^T dS^T with
//   dS^T fed from registers (K^T pre-permuted to match the MFMA lane layout).
// The pixel reductions are split-K MFMA GEMMs over "pixel-blocked transposed"
// copies that k_dec_rows writes, X^T_blk[block][row][32 pixels], so every MFMA
// fragment is one 16-byte load: dK = dS^T Q (k_dec_tn) and dV = P~^T G
// (k_dec_dv), which rebuilds P~ from Q, K and the saved row max rather than
// reading it.  The softmax is recomputed in the backward part, never stored.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace lam {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr float kFp8Max = 448.0f;  // largest finite OCP E4M3 value

constexpr int kPx = 32;          // pixels per row block
constexpr int kAtomAlign = 64;   // atom padding
constexpr float kLog2e = 1.4426950408889634f;

// ------------------------------------------------------------ precisions

// A fragment holds 8 consecutive K-values of one MFMA row/column per lane:
// lane l covers K-indices 8 (l / 32) + 0..7 of a 16-wide K chunk.
struct TF32 {
    using T = float;
    using Frag = f32x8;
    static constexpr int kBytes = 4;
    __device__ static Frag load(const T* p)
    {
        const float4 a = reinterpret_cast<const float4*>(p)[0];
        const float4 b = reinterpret_cast<const float4*>(p)[1];
        Frag f = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        return f;
    }
    __device__ static Frag from_f32(const float* v)
    {
        Frag f;
#pragma unroll
        for (int t = 0; t < 8; ++t) f[t] = v[t];
        return f;
    }
    __device__ static T cvt(float x) { return x; }
    __device__ static float to_f32(T x) { return x; }
    // K = 16 as 8 steps of the 32x32x2 f32 MFMA (K-index 8h + s in step s)
    __device__ static void mma(f32x16& c, const Frag& a, const Frag& b)
    {
#pragma unroll
        for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], c, 0, 0, 0);
    }
    __device__ static void store4(T* p, float a, float b, float c, float d)
    {
        *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
    }
};

struct TBF16 {
    using T = __bf16;
    using Frag = bf16x8;
    static constexpr int kBytes = 2;
    __device__ static Frag load(const T* p) { return *reinterpret_cast<const bf16x8*>(p); }
    __device__ static Frag from_f32(const float* v)
    {
        Frag f;
#pragma unroll
        for (int t = 0; t < 8; ++t) f[t] = (__bf16)v[t];
        return f;
    }
    __device__ static T cvt(float x) { return (__bf16)x; }
    __device__ static float to_f32(T x) { return (float)x; }
    __device__ static void mma(f32x16& c, const Frag& a, const Frag& b)
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static void store4(T* p, float a, float b, float c, float d)
    {
        bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
        *reinterpret_cast<bf16x4*>(p) = v;
    }
};

// 2^x for the softmax weights, whose arguments (logit minus the row max) are
// never positive: the hardware exp2 without the range fix-ups of exp2f (a
// result below the FP32 normal range becomes zero, which the sums ignore).
__device__ inline float exp2_weight(float x) { return __builtin_amdgcn_exp2f(x); }

// Row of the 32x32 MFMA result held in register r of lane l (column = l % 32).
__device__ inline int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Atom slot k (0..15) of a 16-atom chunk as fed from the result registers of
// the previous MFMA: B fragment element t of lane half h is result register
// 8c + t, i.e. atom 8 (t / 4) + 4 h + t % 4.
__host__ __device__ inline int perm16(int k) { return 8 * ((k & 7) >> 2) + 4 * (k >> 3) + (k & 3); }

// Fragment-major operand layout.  An operand X[R][C] (R a multiple of 32, C of
// 16) used with its row as the MFMA row/column and C as the K dimension is
// stored block by block: block (row / 32, k / 16) holds 64 lanes x 8 elements,
// element (row, k) at lane 32 (k / 8 % 2) + row % 32, slot k % 8.  A wave's
// fragment load is then one contiguous run instead of 32 strided rows.  The
// E4M3 operand uses K chunks of 64: 64 lanes x 32 bytes, lane 32 (k / 32 % 2) +
// row % 32, byte k % 32.
// Fragment (row block rb, K chunk c) of a fragment-major operand with nc chunks.
template <class P>
__device__ inline typename P::Frag load_frag(const typename P::T* X, int rb, int c, int nc, int lane)
{
    return P::load(X + ((((size_t)rb * nc + c) << 6) + lane) * 8);
}

// Row stride (elements) of a wave's dS scratch tile [32 pixels][32 atoms + pad].
constexpr int kScLd = 40;

// Rows [0, nrows) of the transpose of an LDS tile S[pixel][row] (32 pixels,
// leading dimension ld) written to Dst[row][32 pixels] in HBM, one chunk of 8
// pixels (16 bytes in BF16) per store: chunk q = q0, q0 + dq, ... covers row
// q / 4, pixels 8 (q % 4) .. + 7.  This turns the one-pixel-per-lane MFMA
// result layout into whole-chunk stores of the pixel-blocked transposes.
// With PERM the pixels of each 16-pixel half are stored in perm16 order
// (position p holds pixel perm16(p)), the order in which k_dec_dv's recomputed
// P~ fragments hold them.
template <class P, bool PERM = false>
__device__ inline void store_transposed(const typename P::T* S, int ld, int nrows, typename P::T* Dst,
                                        int q0, int dq)
{
    for (int q = q0; q < nrows * 4; q += dq) {
        const int row = q >> 2, pg = (q & 3) * 8;
        typename P::Frag f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int pix = PERM ? (pg & 16) + perm16((pg & 15) + j) : pg + j;
            f[j] = S[pix * ld + row];
        }
        *reinterpret_cast<typename P::Frag*>(Dst + (size_t)row * kPx + pg) = f;
    }
}

// ------------------------------------------------------------ prep

// All four in the fragment-major layout (frag_index), converted to the compute type:
// Kb  = K   [Mp][d]   rows >= M zero
// Vb  = V   [Mp][D]
// Vt  = V^T [D][Mp]
// Ktp = K^T [32][Mp]  rows >= d zero, atoms permuted by perm16 in each 16-chunk
// Each thread writes consecutive destination elements (reads of K and V are
// scattered; both are small and cached).
template <class P>
__global__ __launch_bounds__(256) void k_dec_prep(const float* __restrict__ K, const float* __restrict__ V,
                                                  int M, int Mp, int d, int D, typename P::T* Kb,
                                                  typename P::T* Vb, typename P::T* Vt,
                                                  typename P::T* Ktp)
{
    const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    // inverse of frag_index for an operand with C columns
    auto rowk = [](size_t i, int C, int& row, int& k) {
        const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
        const size_t blk = i >> 9;
        const int nc = C >> 4;
        row = (int)(blk / nc) * 32 + (lane & 31);
        k = (int)(blk % nc) * 16 + (lane >> 5) * 8 + e;
    };
    int row, k;
    for (size_t i = tid; i < (size_t)Mp * D; i += stride) {
        rowk(i, D, row, k);  // row = atom, k = feature
        Vb[i] = P::cvt(row < M ? V[(size_t)row * D + k] : 0.0f);
        if (Vt) {
            rowk(i, Mp, row, k);  // row = feature, k = atom
            Vt[i] = P::cvt(k < M ? V[(size_t)k * D + row] : 0.0f);
        }
    }
    for (size_t i = tid; i < (size_t)Mp * d; i += stride) {
        rowk(i, d, row, k);
        Kb[i] = P::cvt(row < M ? K[(size_t)row * d + k] : 0.0f);
    }
    for (size_t i = tid; i < (size_t)32 * Mp; i += stride) {
        rowk(i, Mp, row, k);
        const int a = (k & ~15) + perm16(k & 15);
        Ktp[i] = P::cvt((row < d && a < M) ? K[(size_t)a * d + row] : 0.0f);
    }
}

// FP8 forward contraction F = P V.  Per-atom scales s^V = amax(V_j) / 448 map
// each row of V onto the E4M3 range; sc = [unused (Mp) | s^V (Mp) | max_j s^V_j bits].
// The logits keep BF16 K and the backward keeps the BF16 copies of the FP32
// dictionary: FP8 logits or an FP8 backward cost far more accuracy than the
// few flops they would save.
__global__ __launch_bounds__(256) void k_dec_scales(const float* __restrict__ V, int M, int Mp, int D,
                                                    float* __restrict__ sc)
{
    __shared__ float sv[256];
    const int row = blockIdx.x;
    float av = 0.f;
    if (row < M)
        for (int j = threadIdx.x; j < D; j += 256) av = fmaxf(av, fabsf(V[(size_t)row * D + j]));
    sv[threadIdx.x] = av;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sv[threadIdx.x] = fmaxf(sv[threadIdx.x], sv[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float v = sv[0] > 0.f ? sv[0] / kFp8Max : 0.0f;
        sc[Mp + row] = v;
        atomicMax(reinterpret_cast<unsigned*>(sc + 2 * Mp), __float_as_uint(v));
    }
}

// E4M3 with round-to-nearest-even; the conversion does not saturate (values
// beyond 448 become NaN), so inputs are clamped to the finite range first.
__device__ inline uint8_t to_e4m3(float x)
{
    x = fminf(fmaxf(x, -kFp8Max), kFp8Max);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF);
}

// Vt8 = E4M3(V / s^V) transposed [D][Mp] in the E4M3 fragment-major layout
// (frag8_index); sv_fold = s^V * 448 / max s^V and unscale = max s^V / 448.
// Kb, Vb, Ktp are filled by k_dec_prep<TBF16>.
__global__ __launch_bounds__(256) void k_dec_prep_fp8(const float* __restrict__ V, int M, int Mp, int D,
                                                      const float* __restrict__ sc, uint8_t* Vt8,
                                                      float* sv_fold, float* unscale)
{
    const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const float vmax = __uint_as_float(reinterpret_cast<const unsigned*>(sc)[2 * Mp]);
    const int nc = Mp >> 6;
    for (size_t i = tid; i < (size_t)Mp * D; i += stride) {
        const int e = (int)(i & 31), lane = (int)((i >> 5) & 63);
        const size_t blk = i >> 11;
        const int c = (int)(blk / nc) * 32 + (lane & 31);       // feature
        const int a = (int)(blk % nc) * 64 + (lane >> 5) * 32 + e;  // atom
        const float s = sc[Mp + a];
        uint8_t q = 0;
        if (a < M && s > 0.f) q = to_e4m3(V[(size_t)a * D + c] / s);
        Vt8[i] = q;
    }
    for (size_t i = tid; i < (size_t)Mp; i += stride)
        sv_fold[i] = vmax > 0.f ? sc[Mp + i] * (kFp8Max / vmax) : 0.0f;
    if (tid == 0) unscale[0] = vmax / kFp8Max;
}

// ------------------------------------------------------------ rows kernel

enum { MODE_INFER = 0, MODE_LOSS = 1, MODE_ADJ = 2 };

struct RowsArgs {
    int n, d, M, Mp, D;
    float scale_log2;   // log2(e) / sqrt(d)
    float inv_sqrt_d;
    float inv_n;
    float lam_cos, lam_l2;  // loss weights of 1 - cos and of |F - T|^2 (LOSS mode)
    const float* Q;
    const float* target;  // MODE_LOSS
    const float* dF;      // MODE_ADJ
    float* F;             // MODE_INFER
    float* dQ;            // nullable
    float* row_cos;       // nullable
    float* loss_part;     // [blocks]
    const void* Kb;
    const void* Vb;
    const void* Vt;
    const void* Ktp;
    const uint8_t* Vt8;     // FP8 forward: V^T / s^V as E4M3 [D, Mp]
    const float* sv_fold;   // FP8 forward: s^V_j * 448 / max_j s^V_j   [Mp]
    const float* fp8_unscale;  // FP8 forward: max_j s^V_j / 448         [1]
    float* M2;  // [blocks, 32]      row max of the logits in log2 units, per pixel
    void* Gt;   // [blocks, D, 32]   G^T
    void* St;   // [blocks, Mp, 32]  dS^T
    void* Qt;   // [blocks, 32, 32]  Q^T (rows >= d zero)
};

// Chunks of fragments kept in flight by the contraction loops (a ring of
// registers): two where two waves share a SIMD, four in the instantiations
// whose registers allow one wave per SIMD anyway (E4M3, or more than four D
// tiles per wave), where the ring alone has to cover the L2 latency.  Callers
// rely on the depth dividing 4 (the chunk counts are multiples of 4).
template <bool DEEP>
constexpr int pipe_depth()
{
    return DEEP ? 4 : 2;
}

// Depth of the uniform rings (the F contraction's V^T and weight fragments
// together, and the 32-pixel block's dP loop): deep where one wave per SIMD
// is all the registers allow.  The 64-pixel block keeps two waves per SIMD:
// it takes the short ring where a deep one would not fit, and its dP loop and
// its F contraction at four D tiles a wave have rings of their own.
template <bool F8, int NT, int NPG, int NW>
constexpr bool kDeepRing = (F8 || NT * NPG > 4) && !(NW == 8 && (NT * NPG >= 8 || (F8 && NT >= 2)));

// Workgroup shape of k_dec_rows: NW waves and NPG groups of 32 pixels.  Every
// wave covers all NPG x 32 pixels of the block and 1 / NW of the D columns
// (NT = D / (32 NW) tiles of 32) in the F contraction, and the atom tiles
// w, w + NW, ... in the logits and dP contractions, so each V fragment it loads
// feeds NPG MFMAs (with NPG = 1, two atom tiles share each G fragment instead).
template <class P, int NT, int DQ, int MODE, bool F8, int NW, int NPG>
__global__ __launch_bounds__(NW * kWave) void k_dec_rows(RowsArgs a)
{
    using T = typename P::T;
    using Frag = typename P::Frag;
    constexpr int NQ = DQ / 16;           // K chunks of the logits contraction
    constexpr int BPX = kPx * NPG;        // pixels per workgroup
    constexpr int NTH = NW * kWave;       // threads per workgroup
    constexpr int TT = NPG == 1 ? 2 : 1;  // atom tiles per dP iteration
    extern __shared__ __align__(16) char smem[];
    // LDS: red [4][NW][BPX] floats of per-pixel statistics, the waves' dS
    // staging tiles [NW][32][kScLd] (before the dP loop the E4M3 V scales
    // [Mp] floats), then region X (P~ [BPX][Mp+8], later
    // G [BPX][D+8], later the dQ reduction [NW][32][BPX + 2] floats)
    const int w = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    float* red = reinterpret_cast<float*>(smem);
    T* Wsc = reinterpret_cast<T*>(smem + 4 * NW * BPX * sizeof(float)) + w * kPx * kScLd;
    T* X = reinterpret_cast<T*>(smem + 4 * NW * BPX * sizeof(float) + NW * kPx * kScLd * sizeof(T));
    auto rslot = [&](int set, int ww, int g) { return red + (set * NW + ww) * BPX + g * kPx; };
    const int ldp = a.Mp + 8, ldg = a.D + 8;

    const int col = lane & 31, h = lane >> 5;
    const int blk = blockIdx.x;
    const int ntiles = a.Mp / 32;
    const int nca = a.Mp / 16;  // 16-wide K chunks over the atoms (a multiple of 4)
    const int ncd = a.D / 16;   // 16-wide K chunks over the features (a multiple of 8)
    int pxg[NPG];
    bool valid[NPG];
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        pxg[g] = (blk * NPG + g) * kPx + col;
        valid[g] = pxg[g] < a.n;
    }

    const T* Kb = reinterpret_cast<const T*>(a.Kb);
    const T* Vb = reinterpret_cast<const T*>(a.Vb);
    const T* Vt = reinterpret_cast<const T*>(a.Vt);
    const T* Ktp = reinterpret_cast<const T*>(a.Ktp);

    // query fragments (B operand of S^T = K Q^T): Q[px][16 c + 8 h + t].  They
    // are loaded again for the dP loop rather than held across the F
    // contraction, whose registers they would take (the rows are in L2).
    Frag qf[NPG][NQ];
    auto load_qf = [&]() {
#pragma unroll
        for (int g = 0; g < NPG; ++g)
#pragma unroll
            for (int c = 0; c < NQ; ++c) {
                float v[8];
                if (valid[g]) {
                    const float4* qp = reinterpret_cast<const float4*>(a.Q + (size_t)pxg[g] * DQ + 16 * c + 8 * h);
                    const float4 x0 = qp[0], x1 = qp[1];
                    v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
                    v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
                } else {
#pragma unroll
                    for (int t = 0; t < 8; ++t) v[t] = 0.0f;
                }
                qf[g][c] = P::from_f32(v);
            }
    };
    load_qf();
    // Q^T of 32-pixel block g for the dK reduction, written by wave g (rows >= d zero)
    if (MODE != MODE_INFER) {
#pragma unroll
        for (int g = 0; g < NPG; ++g) {
            if (w != g) continue;
            T* qt = reinterpret_cast<T*>(a.Qt) + (size_t)(blk * NPG + g) * 32 * kPx;
#pragma unroll
            for (int c = 0; c < NQ; ++c)
#pragma unroll
                for (int t = 0; t < 8; ++t) qt[(16 * c + 8 * h + t) * kPx + col] = qf[g][c][t];
            if (DQ == 16) {
#pragma unroll
                for (int t = 0; t < 8; ++t) qt[(16 + 8 * h + t) * kPx + col] = P::cvt(0.0f);
            }
        }
    }

    auto kload = [&](int tt, Frag* kf) {
#pragma unroll
        for (int c = 0; c < NQ; ++c) kf[c] = load_frag<P>(Kb, tt, c, NQ, lane);
    };
    auto s_of = [&](const Frag* kf, int g) {
        f32x16 s = {};
#pragma unroll
        for (int c = 0; c < NQ; ++c) P::mma(s, kf[c], qf[g][c]);
        return s;
    };
    // Visit the wave's atom tiles w, w + NW, ... with their K fragments; those
    // of the next tile are in flight while one is processed.
    auto for_tiles = [&](auto&& body) {
        Frag ka[NQ], kb[NQ];
        if (w < ntiles) kload(w, ka);
        for (int tt = w; tt < ntiles; tt += 2 * NW) {
            if (tt + NW < ntiles) kload(tt + NW, kb);
            body(tt, ka);
            if (tt + 2 * NW < ntiles) kload(tt + 2 * NW, ka);
            if (tt + NW < ntiles) body(tt + NW, kb);
        }
    };

    // The E4M3 weights' per-atom V scales, read once per atom tile in pass 2,
    // staged in the dS scratch region (unused before the dP loop; pass 1's
    // barriers come first), which holds the largest Mp (2048) floats.
    static_assert(!F8 || NW * kPx * kScLd * sizeof(T) >= 2048 * sizeof(float), "V scales fit the dS scratch");
    float* svs = reinterpret_cast<float*>(smem + 4 * NW * BPX * sizeof(float));
    if (F8) {
        for (int i = threadIdx.x; i < a.Mp; i += NTH) svs[i] = a.sv_fold[i];
    }
    // ---- pass 1: row max of the logits (in log2 units)
    float mx[NPG];
#pragma unroll
    for (int g = 0; g < NPG; ++g) mx[g] = -INFINITY;
    for_tiles([&](int tt, const Frag* kf) {
#pragma unroll
        for (int g = 0; g < NPG; ++g) {
            const f32x16 s = s_of(kf, g);
            if (32 * tt + 32 <= a.M) {  // every atom of the tile exists
#pragma unroll
                for (int r = 0; r < 16; ++r) mx[g] = fmaxf(mx[g], s[r]);
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (32 * tt + crow(r, h) < a.M) mx[g] = fmaxf(mx[g], s[r]);
            }
        }
    });
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        mx[g] = fmaxf(mx[g], __shfl_xor(mx[g], 32, kWave));
        if (h == 0) rslot(0, w, g)[col] = mx[g];
    }
    __syncthreads();
    float m2[NPG];
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        float m = -INFINITY;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) m = fmaxf(m, rslot(0, ww, g)[col]);
        m2[g] = m * a.scale_log2;
    }
    __syncthreads();

    // ---- pass 2: P~ = exp2(S scale - m) into LDS [px][atom]
    float lsum[NPG];
#pragma unroll
    for (int g = 0; g < NPG; ++g) lsum[g] = 0.0f;
    for_tiles([&](int tt, const Frag* kf) {
#pragma unroll
        for (int g = 0; g < NPG; ++g) {
            const f32x16 s = s_of(kf, g);
            float p[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) p[r] = exp2_weight(s[r] * a.scale_log2 - m2[g]);
            if (32 * tt + 32 > a.M) {  // padded atoms get no weight
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (32 * tt + crow(r, h) >= a.M) p[r] = 0.0f;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) lsum[g] += p[r];
            const int prow = g * kPx + col;
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
                const int atom0 = 32 * tt + 8 * g4 + 4 * h;
                if (F8) {
                    // P~ of a pixel peaks at exactly 1, so with the V row scales folded
                    // into its columns one fixed factor maps it onto the E4M3 range.
                    // The weights go in as two E4M3 terms, the rounded value and the
                    // rounded residual (relative error 2^-8 instead of 2^-4), so
                    // that F carries only the E4M3 rounding of V.
                    const float4 sv = *reinterpret_cast<const float4*>(svs + atom0);
                    const float q0 = p[4 * g4] * sv.x, q1 = p[4 * g4 + 1] * sv.y;
                    const float q2 = p[4 * g4 + 2] * sv.z, q3 = p[4 * g4 + 3] * sv.w;
                    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(q0, q1, 0, false);
                    hi = __builtin_amdgcn_cvt_pk_fp8_f32(q2, q3, hi, true);
                    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(q0 - __builtin_amdgcn_cvt_f32_fp8(hi, 0),
                                                             q1 - __builtin_amdgcn_cvt_f32_fp8(hi, 1), 0, false);
                    lo = __builtin_amdgcn_cvt_pk_fp8_f32(q2 - __builtin_amdgcn_cvt_f32_fp8(hi, 2),
                                                         q3 - __builtin_amdgcn_cvt_f32_fp8(hi, 3), lo, true);
                    uint8_t* X8 = reinterpret_cast<uint8_t*>(X);
                    *reinterpret_cast<int*>(X8 + prow * (a.Mp + 16) + atom0) = hi;
                    *reinterpret_cast<int*>(X8 + (BPX + prow) * (a.Mp + 16) + atom0) = lo;
                } else {
                    P::store4(X + prow * ldp + atom0, p[4 * g4], p[4 * g4 + 1], p[4 * g4 + 2], p[4 * g4 + 3]);
                }
            }
        }
    });
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        lsum[g] += __shfl_xor(lsum[g], 32, kWave);
        if (h == 0) rslot(1, w, g)[col] = lsum[g];
    }
    __syncthreads();
    float invl[NPG];
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        float l = 0.0f;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) l += rslot(1, ww, g)[col];
        invl[g] = 1.0f / l;
    }
    // the row max of every pixel (past n too) for k_dec_dv, which rebuilds P~
    if (MODE != MODE_INFER && w == 0 && h == 0) {
#pragma unroll
        for (int g = 0; g < NPG; ++g) a.M2[(blk * NPG + g) * kPx + col] = m2[g];
    }

    // ---- F^T = V^T P~^T: wave w owns D tiles [w NT, w NT + NT) for every pixel group
    f32x16 acc[NT][NPG];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int g = 0; g < NPG; ++g) acc[t][g] = f32x16{};
    if (F8) {
        // K = 64 atoms per E4M3 MFMA; lane half h holds atoms 32 h + 0..31.
        // Two chunks in flight; the chunk count Mp / 64 may be odd.
        const int nc8 = a.Mp / 64;
        // the weights' E4M3 terms: part 0 the rounded values, part 1 the residuals
        auto bload = [&](int c, int g, int part) {
            const uint8_t* X8 = reinterpret_cast<const uint8_t*>(X) + (part * BPX + g * kPx + col) * (a.Mp + 16);
            const i32x4 b0 = *reinterpret_cast<const i32x4*>(X8 + 64 * c + 32 * h);
            const i32x4 b1 = *reinterpret_cast<const i32x4*>(X8 + 64 * c + 32 * h + 16);
            const i32x8 bf = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
            return bf;
        };
        // the D tiles of a sweep over the atoms: a divisor of NT, at most four
        // (the ring then holds at most 64 registers); the 64-pixel block takes
        // at most two per sweep and loads the weights' fragments from LDS just
        // before their MFMAs (one buffer, the other wave of the SIMD covering
        // the LDS latency), which keeps it within two waves per SIMD
        constexpr bool kWideF8 = NW == 8;
        constexpr int NH = kWideF8 ? (NT % 2 == 0 ? 2 : 1)
                                   : (NT % 4 == 0 ? 4 : (NT % 3 == 0 ? 3 : (NT % 2 == 0 ? 2 : 1)));
        static_assert(NT % NH == 0, "whole sweeps");
#pragma unroll
        for (int t0 = 0; t0 < NT; t0 += NH) {
            i32x8 ra[NH], rb[NH], ba[kWideF8 ? 1 : NPG][2], bb[kWideF8 ? 1 : NPG][2];
            auto vload = [&](int c, i32x8* af) {
#pragma unroll
                for (int t = 0; t < NH; ++t)
                    af[t] = *reinterpret_cast<const i32x8*>(
                        a.Vt8 + ((((size_t)(w * NT + t0 + t) * nc8 + c) << 6) + lane) * 32);
            };
            auto mma8 = [&](const i32x8* af, const i32x8 (*bf)[2]) {
#pragma unroll
                for (int t = 0; t < NH; ++t)
#pragma unroll
                    for (int g = 0; g < NPG; ++g)
#pragma unroll
                        for (int part = 0; part < 2; ++part)
                            acc[t0 + t][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                af[t], bf[g][part], acc[t0 + t][g], 0, 0, 0, 127, 0, 127);
            };
            auto pload = [&](int c, i32x8 (*bf)[2]) {
#pragma unroll
                for (int g = 0; g < NPG; ++g)
#pragma unroll
                    for (int part = 0; part < 2; ++part) bf[g][part] = bload(c, g, part);
            };
            if constexpr (kWideF8) {
                // one E4M3 term of both pixel groups at a time
                auto mma8p = [&](int c, const i32x8* af) {
#pragma unroll
                    for (int part = 0; part < 2; ++part) {
                        i32x8 bp[NPG];
#pragma unroll
                        for (int g = 0; g < NPG; ++g) bp[g] = bload(c, g, part);
#pragma unroll
                        for (int t = 0; t < NH; ++t)
#pragma unroll
                            for (int g = 0; g < NPG; ++g)
                                acc[t0 + t][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                                    af[t], bp[g], acc[t0 + t][g], 0, 0, 0, 127, 0, 127);
                    }
                };
                vload(0, ra);
                for (int c = 0; c < nc8; c += 2) {
                    if (c + 1 < nc8) vload(c + 1, rb);
                    mma8p(c, ra);
                    if (c + 2 < nc8) vload(c + 2, ra);
                    if (c + 1 < nc8) mma8p(c + 1, rb);
                }
            } else {
                vload(0, ra);
                pload(0, ba);
                for (int c = 0; c < nc8; c += 2) {
                    if (c + 1 < nc8) {
                        vload(c + 1, rb);
                        pload(c + 1, bb);
                    }
                    mma8(ra, ba);
                    if (c + 2 < nc8) {
                        vload(c + 2, ra);
                        pload(c + 2, ba);
                    }
                    if (c + 1 < nc8) mma8(rb, bb);
                }
            }
        }
    } else {
        if constexpr (NW == 8 && NT * NPG >= 8) {
            // the 64-pixel block with four D tiles a wave, whose uniform ring
            // could only be two deep: V^T chunks four deep instead, and the
            // weights' fragments read from LDS just before their MFMAs (the
            // SIMD's other wave covers that latency), as in the E4M3 product
            constexpr int PF = 4;
            Frag vr[PF][NT];
            auto vget = [&](int c, Frag* r) {
#pragma unroll
                for (int t = 0; t < NT; ++t) r[t] = load_frag<P>(Vt, w * NT + t, c, nca, lane);
            };
#pragma unroll
            for (int s = 0; s < PF - 1; ++s)
                if (s < nca) vget(s, vr[s]);
            for (int c0 = 0; c0 < nca; c0 += PF) {
#pragma unroll
                for (int s = 0; s < PF; ++s) {
                    const int c = c0 + s;
                    if (c < nca) {
                        if (c + PF - 1 < nca) vget(c + PF - 1, vr[(s + PF - 1) % PF]);
                        Frag b[NPG];
#pragma unroll
                        for (int g = 0; g < NPG; ++g) b[g] = P::load(X + (g * kPx + col) * ldp + 16 * c + 8 * h);
#pragma unroll
                        for (int t = 0; t < NT; ++t)
#pragma unroll
                            for (int g = 0; g < NPG; ++g) P::mma(acc[t][g], vr[s][t], b[g]);
                    }
                }
            }
        } else {
            // ring of PD chunks: chunk c + PD - 1 is loaded while chunk c is
            // multiplied.  The loads are unconditional (the last PD chunks are
            // peeled) so that each MFMA waits only for its own fragments.
            constexpr int PD = pipe_depth<kDeepRing<F8, NT, NPG, NW>>();
            Frag ring[PD][NT], bring[PD][NPG];
            auto fetch = [&](int c, Frag* r, Frag* b) {
#pragma unroll
                for (int t = 0; t < NT; ++t) r[t] = load_frag<P>(Vt, w * NT + t, c, nca, lane);
#pragma unroll
                for (int g = 0; g < NPG; ++g) b[g] = P::load(X + (g * kPx + col) * ldp + 16 * c + 8 * h);
            };
            auto mma = [&](const Frag* r, const Frag* b) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int g = 0; g < NPG; ++g) P::mma(acc[t][g], r[t], b[g]);
            };
#pragma unroll
            for (int s = 0; s < PD - 1; ++s) fetch(s, ring[s], bring[s]);
            for (int c0 = 0; c0 < nca - PD; c0 += PD) {
#pragma unroll
                for (int s = 0; s < PD; ++s) {
                    fetch(c0 + s + PD - 1, ring[(s + PD - 1) % PD], bring[(s + PD - 1) % PD]);
                    mma(ring[s], bring[s]);
                }
            }
            fetch(nca - 1, ring[PD - 1], bring[PD - 1]);
#pragma unroll
            for (int s = 0; s < PD; ++s) mma(ring[s], bring[s]);
        }
    }
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        const float fscale = F8 ? invl[g] * a.fp8_unscale[0] : invl[g];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][g][r] *= fscale;
    }

    if (MODE == MODE_INFER) {
#pragma unroll
        for (int g = 0; g < NPG; ++g) {
            if (!valid[g]) continue;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int g4 = 0; g4 < 4; ++g4) {
                    const int dr = 32 * (w * NT + t) + 8 * g4 + 4 * h;
                    *reinterpret_cast<float4*>(a.F + (size_t)pxg[g] * a.D + dr) =
                        make_float4(acc[t][g][4 * g4], acc[t][g][4 * g4 + 1], acc[t][g][4 * g4 + 2],
                                    acc[t][g][4 * g4 + 3]);
                }
        }
        return;
    }

    // ---- epilogue: cosine loss gradient (LOSS) or upstream dF (ADJ), G = dL/dF / l.
    // The target (or dF) rows feed the row statistics and, once those are
    // reduced over the waves, G.  All rows are held in registers from one read
    // (kHold), except in the 64-pixel block with four D tiles per wave, whose
    // registers fit two waves per SIMD only without them: that shape reduces
    // the statistics one 32-pixel group at a time (one barrier each) and reads
    // the group's rows again right after, while they are still in L2 (a
    // 128 KB working set per workgroup instead of 256 KB read twice far
    // apart).
    // (Requesting these rows before the F contraction is slower: loads retire in
    // order, so every fragment wait of the contraction would wait for them.)
    // A pixel past n reads row n - 1, unused since its G is zeroed through ca, cb.
    constexpr bool kHold = !(NW == 8 && NT * NPG >= 8);
    const float* rowsrc = MODE == MODE_LOSS ? a.target : a.dF;
    auto row_frag = [&](int g, int t, float* x16) {
        const float* prow = rowsrc + (size_t)(valid[g] ? pxg[g] : a.n - 1) * a.D + 32 * (w * NT + t) + 4 * h;
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            const float4 x = *reinterpret_cast<const float4*>(prow + 8 * g4);
            x16[4 * g4] = x.x; x16[4 * g4 + 1] = x.y; x16[4 * g4 + 2] = x.z; x16[4 * g4 + 3] = x.w;
        }
    };
    float delta[NPG], ca[NPG], cb[NPG];  // G = ca * row + cb * F (zero past n)
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        delta[g] = 0.0f;
        ca[g] = valid[g] ? invl[g] : 0.0f;
        cb[g] = 0.0f;
    }
    // row statistics of pixel group g over this wave's D tiles, into its
    // slots; rows(t, x) yields the group's rows of D tile t
    auto stats_put = [&](int g, auto&& rows) {
        float nf = 0.0f, ft = 0.0f, nt = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float x[16];
            rows(t, x);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                nf += acc[t][g][r] * acc[t][g][r];
                ft += acc[t][g][r] * x[r];
                nt += x[r] * x[r];
            }
        }
        nf += __shfl_xor(nf, 32, kWave);
        ft += __shfl_xor(ft, 32, kWave);
        nt += __shfl_xor(nt, 32, kWave);
        if (h == 0) {
            rslot(0, w, g)[col] = nf;
            rslot(1, w, g)[col] = ft;
            rslot(2, w, g)[col] = nt;
        }
    };
    // the reduced statistics of group g: the cosine, the loss and ca, cb
    auto stats_take = [&](int g) {
        float sf = 0.f, st = 0.f, stt = 0.f;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            sf += rslot(0, ww, g)[col];
            st += rslot(1, ww, g)[col];
            stt += rslot(2, ww, g)[col];
        }
        const float raw = sqrtf(sf) * sqrtf(stt);
        const float den = fmaxf(raw, 1e-8f);
        const float cs = st / den;
        // dL/dF = lam_cos (-(1/n) (T / den - c F / |F|^2)) + lam_l2 (2/n) (F - T),
        // then divided by l
        const float l2 = 2.0f * a.lam_l2 * a.inv_n;
        ca[g] = valid[g] ? (-a.lam_cos * a.inv_n / den - l2) * invl[g] : 0.0f;
        cb[g] = valid[g] ? (((raw > 1e-8f && sf > 0.f) ? a.lam_cos * a.inv_n * cs / sf : 0.0f) + l2) * invl[g]
                         : 0.0f;
        if (w == g && h == 0) {
            if (a.row_cos && valid[g]) a.row_cos[pxg[g]] = cs;
            // sum of the pixel losses over the valid pixels of 32-pixel block g
            float lp = valid[g] ? a.lam_cos * (1.0f - cs) + a.lam_l2 * (sf - 2.0f * st + stt) : 0.0f;
            for (int o = 16; o >= 1; o >>= 1) lp += __shfl_xor(lp, o, kWave);
            if (col == 0) a.loss_part[blk * NPG + g] = lp;
        }
    };
    // G of group g from its rows, staged into LDS [px][D]; delta' = sum_D G F
    // (zero for the pure cosine term up to rounding)
    auto stage_g = [&](int g, auto&& rows) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float x[16], gv[16];
            rows(t, x);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                gv[r] = ca[g] * x[r] + cb[g] * acc[t][g][r];
                delta[g] += gv[r] * acc[t][g][r];
            }
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
                const int dr = 32 * (w * NT + t) + 8 * g4 + 4 * h;
                P::store4(X + (g * kPx + col) * ldg + dr, gv[4 * g4], gv[4 * g4 + 1], gv[4 * g4 + 2], gv[4 * g4 + 3]);
            }
        }
        delta[g] += __shfl_xor(delta[g], 32, kWave);
    };
    if constexpr (kHold) {
        float held[NPG][NT][16];
#pragma unroll
        for (int g = 0; g < NPG; ++g)
#pragma unroll
            for (int t = 0; t < NT; ++t) row_frag(g, t, held[g][t]);
        if (MODE == MODE_LOSS) {
            float nf[NPG], ft[NPG], nt[NPG];
#pragma unroll
            for (int g = 0; g < NPG; ++g) {
                nf[g] = ft[g] = nt[g] = 0.0f;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        nf[g] += acc[t][g][r] * acc[t][g][r];
                        ft[g] += acc[t][g][r] * held[g][t][r];
                        nt[g] += held[g][t][r] * held[g][t][r];
                    }
                nf[g] += __shfl_xor(nf[g], 32, kWave);
                ft[g] += __shfl_xor(ft[g], 32, kWave);
                nt[g] += __shfl_xor(nt[g], 32, kWave);
            }
            __syncthreads();  // every wave is done reading the row sums of pass 2
            if (h == 0) {
#pragma unroll
                for (int g = 0; g < NPG; ++g) {
                    rslot(0, w, g)[col] = nf[g];
                    rslot(1, w, g)[col] = ft[g];
                    rslot(2, w, g)[col] = nt[g];
                }
            }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < NPG; ++g) stats_take(g);
        }
        __syncthreads();  // everyone is done reading P~ (region X) and the statistics
#pragma unroll
        for (int g = 0; g < NPG; ++g) {
            auto rows = [&](int t, float* x) {
#pragma unroll
                for (int r = 0; r < 16; ++r) x[r] = held[g][t][r];
            };
            stage_g(g, rows);
        }
    } else {
        __syncthreads();  // as above
#pragma unroll
        for (int g = 0; g < NPG; ++g) {
            auto rows = [&](int t, float* x) { row_frag(g, t, x); };
            if (MODE == MODE_LOSS) {
                stats_put(g, rows);
                __syncthreads();
                stats_take(g);
            }
            stage_g(g, rows);
        }
    }
    if (h == 0) {
#pragma unroll
        for (int g = 0; g < NPG; ++g) rslot(3, w, g)[col] = delta[g];
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        float s = 0.0f;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) s += rslot(3, ww, g)[col];
        delta[g] = s;
    }
    // G^T of this wave's D rows from the LDS copy, in whole chunks, pixels in the
    // perm16 order of k_dec_dv's P~ fragments
#pragma unroll
    for (int g = 0; g < NPG; ++g) {
        T* Gt = reinterpret_cast<T*>(a.Gt) + ((size_t)(blk * NPG + g) * a.D + 32 * w * NT) * kPx;
        store_transposed<P, true>(X + g * kPx * ldg + 32 * w * NT, ldg, 32 * NT, Gt, lane, kWave);
    }

    // ---- per atom tile: dP = G V^T, dS = P~ (dP - delta) / sqrt(d), dQ^T += K^T dS^T
    load_qf();
    f32x16 dq[NPG];
#pragma unroll
    for (int g = 0; g < NPG; ++g) dq[g] = f32x16{};
    T* Stb = reinterpret_cast<T*>(a.St) + (size_t)blk * NPG * a.Mp * kPx;
    auto finish_tile = [&](int tt, int g, const f32x16& dp, const Frag* kf, const Frag* kt) {
        const f32x16 s = s_of(kf, g);
        // A pixel past n has G = 0, hence dP = 0 and delta = 0, so its dS is
        // zero without a mask; padded atoms are masked.
        float ds[16];
#pragma unroll
        for (int r = 0; r < 16; ++r)
            ds[r] = exp2_weight(s[r] * a.scale_log2 - m2[g]) * (dp[r] - delta[g]) * a.inv_sqrt_d;
        if (32 * tt + 32 > a.M) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (32 * tt + crow(r, h) >= a.M) ds[r] = 0.0f;
        }
        // dS^T of the tile through the wave's scratch [px][atom], in whole chunks
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4)
            P::store4(Wsc + col * kScLd + 8 * g4 + 4 * h, ds[4 * g4], ds[4 * g4 + 1], ds[4 * g4 + 2], ds[4 * g4 + 3]);
        __builtin_amdgcn_wave_barrier();
        store_transposed<P>(Wsc, kScLd, 32, Stb + ((size_t)g * a.Mp + 32 * tt) * kPx, lane, kWave);
        __builtin_amdgcn_wave_barrier();
        if (a.dQ) {  // no dQ requested (the decode-only iterations): skip its products
#pragma unroll
            for (int c = 0; c < 2; ++c) P::mma(dq[g], kt[c], P::from_f32(ds + 8 * c));
        }
    };
    // TT atom tiles per iteration share each G fragment read from LDS, and each
    // V fragment feeds the NPG pixel groups; the V fragments (from L2) run PV
    // chunks ahead of the MFMAs and the G fragments (from LDS) PGD chunks, and
    // the K fragments of the dS step are requested before the contraction that
    // hides their latency.  The 8-wave block has registers to spare in this
    // loop (not in the F contraction), so its V ring is 8 chunks deep: the two
    // MFMAs of a chunk are far shorter than an L2 round trip.  Its D is a
    // multiple of 256, so the 16-wide chunk count ncd is a multiple of PV.
    constexpr int PV = NW == 8 ? 8 : pipe_depth<kDeepRing<F8, NT, NPG, NW>>();
    constexpr int PGD = NW == 8 ? 2 : PV;
    static_assert(PGD >= 2 && PV % PGD == 0, "G ring within the V ring");
    for (int tt = w; tt < ntiles; tt += TT * NW) {
        bool has[TT];
        int tj[TT];
#pragma unroll
        for (int j = 0; j < TT; ++j) {
            has[j] = tt + j * NW < ntiles;
            // a missing tile repeats the first one (multiplied, never used),
            // which keeps the loop free of branches
            tj[j] = has[j] ? tt + j * NW : tt;
        }
        Frag kf[TT][NQ], kt[TT][2];
#pragma unroll
        for (int j = 0; j < TT; ++j) {
            kload(tj[j], kf[j]);
#pragma unroll
            for (int c = 0; c < 2; ++c) kt[j][c] = load_frag<P>(Ktp, 0, 2 * tj[j] + c, nca, lane);
        }
        f32x16 dp[TT][NPG];
#pragma unroll
        for (int j = 0; j < TT; ++j)
#pragma unroll
            for (int g = 0; g < NPG; ++g) dp[j][g] = f32x16{};
        Frag rv[PV][TT], gb[PGD][NPG];
        auto vfetch = [&](int c, Frag* v) {
#pragma unroll
            for (int j = 0; j < TT; ++j) v[j] = load_frag<P>(Vb, tj[j], c, ncd, lane);
        };
        auto gfetch = [&](int c, Frag* gg) {
#pragma unroll
            for (int g = 0; g < NPG; ++g) gg[g] = P::load(X + (g * kPx + col) * ldg + 16 * c + 8 * h);
        };
        auto mma = [&](const Frag* v, const Frag* gg) {
#pragma unroll
            for (int j = 0; j < TT; ++j)
#pragma unroll
                for (int g = 0; g < NPG; ++g) P::mma(dp[j][g], v[j], gg[g]);
        };
#pragma unroll
        for (int s = 0; s < PV - 1; ++s) vfetch(s, rv[s]);
#pragma unroll
        for (int s = 0; s < PGD - 1; ++s) gfetch(s, gb[s]);
        for (int c0 = 0; c0 < ncd - PV; c0 += PV) {
#pragma unroll
            for (int s = 0; s < PV; ++s) {
                vfetch(c0 + s + PV - 1, rv[(s + PV - 1) % PV]);
                gfetch(c0 + s + PGD - 1, gb[(s + PGD - 1) % PGD]);
                mma(rv[s], gb[s % PGD]);
            }
        }
        vfetch(ncd - 1, rv[PV - 1]);
#pragma unroll
        for (int s = 0; s < PV; ++s) {
            if (s + PGD - 1 < PV) gfetch(ncd - PV + s + PGD - 1, gb[(s + PGD - 1) % PGD]);
            mma(rv[s], gb[s % PGD]);
        }
#pragma unroll
        for (int j = 0; j < TT; ++j)
            if (has[j]) {
#pragma unroll
                for (int g = 0; g < NPG; ++g) finish_tile(tj[j], g, dp[j][g], kf[j], kt[j]);
            }
    }
    if (!a.dQ) return;
    __syncthreads();  // region X (G) no longer read
    // [NW][32][BPX + 2] floats: with the two-float pad the reads below, 32
    // lanes of one pixel at consecutive k, fall on banks 2 k + p, distinct over
    // the wave (unpadded, a pixel's 32 lanes would share one bank)
    constexpr int RLD = BPX + 2;
    float* dqr = reinterpret_cast<float*>(X);
#pragma unroll
    for (int g = 0; g < NPG; ++g)
#pragma unroll
        for (int r = 0; r < 16; ++r) dqr[(w * 32 + crow(r, h)) * RLD + g * kPx + col] = dq[g][r];
    __syncthreads();
    for (int i = threadIdx.x; i < BPX * DQ; i += NTH) {
        const int p = i / DQ, k = i % DQ;
        float v = 0.0f;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) v += dqr[(ww * 32 + k) * RLD + p];
        const int gp = blk * BPX + p;
        if (gp < a.n) a.dQ[(size_t)gp * DQ + k] = v;
    }
}

// ------------------------------------------------------------ split-K TN GEMM

// C_part[split][i][j] = sum over the split's pixel blocks of A^T[i][p] B^T[j][p]
// with A^T, B^T in the pixel-blocked transposed layout X^T[blk][row][32].
// A wave owns WI x WJ result tiles of 32 x 32, the 4 waves are arranged
// WVI x WVJ, so a workgroup covers (32 WI WVI) x (32 WJ WVJ); rowsA must be a
// multiple of 32 WI and rowsB of 32 WJ.  The fragments of RB pixel blocks are in
// flight at once (a ring of registers, loads never skipped so that each MFMA
// waits only for its own block).  The grid is tiles x splits, mapped so that
// the tiles of one split share an XCD.
template <class P, int WI, int WJ, int WVI, int WVJ>
__global__ __launch_bounds__(256) void k_dec_tn(const void* At_, int rowsA, const void* Bt_, int rowsB,
                                                int nblocks, int splits, int tiles_i, int tiles_j,
                                                float* __restrict__ part)
{
    static_assert(WVI * WVJ == 4, "four waves");
    using T = typename P::T;
    using Frag = typename P::Frag;
    constexpr int kFragRegs = (int)(sizeof(Frag) / 4);
    constexpr int RB = 2 * (WI + WJ) * kFragRegs * 4 <= 128 ? 4 : 2;
    const T* At = reinterpret_cast<const T*>(At_);
    const T* Bt = reinterpret_cast<const T*>(Bt_);
    const int ntiles = tiles_i * tiles_j;
    const int b = blockIdx.x;
    const int xcd = b % 8, idx = b / 8;
    const int split = (idx / ntiles) * 8 + xcd;
    const int tile = idx % ntiles;
    if (split >= splits) return;
    const int ti = tile / tiles_j, tj = tile % tiles_j;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int col = lane & 31, h = lane >> 5;
    const int i0 = (ti * WVI + w / WVJ) * WI * 32, j0 = (tj * WVJ + w % WVJ) * WJ * 32;
    if (i0 >= rowsA || j0 >= rowsB) return;
    const int per = (nblocks + splits - 1) / splits;
    const int b0 = split * per, b1 = min(nblocks, b0 + per);
    f32x16 c[WI][WJ];
#pragma unroll
    for (int a = 0; a < WI; ++a)
#pragma unroll
        for (int q = 0; q < WJ; ++q) c[a][q] = f32x16{};
    Frag fa[RB][2 * WI], fb[RB][2 * WJ];
    auto load = [&](int blk, Frag* xa, Frag* xb) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
#pragma unroll
            for (int a = 0; a < WI; ++a)
                xa[k * WI + a] = P::load(At + ((size_t)blk * rowsA + i0 + 32 * a + col) * kPx + 16 * k + 8 * h);
#pragma unroll
            for (int q = 0; q < WJ; ++q)
                xb[k * WJ + q] = P::load(Bt + ((size_t)blk * rowsB + j0 + 32 * q + col) * kPx + 16 * k + 8 * h);
        }
    };
    auto mma = [&](const Frag* xa, const Frag* xb) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int a = 0; a < WI; ++a)
#pragma unroll
                for (int q = 0; q < WJ; ++q) P::mma(c[a][q], xa[k * WI + a], xb[k * WJ + q]);
    };
    // whole groups of RB blocks through the ring, the rest one at a time
    const int nfull = b1 > b0 ? (b1 - b0) / RB * RB : 0;
    if (nfull > 0) {
#pragma unroll
        for (int s = 0; s < RB - 1; ++s) load(b0 + s, fa[s], fb[s]);
        for (int base = b0; base < b0 + nfull - RB; base += RB) {
#pragma unroll
            for (int s = 0; s < RB; ++s) {
                const int sl = (s + RB - 1) % RB;
                load(base + s + RB - 1, fa[sl], fb[sl]);
                mma(fa[s], fb[s]);
            }
        }
        load(b0 + nfull - 1, fa[RB - 1], fb[RB - 1]);
#pragma unroll
        for (int s = 0; s < RB; ++s) mma(fa[s], fb[s]);
    }
    for (int blk = b0 + nfull; blk < b1; ++blk) {
        load(blk, fa[0], fb[0]);
        mma(fa[0], fb[0]);
    }
    float* out = part + (size_t)split * rowsA * rowsB;
#pragma unroll
    for (int a = 0; a < WI; ++a)
#pragma unroll
        for (int q = 0; q < WJ; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                out[(size_t)(i0 + 32 * a + crow(r, h)) * rowsB + j0 + 32 * q + col] = c[a][q][r];
}

// dV partials with P~ rebuilt instead of read: C_part[split][i][j] = sum over
// the split's 32-pixel blocks of P~[px][i] G[px][j].  Per block the wave's two
// atom tiles of S = Q K^T come from MFMA with the pixel as the row, so a lane
// holds one atom and 16 pixels (rows crow(r, h)); P~ = exp2(S log2(e)/sqrt(d)
// - m2[px]) with the row max k_dec_rows saved, and result registers 8k..8k+7
// are directly the A fragment of pixel chunk k in perm16 order, the order in
// which k_dec_rows stores G^T.  Waves 2 x 2, each 64 atoms x 64 features; two
// blocks of Q, m2 and G^T fragments in flight; splits mapped as in k_dec_tn.
// dV split-K GEMM.  A workgroup owns 128 atoms x 128 QT feature columns and a
// range of pixel blocks.  Per block, wave w rebuilds P~ for atom tile w only
// (S = Q K^T with the pixel as the MFMA row, so each lane holds one atom and
// 16 pixels in perm16 order, then exp2 against the saved row max) and leaves
// it in LDS as the A fragments of the dV product; after one barrier every
// wave multiplies all four atom tiles by the G^T fragments of its own 32 QT
// columns.  P~ is thus computed once per (atom, pixel) and feature-column
// tile, and the LDS slots alternate between blocks so one barrier per block
// suffices (a wave can write slot b + 1 while a slower one still reads slot b,
// and cannot reach slot b + 2 before that wave has passed the barrier of b + 1).
template <class P, int DQ, int QT>
__global__ __launch_bounds__(256, P::kBytes == 2 ? 2 : 1) void k_dec_dv(const float* __restrict__ Q, int n, const void* Kb_, int M,
                                                const float* __restrict__ m2, float scale_log2, const void* Gt_,
                                                int Mp, int D, int nblocks, int splits, int tiles_i, int tiles_j,
                                                float* __restrict__ part)
{
    using T = typename P::T;
    using Frag = typename P::Frag;
    constexpr int NQ = DQ / 16;
    __shared__ __align__(32) T pf[2][4][2][kWave * 8];
    const T* Kb = reinterpret_cast<const T*>(Kb_);
    const T* Gt = reinterpret_cast<const T*>(Gt_);
    const int ntiles = tiles_i * tiles_j;
    const int b = blockIdx.x;
    const int xcd = b % 8, idx = b / 8;
    const int split = (idx / ntiles) * 8 + xcd;
    const int tile = idx % ntiles;
    if (split >= splits) return;  // whole workgroups
    const int ti = tile / tiles_j, tj = tile % tiles_j;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int col = lane & 31, h = lane >> 5;
    const int i0 = ti * 128;                       // the workgroup's atoms
    const int j0 = (tj * 4 + w) * 32 * QT;         // this wave's feature columns
    const int ntv = min(4, (Mp - i0) / 32);        // atom tiles inside Mp (Mp is a multiple of 64)
    const bool mine_ok = w < ntv;                  // the atom tile this wave rebuilds
    const int per = (nblocks + splits - 1) / splits;
    const int b0 = split * per, b1 = min(nblocks, b0 + per);

    Frag kf[NQ];
    const bool atom_ok = mine_ok && i0 + 32 * w + col < M;
#pragma unroll
    for (int c = 0; c < NQ; ++c) kf[c] = load_frag<P>(Kb, mine_ok ? i0 / 32 + w : 0, c, NQ, lane);
    f32x16 acc[4][QT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < QT; ++q) acc[t][q] = f32x16{};

    // one block's operands, requested a block ahead: the Q fragments of pixel
    // col (converted when their loads land; zero past n), the row max of pixel
    // col (the lane's 16 pixels take theirs by lane shuffles when used), and
    // the G^T fragments of this wave's columns.  Holding the converted
    // fragments and one row max per lane instead of the float rows and 16 row
    // maxima keeps the kernel within two waves per SIMD.
    struct Blk {
        Frag q[NQ];
        float m;
        Frag g[QT][2];
    };
    auto load = [&](int blk, Blk& B) {
        const int px = blk * kPx + col;
        const bool valid = px < n;
        const float* qrow = Q + (size_t)(valid ? px : n - 1) * DQ;
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
            const float4 x0 = *reinterpret_cast<const float4*>(qrow + 16 * c + 8 * h);
            const float4 x1 = *reinterpret_cast<const float4*>(qrow + 16 * c + 8 * h + 4);
            const float v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            float z[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) z[e] = valid ? v[e] : 0.0f;
            B.q[c] = P::from_f32(z);
        }
        B.m = m2[(size_t)blk * kPx + col];
#pragma unroll
        for (int q = 0; q < QT; ++q)
#pragma unroll
            for (int k = 0; k < 2; ++k)
                B.g[q][k] = P::load(Gt + ((size_t)blk * D + j0 + 32 * q + col) * kPx + 16 * k + 8 * h);
    };
    auto compute = [&](int blk, const Blk& B) {
        const int slot = blk & 1;
        {
            f32x16 sacc = {};
#pragma unroll
            for (int c = 0; c < NQ; ++c) P::mma(sacc, B.q[c], kf[c]);
            float p[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float mr = __shfl(B.m, crow(r, h), kWave);  // row max of the pixel in row crow(r, h)
                p[r] = atom_ok ? exp2_weight(sacc[r] * scale_log2 - mr) : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < 2; ++k)
                *reinterpret_cast<Frag*>(&pf[slot][w][k][lane * 8]) = P::from_f32(p + 8 * k);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < ntv) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const Frag af = *reinterpret_cast<const Frag*>(&pf[slot][t][k][lane * 8]);
#pragma unroll
                    for (int q = 0; q < QT; ++q) P::mma(acc[t][q], af, B.g[q][k]);
                }
            }
        }
    };
    if (b0 < b1) {
        Blk ring[2];
        load(b0, ring[0]);
        int blk = b0;
        for (; blk + 2 <= b1; blk += 2) {
            load(min(blk + 1, b1 - 1), ring[1]);
            compute(blk, ring[0]);
            load(min(blk + 2, b1 - 1), ring[0]);
            compute(blk + 1, ring[1]);
        }
        if (blk < b1) compute(blk, ring[0]);
    }
    float* out = part + (size_t)split * Mp * D;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (t < ntv)
#pragma unroll
            for (int q = 0; q < QT; ++q)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    out[(size_t)(i0 + 32 * t + crow(r, h)) * D + j0 + 32 * q + col] = acc[t][q][r];
}

// out[i][j] = sum_split part[split][i][j] (+ 2 lambda (K - K0)[i][j] for dK)
// for i < rows_out, j < cols_out (a multiple of 4); part has ld = ldp columns
// and rows_p rows per split.  A workgroup covers 64 groups of 4 consecutive
// outputs; wave w sums the splits w, w + 4, ... with four 16-byte loads in
// flight, and the four wave sums are added in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_dec_reduce(const float* __restrict__ part, int splits,
                                                    int rows_p, int ldp, int rows_out, int cols_out,
                                                    float* __restrict__ out, const float* __restrict__ K,
                                                    const float* __restrict__ K0, float two_lambda)
{
    __shared__ float4 sh[4][64];
    const int c4 = cols_out >> 2;
    const size_t n4 = (size_t)rows_out * c4;
    const int g = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t e4 = (size_t)blockIdx.x * 64 + g;
    int i = 0, j = 0;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e4 < n4) {
        i = (int)(e4 / c4);
        j = (int)(e4 % c4) * 4;
        const float* p = part + (size_t)i * ldp + j;
        const size_t ss = (size_t)rows_p * ldp;
        float4 a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        int k = wv;
        for (; k + 12 < splits; k += 16) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = *reinterpret_cast<const float4*>(p + (size_t)(k + 4 * u) * ss);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u].x += x[u].x; a[u].y += x[u].y; a[u].z += x[u].z; a[u].w += x[u].w;
            }
        }
        for (; k < splits; k += 4) {
            const float4 x = *reinterpret_cast<const float4*>(p + (size_t)k * ss);
            a[0].x += x.x; a[0].y += x.y; a[0].z += x.z; a[0].w += x.w;
        }
        acc.x = (a[0].x + a[1].x) + (a[2].x + a[3].x);
        acc.y = (a[0].y + a[1].y) + (a[2].y + a[3].y);
        acc.z = (a[0].z + a[1].z) + (a[2].z + a[3].z);
        acc.w = (a[0].w + a[1].w) + (a[2].w + a[3].w);
    }
    sh[wv][g] = acc;
    __syncthreads();
    if (wv == 0 && e4 < n4) {
        const float4 s0 = sh[0][g], s1 = sh[1][g], s2 = sh[2][g], s3 = sh[3][g];
        const float r[4] = {(s0.x + s1.x) + (s2.x + s3.x), (s0.y + s1.y) + (s2.y + s3.y),
                            (s0.z + s1.z) + (s2.z + s3.z), (s0.w + s1.w) + (s2.w + s3.w)};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const size_t o = (size_t)i * cols_out + j + t;
            float v = r[t];
            if (K0) v += two_lambda * (K[o] - K0[o]);
            out[o] = v;
        }
    }
}

// loss = (1/n) sum_blocks part + lambda ||K - K0||^2: one 1024-thread
// workgroup, each thread with eight independent loads in flight per round,
// then a fixed-order tree in LDS (deterministic).
__global__ __launch_bounds__(1024) void k_dec_loss(const float* __restrict__ part, int nblocks, float inv_n,
                                                   const float* __restrict__ K, const float* __restrict__ K0,
                                                   int nk, float lambda, float* __restrict__ loss)
{
    __shared__ float sh[1024];
    constexpr int U = 8;
    float s[U], tr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = tr[u] = 0.0f;
    for (int i0 = 0; i0 < nblocks; i0 += 1024 * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * 1024 + (int)threadIdx.x;
            const float x = part[i < nblocks ? i : nblocks - 1];  // every load issued, then masked
            s[u] += i < nblocks ? x : 0.0f;
        }
    }
    if (K0 && lambda != 0.f) {
        for (int i0 = 0; i0 < nk; i0 += 1024 * U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * 1024 + (int)threadIdx.x;
                const int ic = i < nk ? i : nk - 1;
                const float dlt = K[ic] - K0[ic];
                tr[u] += i < nk ? dlt * dlt : 0.0f;
            }
        }
    }
    float ss = 0.0f, tt = 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        ss += s[u];
        tt += tr[u];
    }
    sh[threadIdx.x] = ss * inv_n + lambda * tt;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0];
}

// ------------------------------------------------------------ host side

// LDS bytes of k_dec_rows with NW waves and NPG 32-pixel groups.
static size_t rows_lds(int prec, int Mp, int D, int NW, int NPG)
{
    const size_t tb = prec == LAM_FP32 ? 4 : 2;
    const size_t bpx = (size_t)kPx * NPG;
    size_t x = std::max(bpx * (Mp + 8) * tb, bpx * (D + 8) * tb);
    if (prec == LAM_FP8_E4M3) x = std::max(x, 2 * bpx * (Mp + 16));  // the weights' two E4M3 terms
    x = std::max(x, (size_t)NW * 32 * (bpx + 2) * 4);  // dQ reduction
    return 4 * NW * bpx * 4 + (size_t)NW * kPx * kScLd * tb + x;
}

constexpr size_t kMaxLds = 160 * 1024;  // LDS of a gfx950 workgroup

// 64-pixel blocks of 8 waves (each V fragment feeds two MFMAs) where the
// registers and LDS allow: BF16 and E4M3 with D a multiple of 256 up to 1024.
static bool wide_ok(int prec, int Mp, int D)
{
    const int max_nt = 4;
    return prec != LAM_FP32 && D % 256 == 0 && D / 256 <= max_nt && rows_lds(prec, Mp, D, 8, 2) <= kMaxLds;
}


// 32-column tiles per wave in the dV GEMM: two when D is a multiple of 256.
static int dv_cols(int D) { return D % 256 == 0 ? 2 : 1; }

// Pixel-range splits of a dictionary GEMM with ``tiles`` output tiles: the
// context's choice, else enough workgroups to fill 256 CUs twice; a multiple
// of 8, at most the (even) number of 32-pixel blocks rounded up to 8.
static int pick_splits(int nblocks, int tiles, int want)
{
    int s = want > 0 ? want : (512 + tiles - 1) / tiles;
    s = ((s + 7) / 8) * 8;
    if (s > nblocks) s = ((nblocks + 7) / 8) * 8;
    if (s < 8) s = 8;
    return s;
}

bool decode_layout(const lam_ctx* ctx, int prec, int n, int d, int M, int D, DecodeLayout* L)
{
    if (prec != LAM_FP32 && prec != LAM_BF16 && prec != LAM_FP8_E4M3) return false;
    if ((d != 16 && d != 32) || M < 1 || M > 2048 || D < 128 || D > 1024 || D % 128 != 0 || n < 0)
        return false;
    const size_t tb = prec == LAM_FP32 ? 4 : 2;
    const int Mp = (M + kAtomAlign - 1) / kAtomAlign * kAtomAlign;
    // 32-pixel blocks, rounded up to an even count so that the 64-pixel
    // workgroups of k_dec_rows never write past the pixel-blocked buffers (a
    // block of padding pixels contributes zeros to every reduction)
    const int nb = ((n + 2 * kPx - 1) / (2 * kPx)) * 2;
    if (rows_lds(prec, Mp, D, 4, 1) > kMaxLds) return false;  // the 32 x 4 shape always fits
    L->Mp = Mp;
    L->row_blocks = nb;
    // block shape (Same results up to the order of the per-pixel sums over the
    // waves): 64 pixels x 8 waves where wide_ok allows and the context asks
    L->wide = ctx->decode_shape.load() == 1 && wide_ok(prec, Mp, D);
    const int tiles_v = ((Mp + 127) / 128) * (D / (128 * dv_cols(D)));
    const int tiles_k = (Mp + 255) / 256;
    // the context may set the dV GEMM's splits (the larger GEMM); dK's keep the rule
    const int sv = pick_splits(std::max(nb, 1), tiles_v, ctx->decode_splits.load());
    const int sk = pick_splits(std::max(nb, 1), tiles_k, 0);
    L->splits = sv;
    L->splits_k = sk;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L->off_kb = take((size_t)Mp * d * tb);
    L->off_vb = take((size_t)Mp * D * tb);
    L->off_vt = take((size_t)Mp * D * tb);
    L->off_kt = take((size_t)32 * Mp * tb);
    L->off_m2 = take((size_t)nb * kPx * 4);
    L->off_gf = take((size_t)nb * D * kPx * tb);
    L->off_ds = take((size_t)nb * Mp * kPx * tb);
    L->off_qt = take((size_t)nb * 32 * kPx * tb);
    L->off_part = take((size_t)std::max((size_t)sv * Mp * D, (size_t)sk * Mp * 32) * 4);
    L->off_loss = take((size_t)std::max(nb, 1) * 4);
    L->off_sc = take(((size_t)3 * Mp + 64) * 4);
    L->bytes = off;
    return true;
}

// The inference decode reads only the prepared dictionary (converted K and V,
// V transposed, K permuted, the E4M3 scales); this layout packs just those at
// the front of a buffer.  The per-pixel buffers of the gradient passes are
// never touched in that mode, so their offsets point at the buffer start.
bool decode_dict_layout(const lam_ctx* ctx, int prec, int n, int d, int M, int D, DecodeLayout* L)
{
    if (!decode_layout(ctx, prec, n, d, M, D, L)) return false;
    const size_t tb = prec == LAM_FP32 ? 4 : 2;
    const int Mp = L->Mp;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    L->off_kb = take((size_t)Mp * d * tb);
    L->off_vb = take((size_t)Mp * D * tb);
    L->off_vt = take((size_t)Mp * D * tb);
    L->off_kt = take((size_t)32 * Mp * tb);
    L->off_sc = take(((size_t)3 * Mp + 64) * 4);
    L->off_m2 = L->off_gf = L->off_ds = L->off_qt = L->off_part = L->off_loss = 0;
    L->bytes = off;
    return true;
}

template <class P, int MODE, bool F8>
static hipError_t launch_rows(lam_ctx* ctx, const RowsArgs& ra, bool wide, int nb, int D, int d, int Mp, int prec,
                              hipStream_t st)
{
    const int NW = wide ? 8 : 4, NPG = wide ? 2 : 1;
    const int NT = D / (32 * NW);
    const size_t lds = rows_lds(prec, Mp, D, NW, NPG);
#define LAM_ROWS(NWV, NPGV, NTV, DQV)                                                                \
    if (NW == NWV && NT == NTV && d == DQV) {                                                        \
        auto kern = k_dec_rows<P, NTV, DQV, MODE, F8, NWV, NPGV>;                                     \
        const hipError_t el = ctx_ensure_lds(ctx, (const void*)kern, lds);                           \
        if (el != hipSuccess) return el;                                                             \
        hipLaunchKernelGGL(kern, dim3(nb / NPGV), dim3(NWV * kWave), lds, st, ra);                  \
        return hipGetLastError();                                                                    \
    }
    LAM_ROWS(4, 1, 1, 16) LAM_ROWS(4, 1, 2, 16) LAM_ROWS(4, 1, 3, 16) LAM_ROWS(4, 1, 4, 16)
    LAM_ROWS(4, 1, 5, 16) LAM_ROWS(4, 1, 6, 16) LAM_ROWS(4, 1, 7, 16) LAM_ROWS(4, 1, 8, 16)
    LAM_ROWS(4, 1, 1, 32) LAM_ROWS(4, 1, 2, 32) LAM_ROWS(4, 1, 3, 32) LAM_ROWS(4, 1, 4, 32)
    LAM_ROWS(4, 1, 5, 32) LAM_ROWS(4, 1, 6, 32) LAM_ROWS(4, 1, 7, 32) LAM_ROWS(4, 1, 8, 32)
    if constexpr (P::kBytes == 2) {  // the 64 x 8 shape (wide_ok): up to 4 D tiles a wave
        LAM_ROWS(8, 2, 1, 16) LAM_ROWS(8, 2, 1, 32)
        LAM_ROWS(8, 2, 2, 16) LAM_ROWS(8, 2, 2, 32) LAM_ROWS(8, 2, 3, 16) LAM_ROWS(8, 2, 3, 32)
        LAM_ROWS(8, 2, 4, 16) LAM_ROWS(8, 2, 4, 32)
    }
#undef LAM_ROWS
    return hipErrorInvalidValue;
}

template <class P, bool F8>
static hipError_t run_decode(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, int mode, hipStream_t st,
                             hipStream_t st_dict)
{
    using T = typename P::T;
    char* base = reinterpret_cast<char*>(L.base);
    T* Kb = reinterpret_cast<T*>(base + L.off_kb);
    T* Vb = reinterpret_cast<T*>(base + L.off_vb);
    T* Vt = reinterpret_cast<T*>(base + L.off_vt);
    T* Ktp = reinterpret_cast<T*>(base + L.off_kt);
    const int Mp = L.Mp, nb = L.row_blocks;
    {
        size_t work = std::max((size_t)Mp * A.D, (size_t)32 * Mp);
        int grid = (int)std::min<size_t>((work + 255) / 256, 2048);
        if (F8) {
            float* sc = reinterpret_cast<float*>(base + L.off_sc);
            hipError_t e0 = launch_fill_u32(reinterpret_cast<uint32_t*>(sc + 2 * Mp), 1, 0u, st);
            if (e0 != hipSuccess) return e0;
            hipLaunchKernelGGL(k_dec_scales, dim3(Mp), dim3(256), 0, st, A.V, A.M, Mp, A.D, sc);
            hipLaunchKernelGGL(k_dec_prep<P>, dim3(grid), dim3(256), 0, st, A.K, A.V, A.M, Mp, A.d, A.D,
                               Kb, Vb, (T*)nullptr, Ktp);
            hipLaunchKernelGGL(k_dec_prep_fp8, dim3(grid), dim3(256), 0, st, A.V, A.M, Mp, A.D,
                               (const float*)sc, reinterpret_cast<uint8_t*>(Vt), sc + 2 * Mp + 64,
                               sc + 2 * Mp + 8);
        } else {
            hipLaunchKernelGGL(k_dec_prep<P>, dim3(grid), dim3(256), 0, st, A.K, A.V, A.M, Mp, A.d, A.D,
                               Kb, Vb, Vt, Ktp);
        }
    }
    RowsArgs ra{};
    ra.n = A.n; ra.d = A.d; ra.M = A.M; ra.Mp = Mp; ra.D = A.D;
    // logits Q K^T / sqrt(d), or Q K^T * logit_scale when the caller sets it
    const float lscale = A.logit_scale > 0.0f ? A.logit_scale : 1.0f / sqrtf((float)A.d);
    ra.scale_log2 = kLog2e * lscale;
    ra.inv_sqrt_d = lscale;
    ra.lam_cos = A.lam_cos;
    ra.lam_l2 = A.lam_l2;
    ra.inv_n = A.n > 0 ? 1.0f / (float)A.n : 0.0f;
    ra.Q = A.Q; ra.target = A.target; ra.dF = A.dF; ra.F = A.F; ra.dQ = A.dQ; ra.row_cos = A.row_cos;
    ra.loss_part = reinterpret_cast<float*>(base + L.off_loss);
    ra.Kb = Kb; ra.Vb = Vb; ra.Vt = Vt; ra.Ktp = Ktp;
    ra.M2 = reinterpret_cast<float*>(base + L.off_m2);
    ra.Gt = base + L.off_gf; ra.St = base + L.off_ds; ra.Qt = base + L.off_qt;
    if (F8) {
        float* sc = reinterpret_cast<float*>(base + L.off_sc);
        ra.Vt8 = reinterpret_cast<const uint8_t*>(Vt);
        ra.sv_fold = sc + 2 * Mp + 64;
        ra.fp8_unscale = sc + 2 * Mp + 8;
    }
    hipError_t e = hipSuccess;
    if (nb > 0) {
        ProfScope ps(ctx, "decode_rows", st);
        if (mode == MODE_INFER) e = launch_rows<P, MODE_INFER, F8>(ctx, ra, L.wide, nb, A.D, A.d, Mp, A.prec, st);
        else if (mode == MODE_LOSS) e = launch_rows<P, MODE_LOSS, F8>(ctx, ra, L.wide, nb, A.D, A.d, Mp, A.prec, st);
        else e = launch_rows<P, MODE_ADJ, F8>(ctx, ra, L.wide, nb, A.D, A.d, Mp, A.prec, st);
        if (e != hipSuccess) return e;
    }
    if (mode == MODE_INFER) return hipGetLastError();
    // The dictionary part (dV, dK, their reductions and the loss) reads only
    // the workspace; on a second stream it runs beside whatever the caller
    // queues on st after dQ (the render backward).
    // (the context's event marks the end of the rows kernel; a wait refers to
    // the record made before it, so reusing the event across calls is safe)
    if (st_dict != st) {
        hipEvent_t ev = ctx->fork;
        if (!ev) return hipErrorInvalidValue;
        e = hipEventRecord(ev, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(st_dict, ev, 0);
        if (e != hipSuccess) return e;
        st = st_dict;
    }
    float* part = reinterpret_cast<float*>(base + L.off_part);
    // dV = P~^T G over all pixels, P~ rebuilt from Q, K and the saved row max
    {
        const int qt = dv_cols(A.D);
        const int ti = (Mp + 127) / 128, tj = A.D / (128 * qt);
        if (nb > 0) {
            ProfScope ps(ctx, "decode_tn", st);
            auto kern = qt == 2 ? (A.d == 16 ? k_dec_dv<P, 16, 2> : k_dec_dv<P, 32, 2>)
                                : (A.d == 16 ? k_dec_dv<P, 16, 1> : k_dec_dv<P, 32, 1>);
            hipLaunchKernelGGL(kern, dim3(L.splits * ti * tj), dim3(256), 0, st, A.Q, A.n,
                               (const void*)Kb, A.M, (const float*)ra.M2, ra.scale_log2,
                               (const void*)(base + L.off_gf), Mp, A.D, nb, L.splits, ti, tj, part);
        }
        hipLaunchKernelGGL(k_dec_reduce, dim3((A.M * A.D / 4 + 63) / 64), dim3(256), 0, st,
                           (const float*)part, nb > 0 ? L.splits : 0, Mp, A.D, A.M, A.D, A.dV,
                           (const float*)nullptr, (const float*)nullptr, 0.0f);
    }
    // dK = dS^T Q (1/sqrt(d) already in dS) + 2 lambda (K - K0)
    {
        const int ti = (Mp + 255) / 256, tj = 1;
        if (nb > 0) {
            hipLaunchKernelGGL((k_dec_tn<P, 2, 1, 4, 1>), dim3(L.splits_k * ti * tj), dim3(256), 0, st,
                               (const void*)(base + L.off_ds), Mp, (const void*)(base + L.off_qt), 32, nb,
                               L.splits_k, ti, tj, part);
        }
        const bool tr = mode == MODE_LOSS && A.K0 && A.lambda_tr != 0.0f;
        hipLaunchKernelGGL(k_dec_reduce, dim3((A.M * A.d / 4 + 63) / 64), dim3(256), 0, st,
                           (const float*)part, nb > 0 ? L.splits_k : 0, Mp, 32, A.M, A.d, A.dK,
                           tr ? A.K : (const float*)nullptr, tr ? A.K0 : (const float*)nullptr,
                           tr ? 2.0f * A.lambda_tr : 0.0f);
    }
    if (mode == MODE_LOSS)
        hipLaunchKernelGGL(k_dec_loss, dim3(1), dim3(1024), 0, st, (const float*)ra.loss_part, nb,
                           ra.inv_n, A.K, A.K0, A.M * A.d, A.K0 ? A.lambda_tr : 0.0f, A.loss);
    return hipGetLastError();
}

hipError_t decode_loss_launch(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, hipStream_t st,
                              hipStream_t st_dict)
{
    if (!st_dict) st_dict = st;
    if (A.prec == LAM_FP32) return run_decode<TF32, false>(ctx, A, L, MODE_LOSS, st, st_dict);
    if (A.prec == LAM_FP8_E4M3) return run_decode<TBF16, true>(ctx, A, L, MODE_LOSS, st, st_dict);
    return run_decode<TBF16, false>(ctx, A, L, MODE_LOSS, st, st_dict);
}

hipError_t decode_forward_launch(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, hipStream_t st)
{
    if (A.prec == LAM_FP32) return run_decode<TF32, false>(ctx, A, L, MODE_INFER, st, st);
    if (A.prec == LAM_FP8_E4M3) return run_decode<TBF16, true>(ctx, A, L, MODE_INFER, st, st);
    return run_decode<TBF16, false>(ctx, A, L, MODE_INFER, st, st);
}

hipError_t decode_backward_launch(lam_ctx* ctx, const DecodeArgs& A, const DecodeLayout& L, hipStream_t st)
{
    if (A.prec == LAM_FP32) return run_decode<TF32, false>(ctx, A, L, MODE_ADJ, st, st);
    if (A.prec == LAM_FP8_E4M3) return run_decode<TBF16, true>(ctx, A, L, MODE_ADJ, st, st);
    return run_decode<TBF16, false>(ctx, A, L, MODE_ADJ, st, st);
}

}  // namespace lam

// ------------------------------------------------------------ C ABI

using namespace lam;

// Pixel-row arrays are read and written with 16-byte vector accesses.
static bool a16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static bool dec_ptrs_ok(const float* Q, int n, const float* K, const float* V)
{
    return K && V && (n == 0 || Q) && a16(Q);
}

extern "C" {

lam_status lam_decode_workspace_size(const lam_ctx* ctx, int precision, int n, int d, int M, int D,
                                     uint64_t* bytes)
{
    if (!bytes) return LAM_ERR_INVALID_ARG;
    if (n < 0) return LAM_ERR_INVALID_ARG;
    DecodeLayout L{};
    if (!decode_layout(ctx_options(ctx), precision, n, d, M, D, &L)) return LAM_ERR_UNSUPPORTED;
    *bytes = L.bytes;
    return LAM_OK;
}

static lam_status dec_common(const lam_ctx* ctx, int precision, int n, int d, int M, int D, void* ws,
                             uint64_t ws_bytes, DecodeLayout* L)
{
    if (!ctx_ok(ctx) || n < 0) return LAM_ERR_INVALID_ARG;
    if (!decode_layout(ctx, precision, n, d, M, D, L)) return LAM_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < L->bytes) return LAM_ERR_INVALID_ARG;
    L->base = ws;
    return LAM_OK;
}

lam_status lam_decode_loss(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K, const float* V,
                           int M, int D, const float* target, const float* K0, float lambda_tr,
                           float* loss, float* dQ, float* dK, float* dV, float* row_cos, void* ws,
                           uint64_t ws_bytes, void* stream)
{
    DecodeLayout L{};
    lam_status s = dec_common(ctx, precision, n, d, M, D, ws, ws_bytes, &L);
    if (s != LAM_OK) return s;
    if (!dec_ptrs_ok(Q, n, K, V) || !loss || !dK || !dV || (n > 0 && !target)) return LAM_ERR_INVALID_ARG;
    if (!a16(target) || !a16(dQ)) return LAM_ERR_INVALID_ARG;
    if (lambda_tr != 0.0f && !K0) return LAM_ERR_INVALID_ARG;
    DecodeArgs A{};
    A.prec = precision; A.n = n; A.d = d; A.M = M; A.D = D;
    A.Q = Q; A.K = K; A.V = V; A.target = target; A.K0 = K0; A.lambda_tr = lambda_tr;
    A.loss = loss; A.dQ = dQ; A.dK = dK; A.dV = dV; A.row_cos = row_cos;
    return decode_loss_launch(ctx, A, L, (hipStream_t)stream) == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_decode_loss_overlap(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K, const float* V,
                                   int M, int D, const float* target, const float* K0, float lambda_tr,
                                   float* loss, float* dQ, float* dK, float* dV, float* row_cos, void* ws,
                                   uint64_t ws_bytes, void* stream, void* dict_stream)
{
    DecodeLayout L{};
    lam_status s = dec_common(ctx, precision, n, d, M, D, ws, ws_bytes, &L);
    if (s != LAM_OK) return s;
    if (!dec_ptrs_ok(Q, n, K, V) || !loss || !dK || !dV || (n > 0 && !target)) return LAM_ERR_INVALID_ARG;
    if (!a16(target) || !a16(dQ)) return LAM_ERR_INVALID_ARG;
    if (lambda_tr != 0.0f && !K0) return LAM_ERR_INVALID_ARG;
    DecodeArgs A{};
    A.prec = precision; A.n = n; A.d = d; A.M = M; A.D = D;
    A.Q = Q; A.K = K; A.V = V; A.target = target; A.K0 = K0; A.lambda_tr = lambda_tr;
    A.loss = loss; A.dQ = dQ; A.dK = dK; A.dV = dV; A.row_cos = row_cos;
    return decode_loss_launch(ctx, A, L, (hipStream_t)stream, (hipStream_t)dict_stream) == hipSuccess ? LAM_OK
                                                                                                   : LAM_ERR_HIP;
}

lam_status lam_decode_forward(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K, const float* V,
                              int M, int D, float* F, void* ws, uint64_t ws_bytes, void* stream)
{
    DecodeLayout L{};
    lam_status s = dec_common(ctx, precision, n, d, M, D, ws, ws_bytes, &L);
    if (s != LAM_OK) return s;
    if (!dec_ptrs_ok(Q, n, K, V) || (n > 0 && !F) || !a16(F)) return LAM_ERR_INVALID_ARG;
    DecodeArgs A{};
    A.prec = precision; A.n = n; A.d = d; A.M = M; A.D = D;
    A.Q = Q; A.K = K; A.V = V; A.F = F;
    return decode_forward_launch(ctx, A, L, (hipStream_t)stream) == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_decode_forward_noalloc(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K,
                                      const float* V, int M, int D, float* F, void* stream)
{
    if (!ctx_ok(ctx) || n < 0) return LAM_ERR_INVALID_ARG;
    DecodeLayout L{};
    if (!decode_dict_layout(ctx, precision, n, d, M, D, &L)) return LAM_ERR_UNSUPPORTED;
    if (!ctx->static_scratch || L.bytes > ctx->static_scratch_bytes) return LAM_ERR_UNSUPPORTED;
    if (!dec_ptrs_ok(Q, n, K, V) || (n > 0 && !F) || !a16(F)) return LAM_ERR_INVALID_ARG;
    L.base = ctx->static_scratch;
    DecodeArgs A{};
    A.prec = precision; A.n = n; A.d = d; A.M = M; A.D = D;
    A.Q = Q; A.K = K; A.V = V; A.F = F;
    return decode_forward_launch(ctx, A, L, (hipStream_t)stream) == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

lam_status lam_decode_backward(lam_ctx* ctx, int precision, const float* Q, int n, int d, const float* K, const float* V,
                               int M, int D, const float* dF, float* dQ, float* dK, float* dV, void* ws,
                               uint64_t ws_bytes, void* stream)
{
    DecodeLayout L{};
    lam_status s = dec_common(ctx, precision, n, d, M, D, ws, ws_bytes, &L);
    if (s != LAM_OK) return s;
    if (!dec_ptrs_ok(Q, n, K, V) || !dK || !dV || (n > 0 && !dF) || !a16(dF) || !a16(dQ))
        return LAM_ERR_INVALID_ARG;
    DecodeArgs A{};
    A.prec = precision; A.n = n; A.d = d; A.M = M; A.D = D;
    A.Q = Q; A.K = K; A.V = V; A.dF = dF; A.dQ = dQ; A.dK = dK; A.dV = dV;
    return decode_backward_launch(ctx, A, L, (hipStream_t)stream) == hipSuccess ? LAM_OK : LAM_ERR_HIP;
}

}  // extern "C"
