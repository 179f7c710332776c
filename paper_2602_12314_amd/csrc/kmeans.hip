// Streaming K-means dictionary initialisation (paper Eq. 10) on gfx950.
//
// One Lloyd iteration over points X [n, D] (weights w, or 1) and centres
// C [k, D]:
//   assign  a_i = argmin_j |x_i - c_j|^2 = argmin_j (|c_j|^2 - 2 <x_i, c_j>),
//           ties to the lowest j: an MFMA distance GEMM with the argmin fused
//           into its epilogue (k_km_assign).  A workgroup keeps its block of
//           points resident in LDS (converted once to the product type, in
//           the fragment-major layout) and its four waves sweep the centres,
//           32 NCW at a time, streaming the centre fragments from L2 through a
//           register ring; a lane ends with the best centre of one point for
//           its half of the rows, the halves and the waves then meet.
//   update  c_j = sum_{a_i = j} w_i x_i / sum_{a_i = j} w_i (kept when the
//           weight is zero): the assignments are radix-sorted (stable, so a
//           cluster's points stay in index order), the sorted list is cut into
//           chunks of kChunk points, each chunk sums its runs (a run inside the
//           chunk is final; its first and last runs are partials), and one
//           workgroup per centre adds the partials in chunk order.  The sums
//           are deterministic and independent of the launch schedule.
// The streaming step (Eq. 10) chains two Lloyd runs: the keyframe's embeddings
// into m weighted micro-centres, then the micro-centres merged with the
// weighted global centres into K.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "kmeans.h"

namespace lam {
namespace km {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kChunk = 128;     // sorted points per update chunk
constexpr int kNcw = 2;         // 32-centre row blocks per wave step
constexpr int kCentreAlign = 32 * kNcw;
constexpr int kPipe = 4;        // centre fragments in flight per wave
constexpr int kAssignThreads = 256;
constexpr size_t kMaxTileLds = 64 * 1024;  // two workgroups per CU
constexpr int kSlice = 2048;    // centres per assign launch (their norms sit in LDS)

// Products in float32 (the 32x32x2 f32 MFMA, eight steps per 16-wide K chunk).
struct PF32 {
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
    __device__ static void store8(T* p, const float* v)
    {
        reinterpret_cast<float4*>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
        reinterpret_cast<float4*>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
    __device__ static void mma(f32x16& c, const Frag& a, const Frag& b)
    {
#pragma unroll
        for (int s = 0; s < 8; ++s) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], c, 0, 0, 0);
    }
};

// Products on bfloat16 operands with float32 accumulation.
struct PBF16 {
    using T = __bf16;
    using Frag = bf16x8;
    static constexpr int kBytes = 2;
    __device__ static Frag load(const T* p) { return *reinterpret_cast<const bf16x8*>(p); }
    __device__ static void store8(T* p, const float* v)
    {
        bf16x8 f;
#pragma unroll
        for (int t = 0; t < 8; ++t) f[t] = (__bf16)v[t];
        *reinterpret_cast<bf16x8*>(p) = f;
    }
    __device__ static void mma(f32x16& c, const Frag& a, const Frag& b)
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// Fragment-major layout (shared with the decode operands): block (row / 32,
// k / 16) of an operand X[R][K] holds 64 lanes x 8 elements, element (row, k)
// at lane 32 (k / 8 % 2) + row % 32, slot k % 8.
__device__ inline size_t frag_off(int row, int j8, int nc)
{
    // j8 = k / 8 (the 8-element group within the row)
    return ((((size_t)(row >> 5) * nc + (j8 >> 1)) << 6) + (j8 & 1) * 32 + (row & 31)) * 8;
}

// Row of the 32x32 MFMA result held in register r of lane half h.
__device__ inline int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// (value, index) pairs ordered by value, then index.
__device__ inline bool better(float v, int j, float bv, int bj) { return v < bv || (v == bv && j < bj); }

// Centres C [k, D] -> fragment-major Cf [kp, D] in the product type (rows
// k .. kp-1 zero).
template <class P>
__global__ __launch_bounds__(256) void k_km_prep(const float* __restrict__ C, int k, int kp, int D,
                                                 typename P::T* __restrict__ Cf)
{
    const int g8 = D / 8, nc = D / 16;
    const size_t total = (size_t)kp * g8;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const int row = (int)(g / g8), j = (int)(g - (size_t)row * g8);
        float v[8];
        if (row < k) {
            const float4* src = reinterpret_cast<const float4*>(C + (size_t)row * D + j * 8);
            const float4 a = src[0], b = src[1];
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = 0.0f;
        }
        P::store8(Cf + frag_off(row, j, nc), v);
    }
}

// cn[j] = |c_j|^2 in float32 for j < k, +inf for the padding rows (never
// chosen).  One wave per row.
__global__ __launch_bounds__(256) void k_km_norms(const float* __restrict__ C, int k, int kp, int D,
                                                  float* __restrict__ cn)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= kp) return;
    float s = 0.0f;
    if (row < k)
        for (int c = lane; c < D; c += kWave) {
            const float v = C[(size_t)row * D + c];
            s += v * v;
        }
    s = wave_allsum(s);
    if (lane == 0) cn[row] = row < k ? s : __builtin_huge_valf();
}

// Nearest centre of 32 NP points per workgroup (NP <= 2: with the tile at most
// 64 KB, two workgroups share a CU and one stages its points while the other
// computes) among one slice of at most
// kSlice centres (global indices kbase ..): the slice's norms are staged in
// LDS next to the points' tile (product type, fragment-major [NP][D/16][64][8]),
// so the epilogue reads only LDS and every global load is a centre fragment of
// the branch-free ring, whose waits the compiler can count exactly.  With
// merge, the result is compared with the best of the earlier slices (lower
// indices, so ties keep it).
template <class P, int NP, int PIPE>
__global__ __launch_bounds__(kAssignThreads, 1) void k_km_assign(const float* __restrict__ X, int n, int D,
                                                                 const typename P::T* __restrict__ Cf,
                                                                 const float* __restrict__ cn, int kcp,
                                                                 int kbase, int k, int merge,
                                                                 float* __restrict__ best_v,
                                                                 uint32_t* __restrict__ a_out,
                                                                 float* __restrict__ d2_out)
{
    using T = typename P::T;
    using Frag = typename P::Frag;
    constexpr int BP = 32 * NP;
    constexpr int NW = kAssignThreads / kWave;
    extern __shared__ __align__(16) unsigned char smem[];
    T* xs = reinterpret_cast<T*>(smem);
    const int nc = D / 16, g8 = D / 8;
    float* cn_s = reinterpret_cast<float*>(smem + (size_t)BP * D * P::kBytes);
    float* red_v = cn_s + kcp;
    int* red_j = reinterpret_cast<int*>(red_v + NW * BP);
    const int p0 = blockIdx.x * BP;

    // stage the slice's norms and the point tile: 8 consecutive floats of one
    // row per item, the threads walking along the rows (coalesced)
    for (int t = threadIdx.x; t < kcp; t += kAssignThreads) cn_s[t] = cn[t];
    {
        constexpr int U = 8;
        const int items = BP * g8;
        for (int base = threadIdx.x; base < items; base += U * kAssignThreads) {
            float4 va[U], vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int g = base + u * kAssignThreads;
                const int row = g / g8, j = g - row * g8;
                va[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                vb[u] = va[u];
                if (g < items && p0 + row < n) {
                    // read once: streamed past the L2 that holds the centres
                    const f32x4* src = reinterpret_cast<const f32x4*>(X + (size_t)(p0 + row) * D + j * 8);
                    const f32x4 t0 = __builtin_nontemporal_load(src), t1 = __builtin_nontemporal_load(src + 1);
                    va[u] = make_float4(t0.x, t0.y, t0.z, t0.w);
                    vb[u] = make_float4(t1.x, t1.y, t1.z, t1.w);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int g = base + u * kAssignThreads;
                if (g < items) {
                    const int row = g / g8, j = g - row * g8;
                    const float v[8] = {va[u].x, va[u].y, va[u].z, va[u].w, vb[u].x, vb[u].y, vb[u].z, vb[u].w};
                    P::store8(xs + frag_off(row, j, nc), v);
                }
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, h = lane >> 5;
    const int ngroups = kcp / kCentreAlign;
    const int mine = ngroups > w ? (ngroups - w + NW - 1) / NW : 0;
    float bv[NP];
    int bj[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        bv[p] = __builtin_huge_valf();
        bj[p] = 0x7fffffff;
    }
    if (mine > 0) {
        f32x16 acc[kNcw][NP];
#pragma unroll
        for (int i = 0; i < kNcw; ++i)
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][p][r] = 0.0f;
        auto cfrag = [&](int rb, int c) { return P::load(Cf + ((((size_t)rb * nc + c) << 6) + lane) * 8); };
        auto xfrag = [&](int p, int c) { return P::load(xs + ((((size_t)p * nc + c) << 6) + lane) * 8); };
        Frag ring[PIPE][kNcw];
        Frag bcur[NP];
#pragma unroll
        for (int u = 0; u < PIPE; ++u)
#pragma unroll
            for (int i = 0; i < kNcw; ++i) ring[u][i] = cfrag(w * kNcw + i, u);
#pragma unroll
        for (int p = 0; p < NP; ++p) bcur[p] = xfrag(p, 0);
        const int nblk = nc / PIPE;
        for (int q = 0; q < mine; ++q) {
            const int rb0 = (w + NW * q) * kNcw;
            const int rbn = q + 1 < mine ? rb0 + NW * kNcw : rb0;  // the last group refetches its own rows
            for (int cb = 0; cb < nblk; ++cb) {
                const bool lastblk = cb == nblk - 1;
                const int rbp = lastblk ? rbn : rb0;
#pragma unroll
                for (int u = 0; u < PIPE; ++u) {
                    const int c = cb * PIPE + u;
                    Frag bnext[NP];
                    const int cx = c + 1 == nc ? 0 : c + 1;
#pragma unroll
                    for (int p = 0; p < NP; ++p) bnext[p] = xfrag(p, cx);
                    __builtin_amdgcn_sched_barrier(0);  // the next step's LDS reads go out first
#pragma unroll
                    for (int i = 0; i < kNcw; ++i)
#pragma unroll
                        for (int p = 0; p < NP; ++p) P::mma(acc[i][p], ring[u][i], bcur[p]);
                    // chunk c + PIPE of this group, or chunk u of the next one
                    const int cp = lastblk ? u : c + PIPE;
#pragma unroll
                    for (int i = 0; i < kNcw; ++i) ring[u][i] = cfrag(rbp + i, cp);
#pragma unroll
                    for (int p = 0; p < NP; ++p) bcur[p] = bnext[p];
                    // keep the refill in this step: sunk to the end of the
                    // block it would leave the first slots no time in flight
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // epilogue of group q: rows are centres, columns points; rows are
            // visited in increasing order, so strict < keeps the lowest index
#pragma unroll
            for (int i = 0; i < kNcw; ++i) {
                const int jl = 32 * (rb0 + i);
                float cv[16];
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    const float4 t = *reinterpret_cast<const float4*>(cn_s + jl + 8 * q4 + 4 * h);
                    cv[4 * q4] = t.x; cv[4 * q4 + 1] = t.y; cv[4 * q4 + 2] = t.z; cv[4 * q4 + 3] = t.w;
                }
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float v = cv[r] - 2.0f * acc[i][p][r];
                        if (v < bv[p]) {
                            bv[p] = v;
                            bj[p] = kbase + jl + crow(r, h);
                        }
                        acc[i][p][r] = 0.0f;
                    }
            }
        }
    }
    // the two halves of the wave hold different rows for the same point
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const float ov = __shfl_xor(bv[p], 32);
        const int oj = __shfl_xor(bj[p], 32);
        if (better(ov, oj, bv[p], bj[p])) {
            bv[p] = ov;
            bj[p] = oj;
        }
        if (h == 0) {
            red_v[w * BP + 32 * p + lane] = bv[p];
            red_j[w * BP + 32 * p + lane] = bj[p];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < BP; t += kAssignThreads) {
        float v = red_v[t];
        int j = red_j[t];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww)
            if (better(red_v[ww * BP + t], red_j[ww * BP + t], v, j)) {
                v = red_v[ww * BP + t];
                j = red_j[ww * BP + t];
            }
        const int pt = p0 + t;
        if (pt < n) {
            if (merge) {
                const float ov = best_v[pt];
                if (!(v < ov)) {
                    v = ov;
                    j = (int)a_out[pt];
                }
            }
            // a non-finite distance (non-finite input) leaves no winner: centre 0
            if (!(j >= 0 && j < k)) j = 0;
            a_out[pt] = (uint32_t)j;
            if (best_v) best_v[pt] = v;
            if (d2_out) {
                const float4* row = reinterpret_cast<const float4*>(X + (size_t)pt * D);
                float s = 0.0f;
                for (int c = 0; c < D / 4; ++c) {
                    const float4 x = row[c];
                    s += x.x * x.x + x.y * x.y + x.z * x.z + x.w * x.w;
                }
                d2_out[pt] = fmaxf(s + v, 0.0f);
            }
        }
    }
}

// Per-centre [start, end) of the sorted assignment list (centres without
// points keep start = end = 0 from the fill before).
__global__ __launch_bounds__(256) void k_km_ranges(const uint32_t* __restrict__ keys, int n,
                                                   uint32_t* __restrict__ start, uint32_t* __restrict__ end)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    if (i == 0 || keys[i - 1] != key) start[key] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] != key) end[key] = (uint32_t)(i + 1);
}

// Runs of one chunk of the sorted list.  Thread t owns float4 column groups
// t, t + 128, ...  A run that neither starts nor ends at the chunk's edge is a
// whole cluster and is finalised here; the chunk's first run goes to head[c],
// its last (when different) to tail[c].
template <int CG>
__global__ __launch_bounds__(128) void k_km_chunks(const float* __restrict__ X, const float* __restrict__ w,
                                                   int n, int D, const uint32_t* __restrict__ skeys,
                                                   const uint32_t* __restrict__ sidx,
                                                   const float* __restrict__ Cold, float* __restrict__ Cnew,
                                                   float* __restrict__ Wnew, float* __restrict__ head,
                                                   float* __restrict__ tail, float* __restrict__ headw,
                                                   float* __restrict__ tailw)
{
    __shared__ uint32_t keys[kChunk];
    __shared__ uint32_t idx[kChunk];
    __shared__ float wt[kChunk];
    const int c = blockIdx.x, s0 = c * kChunk;
    const int len = min(kChunk, n - s0);
    for (int t = threadIdx.x; t < len; t += 128) {
        const uint32_t id = sidx[s0 + t];
        keys[t] = skeys[s0 + t];
        idx[t] = id;
        wt[t] = w ? w[id] : 1.0f;
    }
    __syncthreads();
    const int D4 = D / 4;
    float4 acc[CG];
#pragma unroll
    for (int g = 0; g < CG; ++g) acc[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    float wsum = 0.0f;
    int rs = 0;
    constexpr int U = 16;  // rows in flight per thread
    for (int i0 = 0; i0 < len; i0 += U) {
        float4 v[U][CG];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u, len - 1);
            const float4* row = reinterpret_cast<const float4*>(X + (size_t)idx[i] * D);
#pragma unroll
            for (int g = 0; g < CG; ++g) {
                const int col = threadIdx.x + 128 * g;
                v[u][g] = col < D4 ? row[col] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i < len) {
                const float wi = wt[i];
#pragma unroll
                for (int g = 0; g < CG; ++g) {
                    acc[g].x += wi * v[u][g].x;
                    acc[g].y += wi * v[u][g].y;
                    acc[g].z += wi * v[u][g].z;
                    acc[g].w += wi * v[u][g].w;
                }
                wsum += wi;
                if (i == len - 1 || keys[i + 1] != keys[i]) {
                    const uint32_t key = keys[i];
                    const bool first = rs == 0, last = i + 1 == len;
                    float* dst;
                    if (first) {
                        dst = head + (size_t)c * D;
                        if (threadIdx.x == 0) headw[c] = wsum;
                    } else if (last) {
                        dst = tail + (size_t)c * D;
                        if (threadIdx.x == 0) tailw[c] = wsum;
                    } else {
                        dst = Cnew + (size_t)key * D;
                        if (threadIdx.x == 0) Wnew[key] = wsum;
                    }
                    const bool fin = !first && !last;
                    const float inv = wsum > 0.0f ? 1.0f / wsum : 0.0f;
#pragma unroll
                    for (int g = 0; g < CG; ++g) {
                        const int col = threadIdx.x + 128 * g;
                        if (col < D4) {
                            float4 o = acc[g];
                            if (fin) {
                                if (wsum > 0.0f)
                                    o = make_float4(o.x * inv, o.y * inv, o.z * inv, o.w * inv);
                                else
                                    o = reinterpret_cast<const float4*>(Cold + (size_t)key * D)[col];
                            }
                            reinterpret_cast<float4*>(dst)[col] = o;
                        }
                        acc[g] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                    wsum = 0.0f;
                    rs = i + 1;
                }
            }
        }
    }
}

// One workgroup per centre: centres whose points touch a chunk edge add their
// partials in chunk order; centres without points keep their position.
template <int CG>
__global__ __launch_bounds__(128) void k_km_fixup(const uint32_t* __restrict__ start,
                                                  const uint32_t* __restrict__ end, int n, int D,
                                                  const float* __restrict__ Cold, float* __restrict__ Cnew,
                                                  float* __restrict__ Wnew, const float* __restrict__ head,
                                                  const float* __restrict__ tail,
                                                  const float* __restrict__ headw,
                                                  const float* __restrict__ tailw)
{
    const int j = blockIdx.x, D4 = D / 4;
    const int s = (int)start[j], e = (int)end[j];
    float4* out = reinterpret_cast<float4*>(Cnew + (size_t)j * D);
    if (s >= e) {
        const float4* old = reinterpret_cast<const float4*>(Cold + (size_t)j * D);
        for (int col = threadIdx.x; col < D4; col += 128) out[col] = old[col];
        if (threadIdx.x == 0) Wnew[j] = 0.0f;
        return;
    }
    const int cs = s / kChunk, ce = (e - 1) / kChunk;
    const bool first = s == cs * kChunk;
    if (cs == ce && !first && e != min((cs + 1) * kChunk, n)) return;  // finalised by its chunk
    const float* src0 = first ? head + (size_t)cs * D : tail + (size_t)cs * D;
    float W = first ? headw[cs] : tailw[cs];
    for (int c = cs + 1; c <= ce; ++c) W += headw[c];
    const float inv = W > 0.0f ? 1.0f / W : 0.0f;
#pragma unroll
    for (int g = 0; g < CG; ++g) {
        const int col = threadIdx.x + 128 * g;
        if (col < D4) {
            float4 a = reinterpret_cast<const float4*>(src0)[col];
            for (int c = cs + 1; c <= ce; ++c) {
                const float4 b = reinterpret_cast<const float4*>(head + (size_t)c * D)[col];
                a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
            }
            out[col] = W > 0.0f ? make_float4(a.x * inv, a.y * inv, a.z * inv, a.w * inv)
                                : reinterpret_cast<const float4*>(Cold + (size_t)j * D)[col];
        }
    }
    if (threadIdx.x == 0) Wnew[j] = W;
}

// out[r] = X[rows[r]] for r < m (rows validated on the host).
__global__ __launch_bounds__(128) void k_km_gather(const float* __restrict__ X, int D,
                                                   const int32_t* __restrict__ rows, int m, float* __restrict__ out)
{
    const int r = blockIdx.x;
    if (r >= m) return;
    const float4* src = reinterpret_cast<const float4*>(X + (size_t)rows[r] * D);
    float4* dst = reinterpret_cast<float4*>(out + (size_t)r * D);
    for (int c = threadIdx.x; c < D / 4; c += 128) dst[c] = src[c];
}

// ------------------------------------------------------------ host side

// Points per assign workgroup: tiles of at most 64 KB (two workgroups per CU),
// else 32 points in up to 128 KB (one per CU) for the widest rows.
static int tile_points(int prec, int D)
{
    const size_t bytes = prec == LAM_BF16 ? 2 : 4;
    for (int bp : {64, 32})
        if ((size_t)bp * D * bytes <= kMaxTileLds) return bp;
    return (size_t)32 * D * bytes <= 2 * kMaxTileLds ? 32 : 0;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Key bits of the sort by centre index.
static int kmeans_key_bits(int k)
{
    int bits = 1;
    while ((1 << bits) < k) ++bits;
    return bits;
}

bool kmeans_shape_ok(int prec, int D, int k)
{
    if (prec != LAM_FP32 && prec != LAM_BF16) return false;
    if (D < 32 || D % 32 != 0 || D > 2048 || k < 1 || k > 65536) return false;
    return tile_points(prec, D) > 0;
}

KmLayout kmeans_layout(int prec, int npts, int D, int k)
{
    KmLayout L{};
    const size_t kp = align_up((size_t)k, kCentreAlign);
    const size_t nchunks = ((size_t)npts + kChunk - 1) / kChunk;
    const size_t np = std::max<size_t>((size_t)npts, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.off_cf = take(kp * D * (prec == LAM_BF16 ? 2 : 4));
    L.off_cn = take(kp * 4);
    L.off_a = take(np * 4);
    L.off_bv = take(np * 4);
    L.off_ka = take(np * 4);
    L.off_va = take(np * 4);
    L.off_kb = take(np * 4);
    L.off_vb = take(np * 4);
    L.off_sort = take(radix_scratch_words(kmeans_key_bits(k), (uint32_t)np) * 4);
    L.off_start = take((size_t)k * 4);
    L.off_end = take((size_t)k * 4);
    L.off_head = take(std::max<size_t>(nchunks, 1) * D * 4);
    L.off_tail = take(std::max<size_t>(nchunks, 1) * D * 4);
    L.off_headw = take(std::max<size_t>(nchunks, 1) * 4);
    L.off_tailw = take(std::max<size_t>(nchunks, 1) * 4);
    L.off_c0 = take((size_t)k * D * 4);
    L.off_c1 = take((size_t)k * D * 4);
    L.off_w = take((size_t)k * 4);
    L.off_n = take(16);
    L.bytes = o;
    L.npts = npts;
    L.k = k;
    L.D = D;
    return L;
}

template <class P, int NP, int PIPE>
static hipError_t launch_assign_np(lam_ctx* ctx, const float* X, int n, int D, const typename P::T* Cf,
                                   const float* cn, int kp, int k, float* best_v, uint32_t* a, float* d2,
                                   hipStream_t st)
{
    auto kern = k_km_assign<P, NP, PIPE>;
    const size_t lds_max = (size_t)32 * NP * D * P::kBytes + (size_t)kSlice * 4 + (size_t)2 * 4 * 32 * NP * 4;
    hipError_t el = ctx_ensure_lds(ctx, (const void*)kern, lds_max);
    if (el != hipSuccess) return el;
    const int blocks = (n + 32 * NP - 1) / (32 * NP);
    const int nc = D / 16;
    const int slices = (kp + kSlice - 1) / kSlice;
    ProfScope ps(ctx, "kmeans_assign", st);
    for (int s = 0; s < slices; ++s) {
        const int kbase = s * kSlice, kcp = std::min(kSlice, kp - kbase);
        const bool last = s == slices - 1;
        const size_t lds = (size_t)32 * NP * D * P::kBytes + (size_t)kcp * 4 + (size_t)2 * 4 * 32 * NP * 4;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kAssignThreads), lds, st, X, n, D,
                           Cf + (size_t)(kbase / 32) * nc * 512, cn + kbase, kcp, kbase, k, s > 0 ? 1 : 0,
                           slices > 1 ? best_v : nullptr, a, last ? d2 : nullptr);
    }
    return hipGetLastError();
}

template <class P, int NP>
static hipError_t launch_assign_pipe(lam_ctx* ctx, const float* X, int n, int D, const typename P::T* Cf,
                                     const float* cn, int kp, int k, float* best_v, uint32_t* a, float* d2,
                                     hipStream_t st)
{
    if ((D / 16) % 4 == 0) return launch_assign_np<P, NP, 4>(ctx, X, n, D, Cf, cn, kp, k, best_v, a, d2, st);
    return launch_assign_np<P, NP, 2>(ctx, X, n, D, Cf, cn, kp, k, best_v, a, d2, st);
}

template <class P>
static hipError_t launch_assign_p(lam_ctx* ctx, const float* X, int n, int D, const float* C, int k, const KmLayout& L,
                                  char* base, uint32_t* a, float* d2, hipStream_t st)
{
    const int kp = (int)align_up((size_t)k, kCentreAlign);
    auto* Cf = reinterpret_cast<typename P::T*>(base + L.off_cf);
    float* cn = reinterpret_cast<float*>(base + L.off_cn);
    float* best_v = reinterpret_cast<float*>(base + L.off_bv);
    const size_t groups = (size_t)kp * (D / 8);
    hipLaunchKernelGGL(k_km_prep<P>, dim3((unsigned)std::min<size_t>((groups + 255) / 256, 4096)), dim3(256), 0,
                       st, C, k, kp, D, Cf);
    hipLaunchKernelGGL(k_km_norms, dim3((kp + 3) / 4), dim3(256), 0, st, C, k, kp, D, cn);
    if (n == 0) return hipGetLastError();
    const int bp = tile_points(P::kBytes == 2 ? LAM_BF16 : LAM_FP32, D);
    if (bp == 64) return launch_assign_pipe<P, 2>(ctx, X, n, D, Cf, cn, kp, k, best_v, a, d2, st);
    return launch_assign_pipe<P, 1>(ctx, X, n, D, Cf, cn, kp, k, best_v, a, d2, st);
}

hipError_t kmeans_assign_launch(lam_ctx* ctx, int prec, const float* X, int n, int D, const float* C, int k, const KmLayout& L,
                                void* ws, uint32_t* a, float* d2, hipStream_t st)
{
    char* base = static_cast<char*>(ws);
    uint32_t* aa = a ? a : reinterpret_cast<uint32_t*>(base + L.off_a);
    if (prec == LAM_BF16) return launch_assign_p<PBF16>(ctx, X, n, D, C, k, L, base, aa, d2, st);
    return launch_assign_p<PF32>(ctx, X, n, D, C, k, L, base, aa, d2, st);
}

template <int CG>
static void launch_update_cg(const float* X, const float* w, int n, int D, const uint32_t* skeys,
                             const uint32_t* sidx, const uint32_t* start, const uint32_t* end, int k,
                             const float* Cold, float* Cnew, float* Wnew, float* head, float* tail, float* headw,
                             float* tailw, hipStream_t st)
{
    const int nchunks = (n + kChunk - 1) / kChunk;
    if (nchunks > 0)
        hipLaunchKernelGGL(k_km_chunks<CG>, dim3(nchunks), dim3(128), 0, st, X, w, n, D, skeys, sidx, Cold, Cnew,
                           Wnew, head, tail, headw, tailw);
    hipLaunchKernelGGL(k_km_fixup<CG>, dim3(k), dim3(128), 0, st, start, end, n, D, Cold, Cnew, Wnew, head, tail,
                       headw, tailw);
}

// Means of the assigned points (assignments in the workspace's a buffer).
static hipError_t kmeans_update(const float* X, const float* w, int n, int D, int k, const float* Cold,
                                float* Cnew, float* Wnew, const KmLayout& L, char* base, hipStream_t st)
{
    uint32_t* a = reinterpret_cast<uint32_t*>(base + L.off_a);
    uint32_t* ka = reinterpret_cast<uint32_t*>(base + L.off_ka);
    uint32_t* va = reinterpret_cast<uint32_t*>(base + L.off_va);
    uint32_t* kb = reinterpret_cast<uint32_t*>(base + L.off_kb);
    uint32_t* vb = reinterpret_cast<uint32_t*>(base + L.off_vb);
    uint32_t* scratch = reinterpret_cast<uint32_t*>(base + L.off_sort);
    uint32_t* start = reinterpret_cast<uint32_t*>(base + L.off_start);
    uint32_t* end = reinterpret_cast<uint32_t*>(base + L.off_end);
    uint32_t* ndev = reinterpret_cast<uint32_t*>(base + L.off_n);
    float* head = reinterpret_cast<float*>(base + L.off_head);
    float* tail = reinterpret_cast<float*>(base + L.off_tail);
    float* headw = reinterpret_cast<float*>(base + L.off_headw);
    float* tailw = reinterpret_cast<float*>(base + L.off_tailw);
    hipError_t e = launch_fill_u32(ndev, 1, (uint32_t)n, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(start, (size_t)k, 0u, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(end, (size_t)k, 0u, st);
    if (e != hipSuccess) return e;
    const uint32_t* skeys = a;
    const uint32_t* sidx = nullptr;
    if (n > 0) {
        bool in_b = false;
        e = launch_radix_sort(a, ka, va, kb, vb, true, ndev, (uint32_t)n, kmeans_key_bits(k), scratch, true,
                              nullptr, &in_b, st);
        if (e != hipSuccess) return e;
        skeys = in_b ? kb : ka;
        sidx = in_b ? vb : va;
        hipLaunchKernelGGL(k_km_ranges, dim3((n + 255) / 256), dim3(256), 0, st, skeys, n, start, end);
    }
    const int cg = (D / 4 + 127) / 128;
    switch (cg) {
    case 1: launch_update_cg<1>(X, w, n, D, skeys, sidx, start, end, k, Cold, Cnew, Wnew, head, tail, headw, tailw, st); break;
    case 2: launch_update_cg<2>(X, w, n, D, skeys, sidx, start, end, k, Cold, Cnew, Wnew, head, tail, headw, tailw, st); break;
    case 3: launch_update_cg<3>(X, w, n, D, skeys, sidx, start, end, k, Cold, Cnew, Wnew, head, tail, headw, tailw, st); break;
    default: launch_update_cg<4>(X, w, n, D, skeys, sidx, start, end, k, Cold, Cnew, Wnew, head, tail, headw, tailw, st); break;
    }
    return hipGetLastError();
}

hipError_t kmeans_lloyd_launch(lam_ctx* ctx, int prec, const float* X, const float* w, int n, int D, const float* C0, int k,
                               int iters, float* C, float* W, uint32_t* a_out, const KmLayout& L, void* ws,
                               hipStream_t st)
{
    char* base = static_cast<char*>(ws);
    float* cbuf[2] = {reinterpret_cast<float*>(base + L.off_c0), reinterpret_cast<float*>(base + L.off_c1)};
    float* wbuf = reinterpret_cast<float*>(base + L.off_w);
    uint32_t* a = reinterpret_cast<uint32_t*>(base + L.off_a);
    ProfScope ps(ctx, "kmeans", st);
    const float* cur = C0;
    for (int it = 0; it < iters; ++it) {
        const bool last = it == iters - 1;
        float* next = last ? C : cbuf[it & 1];
        float* wn = (last && W) ? W : wbuf;
        hipError_t e = kmeans_assign_launch(ctx, prec, X, n, D, cur, k, L, ws, a, nullptr, st);
        if (e != hipSuccess) return e;
        e = kmeans_update(X, w, n, D, k, cur, next, wn, L, base, st);
        if (e != hipSuccess) return e;
        cur = next;
    }
    if (a_out && n > 0) {
        hipError_t e = hipMemcpyAsync(a_out, a, (size_t)n * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

StreamKmLayout stream_kmeans_layout(int prec, int n, int D, int Kp, int K, int m)
{
    StreamKmLayout S{};
    const int npts = std::max(n, Kp + m);
    const int kc = std::max(m, K);
    S.lloyd = kmeans_layout(prec, npts, D, std::max(kc, 1));
    size_t o = align_up(S.lloyd.bytes, 256);
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    S.off_m0 = take((size_t)m * D * 4);
    S.off_mc = take((size_t)m * D * 4);
    S.off_mw = take((size_t)m * 4);
    S.off_p = take((size_t)(Kp + m) * D * 4);
    S.off_pw = take((size_t)(Kp + m) * 4);
    S.off_g0 = take((size_t)K * D * 4);
    S.off_seeds = take((size_t)m * 4);
    S.bytes = o;
    return S;
}

hipError_t stream_kmeans_launch(lam_ctx* ctx, int prec, const float* F, int n, int D, const float* Dprev, const float* wprev,
                                int Kp, int K, const int32_t* seeds_host, int m, int iters_local, int iters_global,
                                float* Dout, float* Wout, const StreamKmLayout& S, void* ws, hipStream_t st)
{
    char* base = static_cast<char*>(ws);
    float* M0 = reinterpret_cast<float*>(base + S.off_m0);
    float* Mc = reinterpret_cast<float*>(base + S.off_mc);
    float* Mw = reinterpret_cast<float*>(base + S.off_mw);
    float* P = reinterpret_cast<float*>(base + S.off_p);
    float* Pw = reinterpret_cast<float*>(base + S.off_pw);
    float* G0 = reinterpret_cast<float*>(base + S.off_g0);
    int32_t* seeds = reinterpret_cast<int32_t*>(base + S.off_seeds);
    const size_t row = (size_t)D * 4;
    hipError_t e;
    if (m > 0) {
        e = hipMemcpyAsync(seeds, seeds_host, (size_t)m * 4, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_km_gather, dim3(m), dim3(128), 0, st, F, D, (const int32_t*)seeds, m, M0);
        e = kmeans_lloyd_launch(ctx, prec, F, nullptr, n, D, M0, m, iters_local, Mc, Mw, nullptr, S.lloyd, ws, st);
        if (e != hipSuccess) return e;
    }
    // merged weighted set [D_prev; micro] and the initial centres [D_prev; micro[0 .. K - Kp)]
    if (Kp > 0) {
        e = hipMemcpyAsync(P, Dprev, (size_t)Kp * row, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(Pw, wprev, (size_t)Kp * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(G0, Dprev, (size_t)Kp * row, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    if (m > 0) {
        e = hipMemcpyAsync(P + (size_t)Kp * D, Mc, (size_t)m * row, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(Pw + Kp, Mw, (size_t)m * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    if (K > Kp) {
        e = hipMemcpyAsync(G0 + (size_t)Kp * D, Mc, (size_t)(K - Kp) * row, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return kmeans_lloyd_launch(ctx, prec, P, Pw, Kp + m, D, G0, K, iters_global, Dout, Wout, nullptr, S.lloyd, ws, st);
}

}  // namespace km
}  // namespace lam

// ------------------------------------------------------------ C ABI

using namespace lam;
using namespace lam::km;

static bool km_aligned(const void* p) { return ((uintptr_t)p & 15u) == 0; }

extern "C" {

lam_status lam_kmeans_workspace_size(const lam_ctx* ctx, int precision, int n, int D, int k, uint64_t* bytes)
{
    if (!bytes || n < 0) return LAM_ERR_INVALID_ARG;
    if (!kmeans_shape_ok(precision, D, k) || n >= (1 << 30)) return LAM_ERR_UNSUPPORTED;
    *bytes = kmeans_layout(precision, n, D, k).bytes;
    return LAM_OK;
}

lam_status lam_kmeans_assign(lam_ctx* ctx, int precision, const float* X, int n, int D, const float* C, int k, int32_t* assign,
                             float* d2, void* ws, uint64_t ws_bytes, void* stream)
{
    if (!ctx_ok(ctx) || n < 0) return LAM_ERR_INVALID_ARG;
    if (!kmeans_shape_ok(precision, D, k) || n >= (1 << 30)) return LAM_ERR_UNSUPPORTED;
    const KmLayout L = kmeans_layout(precision, n, D, k);
    if (!ws || ws_bytes < L.bytes || !C || (n > 0 && (!X || !assign))) return LAM_ERR_INVALID_ARG;
    if (!km_aligned(X) || !km_aligned(C)) return LAM_ERR_INVALID_ARG;
    return kmeans_assign_launch(ctx, precision, X, n, D, C, k, L, ws, reinterpret_cast<uint32_t*>(assign), d2,
                                (hipStream_t)stream) == hipSuccess
               ? LAM_OK
               : LAM_ERR_HIP;
}

lam_status lam_kmeans_lloyd(lam_ctx* ctx, int precision, const float* X, const float* weights, int n, int D, const float* C0,
                            int k, int iters, float* C, float* W, int32_t* assign, void* ws, uint64_t ws_bytes,
                            void* stream)
{
    if (!ctx_ok(ctx) || n < 0 || iters < 1) return LAM_ERR_INVALID_ARG;
    if (!kmeans_shape_ok(precision, D, k) || n >= (1 << 30)) return LAM_ERR_UNSUPPORTED;
    const KmLayout L = kmeans_layout(precision, n, D, k);
    if (!ws || ws_bytes < L.bytes || !C0 || !C || (n > 0 && !X)) return LAM_ERR_INVALID_ARG;
    if (!km_aligned(X) || !km_aligned(C0) || !km_aligned(C)) return LAM_ERR_INVALID_ARG;
    return kmeans_lloyd_launch(ctx, precision, X, weights, n, D, C0, k, iters, C, W,
                               reinterpret_cast<uint32_t*>(assign), L, ws, (hipStream_t)stream) == hipSuccess
               ? LAM_OK
               : LAM_ERR_HIP;
}

lam_status lam_stream_kmeans_workspace_size(const lam_ctx* ctx, int precision, int n, int D, int Kp, int K, int m, uint64_t* bytes)
{
    if (!bytes || n < 0 || Kp < 0 || m < 0 || m > n || Kp > K || m < K - Kp) return LAM_ERR_INVALID_ARG;
    if (!kmeans_shape_ok(precision, D, std::max(std::max(m, K), 1)) || (size_t)Kp + m >= (size_t)1 << 30)
        return LAM_ERR_UNSUPPORTED;
    *bytes = stream_kmeans_layout(precision, n, D, Kp, K, m).bytes;
    return LAM_OK;
}

lam_status lam_stream_kmeans(lam_ctx* ctx, int precision, const float* F, int n, int D, const float* D_prev,
                             const float* w_prev, int Kp, int K, const int32_t* seeds, int m, int iters_local,
                             int iters_global, float* D_out, float* W_out, void* ws, uint64_t ws_bytes,
                             void* stream)
{
    if (!ctx_ok(ctx) || n < 0 || Kp < 0 || m < 0 || m > n || Kp > K || m < K - Kp || iters_global < 1 ||
        (m > 0 && iters_local < 1))
        return LAM_ERR_INVALID_ARG;
    if (!kmeans_shape_ok(precision, D, std::max(std::max(m, K), 1))) return LAM_ERR_UNSUPPORTED;
    const StreamKmLayout S = stream_kmeans_layout(precision, n, D, Kp, K, m);
    if (!ws || ws_bytes < S.bytes || !D_out || !W_out) return LAM_ERR_INVALID_ARG;
    if ((m > 0 && (!F || !seeds)) || (Kp > 0 && (!D_prev || !w_prev))) return LAM_ERR_INVALID_ARG;
    if (!km_aligned(F) || !km_aligned(D_prev) || !km_aligned(D_out)) return LAM_ERR_INVALID_ARG;
    for (int i = 0; i < m; ++i)
        if (seeds[i] < 0 || seeds[i] >= n) return LAM_ERR_INVALID_ARG;
    return stream_kmeans_launch(ctx, precision, F, n, D, D_prev, w_prev, Kp, K, seeds, m, iters_local, iters_global,
                                D_out, W_out, S, ws, (hipStream_t)stream) == hipSuccess
               ? LAM_OK
               : LAM_ERR_HIP;
}

}  // extern "C"
