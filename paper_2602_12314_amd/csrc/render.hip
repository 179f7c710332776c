// Query-map rendering (paper Eq. 2 and Eq. 4) and its adjoint on gfx950.
//
// Pipeline of one forward call (one HIP stream, no host synchronisation):
//   k_preprocess      one thread per (camera, Gaussian) record, float32 projection:
//                     screen mean, conic, opacity, integer footprint, depth key
//   radix sort        records by float32 depth bits (stable: ties by record)
//   scan + k_emit     (tile id, record) pairs emitted in depth order
//   radix sort        pairs by tile id (stable, so each tile stays depth-ordered)
//   k_ranges          [start, end) of every tile's list
//   k_raster_fwd      one workgroup per tile; the tile's list is staged through
//                     LDS 256 records at a time; each thread blends one pixel
// The backward walks each pixel's list back to front, rebuilding the
// transmittance by division, reduces the per-Gaussian terms across the wave
// with DPP and adds them with one atomic per wave; k_preprocess_bwd chains the
// screen-space gradients to the raw parameters.
#include "common.h"
#include "kernels.h"

namespace lam {

// ------------------------------------------------------------- preprocess

// exp(x) in float32 by Cody-Waite reduction and a Taylor polynomial: k =
// rint(x log2 e), r = (x - k ln2_hi) - k ln2_lo with ln2_hi carrying 15
// significant bits (so k ln2_hi is exact for |k| < 256), exp(r) to degree 7 by
// Horner with fused multiply-adds (|r| <= ln2 / 2: truncation below 2^-25),
// scaled by 2^k.  Every step is a correctly rounded float32 operation, so the
// result is a fixed function of x, reproducible bit for bit by any IEEE float32
// implementation of the same steps.
__device__ inline float exp_cw(float x)
{
#pragma clang fp contract(off)
    x = fminf(fmaxf(x, -87.0f), 88.0f);
    const float k = rintf(x * 1.44269504f);
    const float r = (x - k * 0.693145751953125f) - k * 1.42860677e-06f;
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)k);
}

// Record outputs: rec0 = (u, v, 0, 0) (the last two words, a low-order part
// of the screen mean, are zero for a float32 projection), rec1 = (A, B, C,
// opacity) with power = -0.5 (A dx^2 + C dy^2) - B dx dy, foot = (x0 | x1 << 16,
// y0 | y1 << 16) the inclusive pixel footprint.
//
// The projection is float32 with every operation written out and rounded on
// its own (no contraction; division and square root correctly rounded;
// exp_cw above), in the order below, so that the integer decisions it takes
// (culling, radius, footprint, depth key) are a fixed function of the float32
// inputs.
//
// The launch also clears the forward's counters and look-back scratch
// (zero[0 .. zero_words)), which the sorts after it need at zero: one launch
// fewer than a separate fill.
__global__ __launch_bounds__(256) void k_preprocess(
    CamSet cs, int N, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits, float4* __restrict__ rec0,
    float4* __restrict__ rec1, uint2* __restrict__ foot, uint32_t* __restrict__ depth_key,
    uint32_t* __restrict__ ntiles, uint32_t* __restrict__ zero, size_t zero_words)
{
#pragma clang fp contract(off)
    {
        const size_t nthreads = (size_t)gridDim.x * gridDim.y * blockDim.x;
        for (size_t k = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; k < zero_words;
             k += nthreads)
            zero[k] = 0u;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const Cam& cam = cs.c[blockIdx.y];
    const size_t r = (size_t)blockIdx.y * N + i;

    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    float Wm[3][3], t[3];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) Wm[a][b] = cam.vm[4 * a + b];
        t[a] = cam.vm[4 * a + 3];
    }
    const float x = ((Wm[0][0] * mx + Wm[0][1] * my) + Wm[0][2] * mz) + t[0];
    const float y = ((Wm[1][0] * mx + Wm[1][1] * my) + Wm[1][2] * mz) + t[1];
    const float z = ((Wm[2][0] * mx + Wm[2][1] * my) + Wm[2][2] * mz) + t[2];

    bool vis = z > kNear;
    float s[3], qn[4];
    if (vis) {
        for (int k = 0; k < 3; ++k) s[k] = exp_cw(log_scales[3 * i + k]);
        const float q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
        const float nrm = sqrtf(((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3);
        vis = nrm > 0.0f;
        qn[0] = q0 / nrm; qn[1] = q1 / nrm; qn[2] = q2 / nrm; qn[3] = q3 / nrm;
    }
    float a = 0, b = 0, c = 0, det = 0, u = 0, v = 0, radius = 0;
    if (vis) {
        const float w = qn[0], qx = qn[1], qy = qn[2], qz = qn[3];
        const float Rg[3][3] = {
            {1.0f - 2.0f * (qy * qy + qz * qz), 2.0f * (qx * qy - w * qz), 2.0f * (qx * qz + w * qy)},
            {2.0f * (qx * qy + w * qz), 1.0f - 2.0f * (qx * qx + qz * qz), 2.0f * (qy * qz - w * qx)},
            {2.0f * (qx * qz - w * qy), 2.0f * (qy * qz + w * qx), 1.0f - 2.0f * (qx * qx + qy * qy)}};
        float S3[3][3], Sc[3][3];
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                float acc = 0.0f;
                for (int k = 0; k < 3; ++k) acc = acc + ((Rg[p][k] * s[k]) * s[k]) * Rg[q][k];
                S3[p][q] = acc;
            }
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                float acc = 0.0f;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc = acc + (Wm[p][k] * S3[k][l]) * Wm[q][l];
                Sc[p][q] = acc;
            }
        const float fx = cam.fx, fy = cam.fy;
        const float limx = kFovClamp * ((float)cam.w / (2.0f * fx));
        const float limy = kFovClamp * ((float)cam.h / (2.0f * fy));
        float tx = x / z, ty = y / z;
        tx = tx < -limx ? -limx : (tx > limx ? limx : tx);
        ty = ty < -limy ? -limy : (ty > limy ? limy : ty);
        const float J[2][3] = {{fx / z, 0.0f, (-fx * tx) / z}, {0.0f, fy / z, (-fy * ty) / z}};
        float cov[2][2];
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
                float acc = 0.0f;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc = acc + (J[p][k] * Sc[k][l]) * J[q][l];
                cov[p][q] = acc;
            }
        a = cov[0][0] + kDilation;
        b = cov[0][1];
        c = cov[1][1] + kDilation;
        det = a * c - b * b;
        vis = det > 0.0f;
        if (vis) {
            const float mid = 0.5f * (a + c);
            const float lam = mid + sqrtf(fmaxf(kEigFloor, mid * mid - det));
            radius = ceilf(kSigmas * sqrtf(lam));
            u = (fx * x) / z + cam.cx;
            v = (fy * y) / z + cam.cy;
            vis = (u + radius >= 0.0f) && (u - radius <= (float)(cam.w - 1)) && (v + radius >= 0.0f) &&
                  (v - radius <= (float)(cam.h - 1));
        }
    }
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    if (vis) {
        const float fx0 = ceilf(u - radius), fx1 = floorf(u + radius);
        const float fy0 = ceilf(v - radius), fy1 = floorf(v + radius);
        x0 = fx0 < 0.0f ? 0 : (int)fx0;
        x1 = fx1 > (float)(cam.w - 1) ? cam.w - 1 : (int)fx1;
        y0 = fy0 < 0.0f ? 0 : (int)fy0;
        y1 = fy1 > (float)(cam.h - 1) ? cam.h - 1 : (int)fy1;
        vis = x0 <= x1 && y0 <= y1;
    }
    if (!vis) {
        depth_key[r] = 0xFFFFFFFFu;
        ntiles[r] = 0u;
        foot[r] = make_uint2(0u, 0u);
        return;
    }
    rec0[r] = make_float4(u, v, 0.0f, 0.0f);
    const float o = 1.0f / (1.0f + exp_cw(-logits[i]));
    rec1[r] = make_float4(c / det, -b / det, a / det, o);
    foot[r] = make_uint2((uint32_t)x0 | ((uint32_t)x1 << 16), (uint32_t)y0 | ((uint32_t)y1 << 16));
    depth_key[r] = __float_as_uint(z);
    const int nx = (x1 >> cs.tile_shift_x) - (x0 >> cs.tile_shift_x) + 1;
    const int ny = (y1 >> cs.tile_shift_y) - (y0 >> cs.tile_shift_y) + 1;
    ntiles[r] = (uint32_t)(nx * ny);
}

// One thread per emitted (tile id, record) pair, so Gaussians covering many
// tiles do not serialise one thread.  Pair o belongs to the depth-sorted
// record s with offsets[s] <= o < offsets[s + 1], and is that record's
// (o - offsets[s])-th tile of its footprint, rows outer.  A workgroup takes
// chunks of 256 consecutive pairs, a contiguous range of them: every visible
// record emits at least one pair and culled records (key 0xFFFFFFFF) sort
// last, so a chunk's pairs belong to a run of at most 256 consecutive
// records.  The run's offsets are staged in LDS and each thread finds its
// record there.  The first record of the workgroup's first chunk is found by
// rounds of 256 probes, each narrowing the range 256-fold (three rounds for
// up to 2^24 records instead of one dependent load per halving); that of each
// later chunk is read off the staged run of the chunk before it, unless the
// run ends first (then the probes again).
__global__ __launch_bounds__(256) void k_emit(CamSet cs, int N, uint32_t R,
                                             const uint32_t* __restrict__ sorted_rec,
                                             const uint32_t* __restrict__ offsets,
                                             const uint2* __restrict__ foot,
                                             const uint32_t* __restrict__ counters, uint32_t cap,
                                             uint32_t* __restrict__ keys,
                                             uint32_t* __restrict__ vals)
{
    __shared__ uint32_t run[257];
    __shared__ uint32_t next_s0;
    const uint32_t total = counters[0] < cap ? counters[0] : cap;
    const uint32_t nchunks = (total + 255) / 256;
    const uint32_t per = (nchunks + gridDim.x - 1) / gridDim.x;
    const uint32_t c0 = blockIdx.x * per;
    const uint32_t c1 = c0 + per < nchunks ? c0 + per : nchunks;
    bool known = false;  // next_s0 holds the first record of chunk c
    for (uint32_t c = c0; c < c1; ++c) {
        const uint32_t o0 = c * 256u;
        uint32_t s0;
        if (known) {
            s0 = next_s0;
        } else {
            // largest s in [lo, hi) with offsets[s] <= o0 (offsets[0] = 0 <= o0)
            uint32_t lo = 0, hi = R;
            while (hi - lo > 1) {
                const uint32_t stride = (hi - lo + 255) / 256;
                const uint32_t idx = lo + threadIdx.x * stride;
                const int le = idx < hi && offsets[idx] <= o0;
                const uint32_t k = (uint32_t)__syncthreads_count(le);  // a prefix of the probes
                const uint32_t nlo = lo + (k - 1) * stride;
                hi = nlo + stride < hi ? nlo + stride : hi;
                lo = nlo;
            }
            s0 = lo;
        }
        const uint32_t si = s0 + threadIdx.x;
        run[threadIdx.x] = si < R ? offsets[si] : 0xFFFFFFFFu;
        if (threadIdx.x == 0) run[256] = s0 + 256 < R ? offsets[s0 + 256] : 0xFFFFFFFFu;
        __syncthreads();
        const uint32_t o = o0 + threadIdx.x;
        if (o < total) {
            uint32_t a = 0, b = 257;  // largest j with run[j] <= o; run[0] <= o
            while (b - a > 1) {
                const uint32_t m = (a + b) >> 1;
                if (run[m] <= o) a = m;
                else b = m;
            }
            const uint32_t s = s0 + a;
            const uint32_t r = sorted_rec[s];
            const int cam = (int)(r / (uint32_t)N);
            int tbase = 0, tx_n = 1;
            for (int k = 0; k < cs.n; ++k)
                if (k == cam) { tbase = cs.c[k].tile_base; tx_n = cs.c[k].tiles_x; }
            const uint2 f = foot[r];
            const int x0 = (f.x & 0xFFFF) >> cs.tile_shift_x, x1 = (f.x >> 16) >> cs.tile_shift_x;
            const int y0 = (f.y & 0xFFFF) >> cs.tile_shift_y;
            const int nx = x1 - x0 + 1;
            const int k = (int)(o - run[a]);
            const int ty = y0 + k / nx, tx = x0 + k % nx;
            keys[o] = (uint32_t)(tbase + ty * tx_n + tx);
            vals[o] = r;
        }
        // the next chunk's first record: the largest j with run[j] <= o0 + 256,
        // if the run reaches past that pair (run[256] > o0 + 256)
        const uint32_t on = o0 + 256u;
        known = run[256] > on;
        if (known && threadIdx.x == 0) {
            uint32_t a = 0, b = 257;
            while (b - a > 1) {
                const uint32_t m = (a + b) >> 1;
                if (run[m] <= on) a = m;
                else b = m;
            }
            next_s0 = s0 + a;
        }
        __syncthreads();  // run[] is rewritten by the next chunk; next_s0 is read
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// [start, end) of every tile's list in the tile-sorted pairs, empty tiles
// included, with no fill first: boundary i (0 <= i <= n) looks at the keys on
// both sides and, where they differ, ends the tile before, starts the tile
// after and gives every tile id strictly between them the empty range (0, 0).
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys,
                                               const uint32_t* __restrict__ counters, uint32_t cap,
                                               uint32_t tiles, uint2* __restrict__ ranges)
{
    const uint32_t n = counters[0] < cap ? counters[0] : cap;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        const uint32_t a = i > 0 ? keys[i - 1] : 0u;
        const uint32_t b = i < n ? keys[i] : tiles;
        if (i > 0 && i < n && a == b) continue;
        if (i > 0 && a < tiles) ranges[a].y = i;
        for (uint32_t t = i > 0 ? a + 1 : 0u; t < b && t < tiles; ++t) ranges[t] = make_uint2(0u, 0u);
        if (i < n && b < tiles) ranges[b].x = i;
    }
}

// ------------------------------------------------------------- raster fwd

constexpr int kChunk = 256;

// RGBD: each staged entry also carries (colour r, g, b, camera-space depth z)
// of its record, blended with the same weights as the query (Eq. 2: colour;
// depth by the same alpha blending).
template <int DQ, bool RGBD>
struct TileStage {
    float4 r0[kChunk];
    float4 r1[kChunk];
    uint2 fp[kChunk];
    uint32_t rec[kChunk];
    float q[kChunk * DQ];
    float4 x[RGBD ? kChunk : 1];
};

// Colour and depth of one record; the depth is the float32 camera-space z the
// depth sort keys hold (positive, so its bits are the key).
__device__ inline float4 rgbz(const float* __restrict__ colors, const uint32_t* __restrict__ depth_key,
                              uint32_t r, uint32_t g)
{
    return make_float4(colors[3 * (size_t)g], colors[3 * (size_t)g + 1], colors[3 * (size_t)g + 2],
                       __uint_as_float(depth_key[r]));
}

template <int DQ, bool RGBD>
__device__ inline void stage_chunk(TileStage<DQ, RGBD>& st, int k, uint32_t end, int base_tile_c,
                                   int N, const uint32_t* __restrict__ tile_recs,
                                   const float4* __restrict__ rec0,
                                   const float4* __restrict__ rec1,
                                   const uint2* __restrict__ foot,
                                   const float* __restrict__ queries,
                                   const float* __restrict__ colors,
                                   const uint32_t* __restrict__ depth_key)
{
    const int t = threadIdx.x;
    if ((uint32_t)k < end) {
        const uint32_t r = tile_recs[k];
        st.r0[t] = rec0[r];
        st.r1[t] = rec1[r];
        st.fp[t] = foot[r];
        st.rec[t] = r;
        const uint32_t g = r - (uint32_t)base_tile_c * (uint32_t)N;
        const float4* qs = reinterpret_cast<const float4*>(queries + (size_t)g * DQ);
        float4* qd = reinterpret_cast<float4*>(st.q + t * DQ);
#pragma unroll
        for (int j = 0; j < DQ / 4; ++j) qd[j] = qs[j];
        if constexpr (RGBD) st.x[t] = rgbz(colors, depth_key, r, g);
    }
}

template <int DQ, bool RGBD>
__device__ inline void raster_fwd_tile(
    TileStage<DQ, RGBD>& st, const int tile, const CamSet& cs, int N, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ tile_recs, const float4* __restrict__ rec0,
    const float4* __restrict__ rec1, const uint2* __restrict__ foot,
    const float* __restrict__ queries, float* __restrict__ Q, float* __restrict__ T_final,
    float* __restrict__ T_save, uint32_t* __restrict__ n_contrib, const float* __restrict__ colors,
    const uint32_t* __restrict__ depth_key, float* __restrict__ rgb, float* __restrict__ depth)
{
    const int c = cam_of_tile(cs, tile);
    const Cam& cam = cs.c[c];
    const int lt = tile - cam.tile_base;
    const int tyi = lt / cam.tiles_x, txi = lt - tyi * cam.tiles_x;
    const int px = (txi << cs.tile_shift_x) + (threadIdx.x & (cs.tile_w - 1));
    const int py = (tyi << cs.tile_shift_y) + (threadIdx.x >> cs.tile_shift_x);
    const bool inside = px < cam.w && py < cam.h;
    const uint2 rg = ranges[tile];

    float acc[DQ];
#pragma unroll
    for (int j = 0; j < DQ; ++j) acc[j] = 0.0f;
    float4 accx = make_float4(0.f, 0.f, 0.f, 0.f);
    float T = 1.0f;
    uint32_t last = 0;
    bool done = !inside;
    const float fpx = (float)px, fpy = (float)py;

    // one list entry staged per thread: chunks are as long as the workgroup
    const uint32_t chunk = blockDim.x;
    for (uint32_t base = rg.x; base < rg.y; base += chunk) {
        if (__syncthreads_count(done) == (int)blockDim.x) break;
        stage_chunk<DQ, RGBD>(st, (int)(base + threadIdx.x), rg.y, c, N, tile_recs, rec0, rec1, foot,
                              queries, colors, depth_key);
        __syncthreads();
        const int cnt = (int)min(chunk, rg.y - base);
        for (int j = 0; j < cnt && !done; ++j) {
            const uint2 f = st.fp[j];
            if (px < (int)(f.x & 0xFFFF) || px > (int)(f.x >> 16) || py < (int)(f.y & 0xFFFF) ||
                py > (int)(f.y >> 16))
                continue;
            const float4 a = st.r0[j];
            const float4 b = st.r1[j];
            const float dx = (a.x - fpx) + a.z;
            const float dy = (a.y - fpy) + a.w;
            const float power = -0.5f * (b.x * dx * dx + b.z * dy * dy) - b.y * dx * dy;
            const float oG = b.w * __expf(power);
            const float al = oG < kAlphaMax ? oG : kAlphaMax;
            if (al < kAlphaMin) continue;
            const float Tn = T * (1.0f - al);
            if (Tn < kTStop) {
                done = true;
                break;
            }
            const float wgt = al * T;
            const float* q = st.q + j * DQ;
#pragma unroll
            for (int k = 0; k < DQ; ++k) acc[k] += wgt * q[k];
            if constexpr (RGBD) {
                const float4 x = st.x[j];
                accx.x += wgt * x.x;
                accx.y += wgt * x.y;
                accx.z += wgt * x.z;
                accx.w += wgt * x.w;
            }
            T = Tn;
            last = base - rg.x + j + 1;
        }
    }
    if (inside) {
        const size_t p = (size_t)cam.pix_base + (size_t)py * cam.w + px;
        float4* qo = reinterpret_cast<float4*>(Q + p * DQ);
#pragma unroll
        for (int k = 0; k < DQ / 4; ++k)
            qo[k] = make_float4(acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]);
        T_final[p] = T;
        T_save[p] = T;
        n_contrib[p] = last;
        if constexpr (RGBD) {
            rgb[3 * p] = accx.x;
            rgb[3 * p + 1] = accx.y;
            rgb[3 * p + 2] = accx.z;
            depth[p] = accx.w;
        }
    }
}

// PERSIST = false: one workgroup per tile.  PERSIST = true: a grid of resident
// workgroups takes tiles from the queue counter until all are done, which
// evens out views of uneven size and tiles of uneven list length.
template <int DQ, bool PERSIST, bool RGBD>
__global__ __launch_bounds__(256) void k_raster_fwd(
    CamSet cs, int N, const uint2* __restrict__ ranges, const uint32_t* __restrict__ tile_recs,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const uint2* __restrict__ foot, const float* __restrict__ queries, float* __restrict__ Q,
    float* __restrict__ T_final, float* __restrict__ T_save, uint32_t* __restrict__ n_contrib,
    uint32_t* __restrict__ queue, const float* __restrict__ colors,
    const uint32_t* __restrict__ depth_key, float* __restrict__ rgb, float* __restrict__ depth)
{
    __shared__ TileStage<DQ, RGBD> st;
    if (!PERSIST) {
        raster_fwd_tile<DQ, RGBD>(st, blockIdx.x, cs, N, ranges, tile_recs, rec0, rec1, foot, queries, Q,
                                  T_final, T_save, n_contrib, colors, depth_key, rgb, depth);
        return;
    }
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();  // the previous tile is done with the staged lists
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int tile = __builtin_amdgcn_readfirstlane(s_tile);
        if (tile >= cs.total_tiles) break;
        raster_fwd_tile<DQ, RGBD>(st, tile, cs, N, ranges, tile_recs, rec0, rec1, foot, queries, Q, T_final,
                                  T_save, n_contrib, colors, depth_key, rgb, depth);
    }
}

// ------------------------------------------------------------- raster bwd

// The partner's copy of x in a halving step with lane mask M (1, 2, 4 or 8),
// through DPP inside a 16-lane row: lane ^ 1 and lane ^ 2 by quad permutes,
// lane ^ 8 by rotating the row by 8, and for M = 4 the mirror lane within the
// 8-lane half row (7 - i), whose M bit is also the opposite one.  A partner
// that differs in bits below M too is as good as lane ^ M: those bits are
// combined at the later steps all the same.
template <int M>
__device__ inline float partner(float x)
{
    constexpr int ctrl = M == 1 ? 0xB1 : M == 2 ? 0x4E : M == 4 ? 0x141 : 0x128;
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, false));
}

// Transposed wave reduction of N values: at the step with lane mask M a lane
// keeps the upper half of its values if its M bit is set, the lower half
// otherwise, and adds the partner's copy of the half it keeps.  For M = 32 and
// 16 one v_permlane32_swap / v_permlane16_swap of the pair (v[k], v[k + H])
// leaves, in every lane, its own kept value and the partner's copy of it in the
// two results (the swap trades the upper lanes of the first operand for the
// lower lanes of the second), so their sum is the step; the smaller masks use
// DPP.  No LDS traffic either way.
template <int N, int M>
__device__ inline void halving_sum(float* v, unsigned lane)
{
    if constexpr (N > 1 && M >= 1) {
        constexpr int H = N / 2;
        if constexpr (M == 32 || M == 16) {
#pragma unroll
            for (int k = 0; k < H; ++k) {
                const auto r = M == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]),
                                                                          __float_as_uint(v[k + H]), false, false)
                                       : __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]),
                                                                          __float_as_uint(v[k + H]), false, false);
                v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
            }
        } else {
            const bool upper = (lane & M) != 0;
#pragma unroll
            for (int k = 0; k < H; ++k) {
                const float send = upper ? v[k] : v[k + H];
                const float keep = upper ? v[k + H] : v[k];
                v[k] = keep + partner<M>(send);
            }
        }
        halving_sum<H, M / 2>(v, lane);
    }
}

// Wave sum of N values (N a power of two, 8 <= N <= 64): the halving steps
// over the masks 32 ... 64 / N, then the lanes that still differ in the lower
// mask bits add their partners' totals.  Afterwards the lanes whose low
// 6 - log2(N) bits are zero hold value lane >> (6 - log2(N)).
template <int N>
__device__ inline float wave_sum_split(float* v, unsigned lane)
{
    static_assert(N >= 8 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two in [8, 64]");
    constexpr int S = N == 8 ? 3 : N == 16 ? 2 : N == 32 ? 1 : 0;
    halving_sum<N, 32>(v, lane);
    if constexpr (S >= 3) v[0] += partner<4>(v[0]);
    if constexpr (S >= 2) v[0] += partner<2>(v[0]);
    if constexpr (S >= 1) v[0] += partner<1>(v[0]);
    return v[0];
}

// rec_grad[r] = (du, dv, dA, dB, dC, dopacity) accumulated over pixels; with
// RGBD also d_colors[g] and rec_dz[r] (the gradient of the record's depth).
template <int DQ, bool RGBD>
__device__ inline void raster_bwd_tile(
    TileStage<DQ, RGBD>& st, uint32_t& s_max, const int tile, const CamSet& cs, int N,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ tile_recs,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const uint2* __restrict__ foot, const float* __restrict__ queries,
    const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dQ, float* __restrict__ rec_grad, float* __restrict__ d_queries,
    const float* __restrict__ colors, const uint32_t* __restrict__ depth_key,
    const float* __restrict__ d_rgb, const float* __restrict__ d_depth, float* __restrict__ d_colors,
    float* __restrict__ rec_dz)
{
    const int c = cam_of_tile(cs, tile);
    const Cam& cam = cs.c[c];
    const int lt = tile - cam.tile_base;
    const int tyi = lt / cam.tiles_x, txi = lt - tyi * cam.tiles_x;
    const int px = (txi << cs.tile_shift_x) + (threadIdx.x & (cs.tile_w - 1));
    const int py = (tyi << cs.tile_shift_y) + (threadIdx.x >> cs.tile_shift_x);
    const bool inside = px < cam.w && py < cam.h;
    const uint2 rg = ranges[tile];
    const unsigned lane = __lane_id();

    float g[DQ], behind[DQ];
    float4 gx = make_float4(0.f, 0.f, 0.f, 0.f), behindx = gx;
    float T = 1.0f;
    uint32_t last = 0;
    if (inside) {
        const size_t p = (size_t)cam.pix_base + (size_t)py * cam.w + px;
        if constexpr (RGBD) gx = make_float4(d_rgb[3 * p], d_rgb[3 * p + 1], d_rgb[3 * p + 2], d_depth[p]);
        const float4* gi = reinterpret_cast<const float4*>(dQ + p * DQ);
#pragma unroll
        for (int k = 0; k < DQ / 4; ++k) {
            const float4 v = gi[k];
            g[4 * k] = v.x; g[4 * k + 1] = v.y; g[4 * k + 2] = v.z; g[4 * k + 3] = v.w;
        }
        T = T_final[p];
        last = n_contrib[p];
    } else {
#pragma unroll
        for (int k = 0; k < DQ; ++k) g[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < DQ; ++k) behind[k] = 0.0f;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, last);
    __syncthreads();
    const uint32_t maxlast = s_max;
    const float fpx = (float)px, fpy = (float)py;

    const int chunk = (int)blockDim.x;  // one staged entry per thread
    for (int end = (int)maxlast; end > 0; end -= chunk) {
        const int start = end > chunk ? end - chunk : 0;
        __syncthreads();
        stage_chunk<DQ, RGBD>(st, (int)(rg.x + start + threadIdx.x), rg.x + end, c, N, tile_recs, rec0,
                              rec1, foot, queries, colors, depth_key);
        __syncthreads();
        for (int j = end - 1; j >= start; --j) {
            const int sj = j - start;
            float gu = 0.f, gv = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, gO = 0.f, wq = 0.f;
            bool hit = false;
            if ((uint32_t)j < last) {
                const uint2 f = st.fp[sj];
                if (px >= (int)(f.x & 0xFFFF) && px <= (int)(f.x >> 16) &&
                    py >= (int)(f.y & 0xFFFF) && py <= (int)(f.y >> 16)) {
                    const float4 a = st.r0[sj];
                    const float4 b = st.r1[sj];
                    const float dx = (a.x - fpx) + a.z;
                    const float dy = (a.y - fpy) + a.w;
                    const float power = -0.5f * (b.x * dx * dx + b.z * dy * dy) - b.y * dx * dy;
                    const float G = __expf(power);
                    const float oG = b.w * G;
                    const float al = oG < kAlphaMax ? oG : kAlphaMax;
                    if (al >= kAlphaMin) {
                        hit = true;
                        // 1 - al >= 0.01: the hardware reciprocal (1 ulp) replaces the
                        // IEEE division sequence
                        T = T * __builtin_amdgcn_rcpf(1.0f - al);
                        wq = al * T;
                        const float* q = st.q + sj * DQ;
                        // B <- al q + (1 - al) B as B + al (q - B), the difference
                        // shared with the alpha gradient: three operations a channel
                        float dal = 0.0f;
#pragma unroll
                        for (int k = 0; k < DQ; ++k) {
                            const float df = q[k] - behind[k];
                            dal += df * g[k];
                            behind[k] += al * df;
                        }
                        if constexpr (RGBD) {
                            const float4 x = st.x[sj];
                            const float d0 = x.x - behindx.x, d1 = x.y - behindx.y;
                            const float d2 = x.z - behindx.z, d3 = x.w - behindx.w;
                            dal += d0 * gx.x + d1 * gx.y + d2 * gx.z + d3 * gx.w;
                            behindx.x += al * d0;
                            behindx.y += al * d1;
                            behindx.z += al * d2;
                            behindx.w += al * d3;
                        }
                        dal *= T;
                        if (oG < kAlphaMax) {
                            const float dp = dal * oG;
                            gu = -dp * (b.x * dx + b.y * dy);
                            gv = -dp * (b.z * dy + b.y * dx);
                            gA = -0.5f * dp * dx * dx;
                            gB = -dp * dx * dy;
                            gC = -0.5f * dp * dy * dy;
                            gO = dal * G;
                        }
                    }
                }
            }
            if (__ballot(hit) == 0ull) continue;
            if constexpr (!RGBD) {
                // The DQ query terms and the 6 screen-space terms (padded to 8)
                // summed over the wave as two sets, each by halving (no padding
                // of the query set to 32 or 64 values): lane l then holds query
                // term l >> (6 - log2 DQ) and screen term l >> 3.
                float vq[DQ], vs[8] = {gu, gv, gA, gB, gC, gO, 0.0f, 0.0f};
#pragma unroll
                for (int k = 0; k < DQ; ++k) vq[k] = wq * g[k];
                const float sq = wave_sum_split<DQ>(vq, lane);
                const float ss = wave_sum_split<8>(vs, lane);
                constexpr int SQ = DQ == 16 ? 2 : 1;
                const bool oq = (lane & ((1u << SQ) - 1u)) == 0 && sq != 0.0f;
                const bool os = (lane & 7u) == 0 && (lane >> 3) < 6 && ss != 0.0f;
                if (oq || os) {
                    const uint32_t r = st.rec[sj];
                    if (oq) unsafeAtomicAdd(d_queries + (size_t)(r - (uint32_t)c * (uint32_t)N) * DQ + (lane >> SQ), sq);
                    if (os) unsafeAtomicAdd(rec_grad + (size_t)r * 6 + (lane >> 3), ss);
                }
                continue;
            }
            // With RGBD: 6 screen-space terms, DQ query terms, 3 colour terms
            // and the depth term, padded to NV, summed over the wave by halving:
            // at each step a lane keeps half of its values and adds the partner's
            // copy of that half, so after log2(64) steps lane l holds the total of
            // value (l >> 1) (NV = 32) or l (NV = 64).
            constexpr int NX = RGBD ? 4 : 0;
            constexpr int NT = 6 + DQ + NX;
            constexpr int NV = (NT <= 32) ? 32 : 64;
            float v[NV];
            v[0] = gu; v[1] = gv; v[2] = gA; v[3] = gB; v[4] = gC; v[5] = gO;
#pragma unroll
            for (int k = 0; k < DQ; ++k) v[6 + k] = wq * g[k];
            if constexpr (RGBD) {
                v[6 + DQ] = wq * gx.x;
                v[7 + DQ] = wq * gx.y;
                v[8 + DQ] = wq * gx.z;
                v[9 + DQ] = wq * gx.w;
            }
#pragma unroll
            for (int k = NT; k < NV; ++k) v[k] = 0.0f;
            halving_sum<NV, 32>(v, lane);
            if (NV == 32) v[0] += partner<1>(v[0]);
            const int idx = NV == 32 ? (int)(lane >> 1) : (int)lane;
            const bool owner = (NV == 64 || (lane & 1) == 0) && idx < NT && v[0] != 0.0f;
            if (owner) {
                const uint32_t r = st.rec[sj];
                const size_t gi = (size_t)(r - (uint32_t)c * (uint32_t)N);
                float* dst = idx < 6 ? rec_grad + (size_t)r * 6 + idx
                           : idx < 6 + DQ ? d_queries + gi * DQ + (idx - 6)
                           : idx < 9 + DQ ? d_colors + gi * 3 + (idx - 6 - DQ)
                                          : rec_dz + r;
                unsafeAtomicAdd(dst, v[0]);
            }
        }
    }
}

template <int DQ, bool PERSIST, bool RGBD>
__global__ __launch_bounds__(256) void k_raster_bwd(
    CamSet cs, int N, const uint2* __restrict__ ranges, const uint32_t* __restrict__ tile_recs,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const uint2* __restrict__ foot, const float* __restrict__ queries,
    const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dQ, float* __restrict__ rec_grad, float* __restrict__ d_queries,
    uint32_t* __restrict__ queue, const float* __restrict__ colors,
    const uint32_t* __restrict__ depth_key, const float* __restrict__ d_rgb,
    const float* __restrict__ d_depth, float* __restrict__ d_colors, float* __restrict__ rec_dz)
{
    __shared__ TileStage<DQ, RGBD> st;
    __shared__ uint32_t s_max;
    if (!PERSIST) {
        raster_bwd_tile<DQ, RGBD>(st, s_max, blockIdx.x, cs, N, ranges, tile_recs, rec0, rec1, foot, queries,
                                  T_final, n_contrib, dQ, rec_grad, d_queries, colors, depth_key, d_rgb,
                                  d_depth, d_colors, rec_dz);
        return;
    }
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int tile = __builtin_amdgcn_readfirstlane(s_tile);
        if (tile >= cs.total_tiles) break;
        raster_bwd_tile<DQ, RGBD>(st, s_max, tile, cs, N, ranges, tile_recs, rec0, rec1, foot, queries,
                                  T_final, n_contrib, dQ, rec_grad, d_queries, colors, depth_key, d_rgb,
                                  d_depth, d_colors, rec_dz);
    }
}

// ------------------------------------------------------ preprocess adjoint

// Chains rec_grad of every camera back to the raw parameters of Gaussian i
// (FP32, matrix form of the chain rule), and rec_dz (nullable: the gradient of
// each record's rendered depth z = row 3 of the view transform applied to the
// mean) to the mean.  Outputs are overwritten.
__global__ __launch_bounds__(256) void k_preprocess_bwd(
    CamSet cs, int N, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const uint32_t* __restrict__ ntiles, const float* __restrict__ rec_grad,
    const float* __restrict__ rec_dz, float* __restrict__ d_means, float* __restrict__ d_log_scales,
    float* __restrict__ d_quats, float* __restrict__ d_logits)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float m0 = means[3 * i], m1 = means[3 * i + 1], m2 = means[3 * i + 2];
    float s[3];
    for (int k = 0; k < 3; ++k) s[k] = __expf(log_scales[3 * i + k]);
    const float q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
    const float qnorm = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const float iq = 1.0f / qnorm;
    const float w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
    float Rm[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                      {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                      {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
    float Mm[3][3];  // M = R diag(s)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Mm[a][b] = Rm[a][b] * s[b];
    float S3[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            S3[a][b] = Mm[a][0] * Mm[b][0] + Mm[a][1] * Mm[b][1] + Mm[a][2] * Mm[b][2];
    const float sig = 1.0f / (1.0f + __expf(-logits[i]));

    float gmean[3] = {0.f, 0.f, 0.f}, gS3[3][3] = {{0.f}}, glogit = 0.f;
    for (int ci = 0; ci < cs.n; ++ci) {
        const size_t r = (size_t)ci * N + i;
        if (ntiles[r] == 0) continue;
        const Cam& cam = cs.c[ci];
        const float* gr = rec_grad + r * 6;
        const float du = gr[0], dv = gr[1], dA = gr[2], dB = gr[3], dC = gr[4], dO = gr[5];
        glogit += dO * sig * (1.0f - sig);
        float W[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) W[a][b] = cam.vm[4 * a + b];
        const float cx = W[0][0] * m0 + W[0][1] * m1 + W[0][2] * m2 + cam.vm[3];
        const float cy = W[1][0] * m0 + W[1][1] * m1 + W[1][2] * m2 + cam.vm[7];
        const float cz = W[2][0] * m0 + W[2][1] * m1 + W[2][2] * m2 + cam.vm[11];
        const float limx = (float)kFovClamp * (cam.w / (2.0f * cam.fx));
        const float limy = (float)kFovClamp * (cam.h / (2.0f * cam.fy));
        const float rx = cx / cz, ry = cy / cz;
        const bool inx = rx >= -limx && rx <= limx, iny = ry >= -limy && ry <= limy;
        const float tx = inx ? rx : (rx < 0.f ? -limx : limx);
        const float ty = iny ? ry : (ry < 0.f ? -limy : limy);
        const float iz = 1.0f / cz;
        const float J[2][3] = {{cam.fx * iz, 0.f, -cam.fx * tx * iz}, {0.f, cam.fy * iz, -cam.fy * ty * iz}};
        // camera covariance Sc = W S3 W^T
        float WS[3][3], Sc[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) WS[a][b] = W[a][0] * S3[0][b] + W[a][1] * S3[1][b] + W[a][2] * S3[2][b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Sc[a][b] = WS[a][0] * W[b][0] + WS[a][1] * W[b][1] + WS[a][2] * W[b][2];
        // screen covariance and its inverse (the conic)
        float JS[2][3];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) JS[a][b] = J[a][0] * Sc[0][b] + J[a][1] * Sc[1][b] + J[a][2] * Sc[2][b];
        const float sa = JS[0][0] * J[0][0] + JS[0][1] * J[0][1] + JS[0][2] * J[0][2] + (float)kDilation;
        const float sb = JS[0][0] * J[1][0] + JS[0][1] * J[1][1] + JS[0][2] * J[1][2];
        const float sc = JS[1][0] * J[1][0] + JS[1][1] * J[1][1] + JS[1][2] * J[1][2] + (float)kDilation;
        const float idet = 1.0f / (sa * sc - sb * sb);
        const float Ci[2][2] = {{sc * idet, -sb * idet}, {-sb * idet, sa * idet}};
        // gradient w.r.t. the conic matrix (off-diagonal shared), then -Ci G Ci
        const float Gc[2][2] = {{dA, 0.5f * dB}, {0.5f * dB, dC}};
        float T1[2][2], G2[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) T1[a][b] = Ci[a][0] * Gc[0][b] + Ci[a][1] * Gc[1][b];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) G2[a][b] = -(T1[a][0] * Ci[0][b] + T1[a][1] * Ci[1][b]);
        // Sigma2 = J Sc J^T: G_Sc = J^T G2 J ; G_J = 2 G2 J Sc
        float GJ[2][3];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b)
                GJ[a][b] = 2.0f * (G2[a][0] * JS[0][b] + G2[a][1] * JS[1][b]);
        float GSc[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                GSc[a][b] = J[0][a] * (G2[0][0] * J[0][b] + G2[0][1] * J[1][b]) +
                            J[1][a] * (G2[1][0] * J[0][b] + G2[1][1] * J[1][b]);
        // Sc = W S3 W^T: G_S3 += W^T G_Sc W
        float GW[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) GW[a][b] = GSc[a][0] * W[0][b] + GSc[a][1] * W[1][b] + GSc[a][2] * W[2][b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) gS3[a][b] += W[0][a] * GW[0][b] + W[1][a] * GW[1][b] + W[2][a] * GW[2][b];
        // camera-space centre through J and through (u, v)
        float gx = du * cam.fx * iz, gy = dv * cam.fy * iz;
        float gz = -(du * cam.fx * cx + dv * cam.fy * cy) * iz * iz;
        gz += -(GJ[0][0] * cam.fx + GJ[1][1] * cam.fy) * iz * iz;
        // J02 = -fx tx / z, tx = x / z when not clamped
        gz += (GJ[0][2] * cam.fx * tx + GJ[1][2] * cam.fy * ty) * iz * iz;
        if (inx) { gx += -GJ[0][2] * cam.fx * iz * iz; gz += GJ[0][2] * cam.fx * cx * iz * iz * iz; }
        if (iny) { gy += -GJ[1][2] * cam.fy * iz * iz; gz += GJ[1][2] * cam.fy * cy * iz * iz * iz; }
        if (rec_dz) gz += rec_dz[r];
        for (int k = 0; k < 3; ++k) gmean[k] += W[0][k] * gx + W[1][k] * gy + W[2][k] * gz;
    }
    // S3 = M M^T: G_M = 2 G_S3 M ; M = R diag(s)
    float GM[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) GM[a][b] = 2.0f * (gS3[a][0] * Mm[0][b] + gS3[a][1] * Mm[1][b] + gS3[a][2] * Mm[2][b]);
    float GR[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) GR[a][b] = GM[a][b] * s[b];
    for (int k = 0; k < 3; ++k)
        d_log_scales[3 * i + k] = (GM[0][k] * Rm[0][k] + GM[1][k] * Rm[1][k] + GM[2][k] * Rm[2][k]) * s[k];
    // rotation entries as functions of the unit quaternion, grouped per component
    const float gw = 2.f * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
    const float gxq = 2.f * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2.f * x * GR[1][1] - w * GR[1][2] +
                             z * GR[2][0] + w * GR[2][1] - 2.f * x * GR[2][2]);
    const float gyq = 2.f * (-2.f * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] -
                             w * GR[2][0] + z * GR[2][1] - 2.f * y * GR[2][2]);
    const float gzq = 2.f * (-2.f * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - 2.f * z * GR[1][1] +
                             y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
    const float dot = gw * w + gxq * x + gyq * y + gzq * z;
    d_quats[4 * i + 0] = (gw - w * dot) * iq;
    d_quats[4 * i + 1] = (gxq - x * dot) * iq;
    d_quats[4 * i + 2] = (gyq - y * dot) * iq;
    d_quats[4 * i + 3] = (gzq - z * dot) * iq;
    for (int k = 0; k < 3; ++k) d_means[3 * i + k] = gmean[k];
    d_logits[i] = glogit;
}

// ------------------------------------------------------------- launchers

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------- scheduling

// The context's tile schedule: 0 one workgroup per tile, 1 persistent, 2
// persistent when several views are rendered.
static bool use_persistent(const lam_ctx* ctx, const CamSet& cs)
{
    const int mode = ctx->raster_schedule.load();
    return mode == 1 || (mode == 2 && cs.n > 1);
}

hipError_t render_forward_launch(lam_ctx* ctx, const RenderArgs& A, const RenderLayout& L, hipStream_t st)
{
    const CamSet& cs = L.cams;
    const uint32_t R = (uint32_t)L.records;
    const uint32_t cap = (uint32_t)L.capacity;
    // counters and every look-back scratch of the sorts start at zero (cleared
    // by the projection launch when there is one)
    hipError_t e = hipSuccess;
    const size_t zero_words = (size_t)(L.zero_end - L.counters);
    if (A.n > 0 && cs.n > 0) {
        ProfScope ps(ctx, "preprocess", st);
        hipLaunchKernelGGL(k_preprocess, dim3((A.n + 255) / 256, cs.n), dim3(256), 0, st, cs, A.n,
                           A.means, A.log_scales, A.quats, A.logits, L.rec0, L.rec1, L.foot,
                           L.depth_key, L.ntiles, L.counters, zero_words);
    } else {
        e = launch_fill_u32(L.counters, zero_words, 0u, st);
        if (e != hipSuccess) return e;
    }
    bool in_b = false;
    const uint32_t* tkeys;
    const uint32_t* trecs;
    {
        ProfScope ps(ctx, "render_sort", st);
        e = launch_radix_sort(L.depth_key, L.depth_a, L.recs_a, L.depth_b, L.recs_b, true, nullptr,
                              R, 32, L.sort_scratch, false, L.counters + 4, &in_b, st);
        if (e != hipSuccess) return e;
        const uint32_t* sorted_rec = in_b ? L.recs_b : L.recs_a;
        // pair offsets of the depth-ordered records; the last tile of the scan
        // writes the pairs needed and the overflow flag
        e = launch_excl_scan(L.ntiles, sorted_rec, R, L.offsets, L.counters, L.counters + 1, cap,
                             L.scan_scratch, false, L.counters + 4, st);
        if (e != hipSuccess) return e;
        if (R > 0 && cap > 0)
            hipLaunchKernelGGL(k_emit, dim3(std::min<uint32_t>((cap + 255) / 256, 8192u)), dim3(256),
                               0, st, cs, A.n, R, sorted_rec, (const uint32_t*)L.offsets,
                               (const uint2*)L.foot, (const uint32_t*)L.counters, cap, L.ikeys_a,
                               L.ivals_a);
        e = launch_radix_sort(nullptr, L.ikeys_a, L.ivals_a, L.ikeys_b, L.ivals_b, false,
                              L.counters, cap, L.tile_bits, L.tile_scratch, false, L.counters + 4, &in_b,
                              st);
        if (e != hipSuccess) return e;
        tkeys = in_b ? L.ikeys_b : L.ikeys_a;
        trecs = in_b ? L.ivals_b : L.ivals_a;
        if (cs.total_tiles > 0)
            hipLaunchKernelGGL(k_ranges, dim3(std::min<uint32_t>(cap / 256 + 1, 8192u)), dim3(256), 0, st,
                               tkeys, (const uint32_t*)L.counters, cap, (uint32_t)cs.total_tiles,
                               L.ranges);
    }
    if (cs.total_tiles > 0) {
        const bool pers = use_persistent(ctx, cs);
        const int threads = cs.tile_w * cs.tile_h;
        const bool rgbd = A.rgbd;
        auto kern = rgbd ? (A.d == 16 ? (pers ? k_raster_fwd<16, true, true> : k_raster_fwd<16, false, true>)
                                      : (pers ? k_raster_fwd<32, true, true> : k_raster_fwd<32, false, true>))
                         : (A.d == 16 ? (pers ? k_raster_fwd<16, true, false> : k_raster_fwd<16, false, false>)
                                      : (pers ? k_raster_fwd<32, true, false> : k_raster_fwd<32, false, false>));
        int grid = cs.total_tiles;
        if (pers)  // its work counter, counters[2], was cleared with the sort scratch
            grid = std::min(grid, ctx_resident_blocks(ctx, (const void*)kern, threads));
        ProfScope ps(ctx, "raster_fwd", st);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, cs, A.n, (const uint2*)L.ranges,
                           trecs, (const float4*)L.rec0, (const float4*)L.rec1, (const uint2*)L.foot,
                           A.queries, A.Q, A.T_final, L.t_final, L.n_contrib, L.counters + 2, A.colors,
                           (const uint32_t*)L.depth_key, A.rgb, A.depth);
    }
    return hipGetLastError();
}

hipError_t render_backward_launch(lam_ctx* ctx, const RenderArgs& A, const RenderLayout& L, hipStream_t st)
{
    const CamSet& cs = L.cams;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(L.rec_grad), (size_t)L.records * 6,
                                   0u, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(A.d_queries), (size_t)A.n * A.d, 0u, st);
    if (e != hipSuccess) return e;
    const bool rgbd = A.rgbd;
    if (rgbd) {
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(A.d_colors), (size_t)A.n * 3, 0u, st);
        if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(L.rec_dz), (size_t)L.records, 0u, st);
        if (e != hipSuccess) return e;
    }
    const uint32_t* trecs = L.tile_in_b ? L.ivals_b : L.ivals_a;
    if (cs.total_tiles > 0) {
        const bool pers = use_persistent(ctx, cs);
        const int threads = cs.tile_w * cs.tile_h;
        auto kern = rgbd ? (A.d == 16 ? (pers ? k_raster_bwd<16, true, true> : k_raster_bwd<16, false, true>)
                                      : (pers ? k_raster_bwd<32, true, true> : k_raster_bwd<32, false, true>))
                         : (A.d == 16 ? (pers ? k_raster_bwd<16, true, false> : k_raster_bwd<16, false, false>)
                                      : (pers ? k_raster_bwd<32, true, false> : k_raster_bwd<32, false, false>));
        int grid = cs.total_tiles;
        if (pers) {
            e = launch_fill_u32(L.counters + 3, 1, 0u, st);
            if (e != hipSuccess) return e;
            grid = std::min(grid, ctx_resident_blocks(ctx, (const void*)kern, threads));
        }
        ProfScope ps(ctx, "raster_bwd", st);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, cs, A.n, (const uint2*)L.ranges,
                           trecs, (const float4*)L.rec0, (const float4*)L.rec1, (const uint2*)L.foot,
                           A.queries, (const float*)L.t_final, (const uint32_t*)L.n_contrib, A.dQ,
                           L.rec_grad, A.d_queries, L.counters + 3, A.colors, (const uint32_t*)L.depth_key,
                           A.d_rgb, A.d_depth, A.d_colors, L.rec_dz);
    }
    if (A.n > 0) {
        ProfScope ps(ctx, "preprocess_bwd", st);
        hipLaunchKernelGGL(k_preprocess_bwd, dim3((A.n + 255) / 256), dim3(256), 0, st, cs, A.n,
                           A.means, A.log_scales, A.quats, A.logits, (const uint32_t*)L.ntiles,
                           (const float*)L.rec_grad, rgbd ? (const float*)L.rec_dz : nullptr, A.d_means,
                           A.d_log_scales, A.d_quats, A.d_logits);
    }
    return hipGetLastError();
}

}  // namespace lam
