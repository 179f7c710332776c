// Device-wide exclusive scan and stable LSD radix sort (u32 keys, u32 values)
// for gfx950.  Both operate on tiles of 4096 items per 256-thread workgroup.
//
// The radix sort ranks the 8-bit digits of a 64-item wave step with eight
// ballots (lanes sharing a digit form a mask), so equal digits keep their
// input order: wave w of a workgroup owns a contiguous 1024-item span, steps
// through it 64 items at a time, and keeps per-digit running counts in LDS.
// Workgroup-level and device-level digit offsets then come from a
// digit-major histogram scan, which is what makes every pass stable.
#include "common.h"
#include "kernels.h"

namespace lam {

constexpr int kTileThreads = 256;
constexpr int kTileItems = 16;
constexpr int kTile = kTileThreads * kTileItems;  // 4096

__device__ inline uint32_t load_count(const uint32_t* n_dev, uint32_t n_cap)
{
    if (!n_dev) return n_cap;
    uint32_t n = *n_dev;
    return n < n_cap ? n : n_cap;
}

// v from lane (lane - shift) in a DPP row pattern; lanes without a source read 0.
template <int CTRL, int ROW_MASK>
__device__ inline uint32_t dpp_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
}

// Inclusive wave scan (u32): Hillis-Steele steps inside each 16-lane row
// (row_shr 1, 2, 4, 8), then the row totals carried with row_bcast:15 into rows
// 1 and 3 and row_bcast:31 into rows 2 and 3.
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    v += dpp_u<0x111, 0xF>(v);  // row_shr:1
    v += dpp_u<0x112, 0xF>(v);  // row_shr:2
    v += dpp_u<0x114, 0xF>(v);  // row_shr:4
    v += dpp_u<0x118, 0xF>(v);  // row_shr:8
    v += dpp_u<0x142, 0xA>(v);  // row_bcast:15
    v += dpp_u<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// Exclusive scan of one value per thread across a 256-thread block; returns
// the block total through *total.  ``sh`` holds 4 words.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total, uint32_t* sh)
{
    unsigned lane = __lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) sh[w] = inc;
    __syncthreads();
    uint32_t wo = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kTileThreads / kWave; ++k) {
        uint32_t s = sh[k];
        if (k < (int)w) wo += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wo + inc - v;
}

// Loads the scan inputs i0 + k * stride (k < kTileItems), zero past n; with
// idx the input is in[idx[i]].  Every load is issued (indices clamped into
// range, n >= 1) before any is used, so the 16 (or 2 x 16) loads are in flight
// together instead of one round trip each.
__device__ inline void load_scan_values(const uint32_t* in, const uint32_t* idx, uint32_t i0,
                                        uint32_t stride, uint32_t n, uint32_t* v)
{
    uint32_t j[kTileItems];
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const uint32_t i = i0 + k * stride;
        j[k] = i < n ? i : n - 1;
    }
    if (idx) {
#pragma unroll
        for (int k = 0; k < kTileItems; ++k) j[k] = idx[j[k]];
    }
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) v[k] = in[j[k]];
#pragma unroll
    for (int k = 0; k < kTileItems; ++k)
        if (i0 + k * stride >= n) v[k] = 0u;
}

// Exclusive scan of the 1024 values of a wave stripe held as v[k] = value
// k * 64 + lane (coalesced loads): 16 chained wave scans.  Returns the stripe
// total; ex[k] receives the exclusive prefix of value k * 64 + lane.
constexpr uint32_t kStripe = kWave * kTileItems;  // 1024 values per wave stripe

__device__ inline uint32_t stripe_excl_scan(const uint32_t* v, uint32_t* ex)
{
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const uint32_t inc = wave_incl_scan(v[k]);
        ex[k] = run + inc - v[k];
        run += (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
    }
    return run;
}

__global__ __launch_bounds__(kTileThreads) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                              const uint32_t* __restrict__ idx,
                                                              uint32_t n, uint32_t* block_sums)
{
    __shared__ uint32_t sh[4];
    uint32_t v[kTileItems], s = 0;
    load_scan_values(in, idx, blockIdx.x * (uint32_t)kTile + threadIdx.x, kTileThreads, n, v);
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) s += v[k];
    uint32_t tot;
    block_excl_scan(s, &tot, sh);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of the block sums in place; the grand total
// goes to *total (may be NULL).
__global__ __launch_bounds__(kTileThreads) void k_scan_top(uint32_t* sums, uint32_t nb, uint32_t* total)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kTile) {
        uint32_t v[kTileItems], s = 0;
        load_scan_values(sums, nullptr, base + threadIdx.x * kTileItems, 1, nb, v);
#pragma unroll
        for (int k = 0; k < kTileItems; ++k) s += v[k];
        uint32_t tot;
        uint32_t off = block_excl_scan(s, &tot, sh) + carry;
        for (int k = 0; k < kTileItems; ++k) {
            uint32_t i = base + threadIdx.x * kTileItems + k;
            if (i < nb) sums[i] = off;
            off += v[k];
        }
        carry += tot;
    }
    if (total && threadIdx.x == 0) *total = carry;
}

// Block b's 4096 values as four wave stripes (coalesced), offset by the block's
// scanned sum and the stripes before it.
__global__ __launch_bounds__(kTileThreads) void k_scan_down(const uint32_t* __restrict__ in,
                                                            const uint32_t* __restrict__ idx,
                                                            uint32_t n,
                                                            const uint32_t* __restrict__ block_off,
                                                            uint32_t* __restrict__ out)
{
    __shared__ uint32_t sh[kTileThreads / kWave];
    const unsigned lane = __lane_id(), w = threadIdx.x / kWave;
    const uint32_t sbase = blockIdx.x * (uint32_t)kTile + w * kStripe;
    uint32_t v[kTileItems], ex[kTileItems];
    load_scan_values(in, idx, sbase + lane, kWave, n, v);
    const uint32_t st = stripe_excl_scan(v, ex);
    if (lane == 0) sh[w] = st;
    __syncthreads();
    uint32_t off = block_off[blockIdx.x];
    for (int k = 0; k < (int)w; ++k) off += sh[k];
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const uint32_t i = sbase + k * kWave + lane;
        if (i < n) out[i] = off + ex[k];
    }
}

// One 1024-thread workgroup scans up to kSingleMax values in tiles of 16384:
// wave w takes the stripe of 1024 values at w * 1024 with coalesced loads (all
// 16 in flight), scans it, and the 16 stripe totals are combined in LDS; a
// carry links the tiles.  One launch instead of three for small inputs.
constexpr int kSingleThreads = 1024;
constexpr uint32_t kSingleTile = kSingleThreads * kTileItems;
constexpr uint32_t kSingleMax = 4 * kSingleTile;

__global__ __launch_bounds__(kSingleThreads) void k_scan_single(const uint32_t* __restrict__ in,
                                                                const uint32_t* __restrict__ idx,
                                                                uint32_t n, uint32_t* __restrict__ out,
                                                                uint32_t* __restrict__ total)
{
    __shared__ uint32_t sh[kSingleThreads / kWave];
    const unsigned lane = __lane_id(), w = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n; base += kSingleTile) {
        const uint32_t sbase = base + w * kStripe;
        uint32_t v[kTileItems], ex[kTileItems];
        load_scan_values(in, idx, sbase + lane, kWave, n, v);
        const uint32_t st = stripe_excl_scan(v, ex);
        if (lane == 0) sh[w] = st;
        __syncthreads();
        uint32_t wo = 0, tot = 0;
        for (int k = 0; k < kSingleThreads / kWave; ++k) {
            const uint32_t x = sh[k];
            if (k < (int)w) wo += x;
            tot += x;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kTileItems; ++k) {
            const uint32_t i = sbase + k * kWave + lane;
            if (i < n) out[i] = carry + wo + ex[k];
        }
        carry += tot;
    }
    if (total && threadIdx.x == 0) *total = carry;
}

size_t scan_scratch_words(uint32_t n) { return (n + kTile - 1) / kTile + 1; }

hipError_t launch_excl_scan(const uint32_t* in, const uint32_t* idx, uint32_t n, uint32_t* out,
                            uint32_t* total, uint32_t* scratch, hipStream_t st)
{
    uint32_t nb = (n + kTile - 1) / kTile;
    if (n <= kSingleMax) {
        // includes n == 0, where only the total (zero) is written
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kSingleThreads), 0, st, in, idx, n, out, total);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kTileThreads), 0, st, in, idx, n, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTileThreads), 0, st, scratch, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kTileThreads), 0, st, in, idx, n,
                       (const uint32_t*)scratch, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix

template <int DB, int ITEMS>
__global__ __launch_bounds__(kTileThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_dev,
                                                             uint32_t n_cap, int shift,
                                                             uint32_t* __restrict__ hist,
                                                             uint32_t nblocks)
{
    constexpr int BINS = 1 << DB;
    __shared__ uint32_t h[BINS];
    for (int k = threadIdx.x; k < BINS; k += kTileThreads) h[k] = 0;
    __syncthreads();
    const uint32_t n = load_count(n_dev, n_cap);
    const uint32_t base = blockIdx.x * (uint32_t)(kTileThreads * ITEMS);
    if (base < n) {  // keys loaded together (clamped), then counted
        uint32_t key[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t i = base + k * kTileThreads + threadIdx.x;
            key[k] = keys[i < n ? i : n - 1];
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            if (base + k * kTileThreads + threadIdx.x < n) atomicAdd(&h[(key[k] >> shift) & (BINS - 1u)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < BINS; k += kTileThreads) hist[(size_t)k * nblocks + blockIdx.x] = h[k];
}

// Stable scatter of one pass.  The keys of a tile are ranked per digit (wave
// ballots, then a prefix over the waves), placed in LDS in their sorted order
// inside the tile, and written out from there: consecutive threads then store
// consecutive elements of each digit's run, so the global writes are whole
// runs instead of one scattered element per key.
template <int DB, int ITEMS>
__global__ __launch_bounds__(kTileThreads) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ n_dev, uint32_t n_cap, int shift,
    const uint32_t* __restrict__ offsets, uint32_t nblocks)
{
    constexpr int BINS = 1 << DB;
    constexpr int WAVES = kTileThreads / kWave;
    constexpr int TILE = kTileThreads * ITEMS;
    constexpr int DPT = BINS / kTileThreads;  // digits per thread in the digit scan
    static_assert(BINS % kTileThreads == 0, "whole digits per thread");
    // the per-wave digit counts, later (same words) the tile's keys and values
    // in sorted order
    constexpr int UWORDS = WAVES * BINS > 2 * TILE ? WAVES * BINS : 2 * TILE;
    __shared__ uint32_t ubuf[UWORDS];
    __shared__ uint32_t gbase[BINS];
    __shared__ uint32_t dstart[BINS];  // first local position of each digit
    __shared__ uint32_t ssh[4];
    uint32_t(*cnt)[BINS] = reinterpret_cast<uint32_t(*)[BINS]>(ubuf);
    uint32_t* lk = ubuf;
    uint32_t* lv = ubuf + TILE;
    const unsigned lane = __lane_id(), w = threadIdx.x / kWave;
    for (int k = threadIdx.x; k < WAVES * BINS; k += kTileThreads) ubuf[k] = 0;
    for (int k = threadIdx.x; k < BINS; k += kTileThreads)
        gbase[k] = offsets[(size_t)k * nblocks + blockIdx.x];
    __syncthreads();

    const uint32_t n = load_count(n_dev, n_cap);
    const uint32_t span = blockIdx.x * (uint32_t)TILE + w * (kWave * ITEMS);
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
    // all keys and values of the wave's span are requested before the ranking
    // (indices clamped into range; entries past n are never placed)
    const uint32_t nl = n > 0 ? n - 1 : 0;
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const uint32_t i = span + s * kWave + lane;
        key[s] = keys_in[i < n ? i : nl];
    }
    if (vals_in) {
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) {
            const uint32_t i = span + s * kWave + lane;
            val[s] = vals_in[i < n ? i : nl];
        }
    } else {
#pragma unroll
        for (int s = 0; s < ITEMS; ++s) val[s] = span + s * kWave + lane;
    }
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        const uint32_t i = span + s * kWave + lane;
        const bool ok = i < n;
        const uint32_t dg = (key[s] >> shift) & (BINS - 1u);
        // lanes holding the same digit: intersect the ballots of its bits
        unsigned long long peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const unsigned long long m = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? m : ~m;
        }
        const uint32_t before = ok ? cnt[w][dg] : 0u;
        rank[s] = ok ? before + (uint32_t)__popcll(peers & lt) : 0xFFFFFFFFu;
        // the lowest lane of each digit group publishes the new running count
        if (ok && (peers & lt) == 0ull) cnt[w][dg] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // exclusive prefix over the waves per digit, and the tile's digit totals
    // scanned over the digits (thread t owns digits DPT t .. DPT t + DPT - 1)
    uint32_t tot[DPT], tsum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int d = threadIdx.x * DPT + j;
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) {
            const uint32_t c = cnt[k][d];
            cnt[k][d] = run;
            run += c;
        }
        tot[j] = run;
        tsum += run;
    }
    uint32_t nvalid;
    uint32_t off = block_excl_scan(tsum, &nvalid, ssh);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        dstart[threadIdx.x * DPT + j] = off;
        off += tot[j];
    }
    __syncthreads();
    // local positions first (they read the counts), then the counts' words
    // take the sorted keys and values
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        if (rank[s] == 0xFFFFFFFFu) continue;
        const uint32_t dg = (key[s] >> shift) & (BINS - 1u);
        rank[s] = dstart[dg] + cnt[w][dg] + rank[s];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        if (rank[s] == 0xFFFFFFFFu) continue;
        lk[rank[s]] = key[s];
        lv[rank[s]] = val[s];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nvalid; i += kTileThreads) {
        const uint32_t k = lk[i];
        const uint32_t dg = (k >> shift) & (BINS - 1u);
        const uint32_t pos = gbase[dg] + (i - dstart[dg]);
        if (pos < n) {  // always true for a consistent histogram; keeps a bad one in bounds
            keys_out[pos] = k;
            vals_out[pos] = lv[i];
        }
    }
}

// Plan of a sort of ``bits`` key bits over at most n_cap keys.  Wide keys over
// a modest count (the depth keys of up to 2^20 records) take 8-bit digits over
// tiles of 1024 keys: four times the workgroups of 4096-key tiles and a
// histogram (bins x tiles) eight times smaller to scan, for one pass more.
// Otherwise at most 11 bits per pass over 4096-key tiles.
struct RadixPlan {
    int passes, width, items;
};

static RadixPlan radix_plan(int bits, uint32_t n_cap)
{
    if (bits < 1) bits = 1;
    if (bits > 16 && n_cap <= (1u << 20)) return RadixPlan{(bits + 7) / 8, 8, 4};
    const int p = (bits + 10) / 11;
    const int wdt = (bits + p - 1) / p;
    return RadixPlan{p, wdt <= 8 ? 8 : 11, kTileItems};
}

size_t radix_scratch_words(uint32_t n_cap)
{
    // the larger histogram of the two plans
    const uint32_t nb4k = std::max((n_cap + kTile - 1) / kTile, 1u);
    const uint32_t nb1k = std::max((n_cap + kTileThreads * 4 - 1) / (kTileThreads * 4), 1u);
    const size_t h = std::max((size_t)2048 * nb4k, (size_t)256 * nb1k);
    return h + scan_scratch_words((uint32_t)h) + 8;
}

// Sorts the ``bits`` low bits of the keys, ping-ponging between the A and B
// buffers; *in_b tells where the result ended.  keys_first, when given, is the
// read-only input of the first pass (it is left intact).  With iota_first the
// first pass takes value = input position instead of vals_a.
hipError_t launch_radix_sort(const uint32_t* keys_first, uint32_t* keys_a, uint32_t* vals_a,
                             uint32_t* keys_b, uint32_t* vals_b, bool iota_first,
                             const uint32_t* n_dev, uint32_t n_cap, int bits, uint32_t* scratch,
                             bool* in_b, hipStream_t st)
{
    const RadixPlan plan = radix_plan(bits, n_cap);
    const uint32_t tile = (uint32_t)(kTileThreads * plan.items);
    const uint32_t nb = (n_cap + tile - 1) / tile;
    *in_b = false;
    if (nb == 0) return hipSuccess;
    const int width = plan.width;
    const uint32_t bins = 1u << width;
    uint32_t* hist = scratch;
    uint32_t* sscr = scratch + (size_t)bins * nb;
    uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
    for (int p = 0; p < plan.passes; ++p) {
        const int shift = width * p;
        const uint32_t* kin = (p == 0 && keys_first) ? keys_first : ki;
        const uint32_t* vin = (p == 0 && iota_first) ? (const uint32_t*)nullptr : vi;
        if (plan.items == 4)
            hipLaunchKernelGGL((k_radix_hist<8, 4>), dim3(nb), dim3(kTileThreads), 0, st, kin, n_dev, n_cap,
                               shift, hist, nb);
        else if (width == 8)
            hipLaunchKernelGGL((k_radix_hist<8, kTileItems>), dim3(nb), dim3(kTileThreads), 0, st, kin, n_dev,
                               n_cap, shift, hist, nb);
        else
            hipLaunchKernelGGL((k_radix_hist<11, kTileItems>), dim3(nb), dim3(kTileThreads), 0, st, kin, n_dev,
                               n_cap, shift, hist, nb);
        hipError_t e = launch_excl_scan(hist, nullptr, bins * nb, hist, nullptr, sscr, st);
        if (e != hipSuccess) return e;
        if (plan.items == 4)
            hipLaunchKernelGGL((k_radix_scatter<8, 4>), dim3(nb), dim3(kTileThreads), 0, st, kin, vin, ko, vo,
                               n_dev, n_cap, shift, hist, nb);
        else if (width == 8)
            hipLaunchKernelGGL((k_radix_scatter<8, kTileItems>), dim3(nb), dim3(kTileThreads), 0, st, kin, vin,
                               ko, vo, n_dev, n_cap, shift, hist, nb);
        else
            hipLaunchKernelGGL((k_radix_scatter<11, kTileItems>), dim3(nb), dim3(kTileThreads), 0, st, kin, vin,
                               ko, vo, n_dev, n_cap, shift, hist, nb);
        uint32_t* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        *in_b = !*in_b;
    }
    return hipGetLastError();
}

int radix_passes(int bits, uint32_t n_cap) { return radix_plan(bits, n_cap).passes; }

}  // namespace lam
