// Device-wide exclusive scan and stable LSD radix sort (u32 keys, u32 values)
// for gfx950, both single-sweep: each pass over the data is one launch.
//
// The radix sort reads the keys once to count the digits of every pass
// (k_radix_hist), then makes one launch per pass (k_radix_pass).  A pass
// ranks the digits of a 64-item wave step with one ballot per digit bit
// (lanes sharing a digit form a mask), so equal digits keep their input
// order: wave w of a workgroup owns a contiguous span, steps through it 64
// items at a time, and keeps per-digit running counts in LDS.  The tile's
// offset among the tiles before it comes from a decoupled look-back over
// per-tile digit counts, and the digit's offset in the output from the
// counts of the first launch, which is what keeps every pass stable without
// a separate scan launch.  The scan uses the same look-back over tile sums.
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

// ----------------------------------------------------------- look-back

// Decoupled look-back.  Workgroup t takes tile t; workgroups are dispatched
// in index order, so every tile below a running one has been started, and a
// tile's own count never waits on anything.  A workgroup publishes its
// tile's count with flag 1 as soon as it has it, walks back over the tiles
// before it adding their counts until it meets one published with flag 2
// (the count of that tile and all before it), and then publishes its own
// inclusive count with flag 2.  (Drawing tile indices from an atomic counter
// instead, which needs no dispatch order, serialised the workgroups on that
// one word: about 35 ns each.)  The status words must be zero when the
// launch starts.
//
// Radix status words are 32 bits: the flag in the top two, the count (below
// 2^30, the largest sort supported) in the rest.  Scan status words are 64
// bits: the flag in the high word, the 32-bit sum in the low one.
constexpr uint32_t kFlagShift = 30;
constexpr uint32_t kCountMask = (1u << kFlagShift) - 1u;
constexpr uint32_t kFlagAgg = 1u << kFlagShift;
constexpr uint32_t kFlagInc = 2u << kFlagShift;
constexpr uint32_t kMaxSortCount = 1u << kFlagShift;
// Polls of a status word that is still zero before the walk gives up and
// raises the error word: with a 64-clock sleep between polls about 0.1 s,
// far beyond any tile's time to publish (a bound, not an expected path).
constexpr uint32_t kSpinLimit = 1u << 22;

template <typename T, typename V>
__device__ inline void status_put(T* p, V v)
{
    __hip_atomic_store(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline T status_get(T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tiles a walk reads per poll: one round trip to a coherent level of memory
// (about a microsecond across the XCDs) then covers up to this many tiles.
constexpr int kLookAhead = 16;

// Exclusive prefix over tiles 0 .. t-1 of the count at status[j * stride + c]:
// each poll requests the next kLookAhead tiles down at once and consumes them
// from the nearest until one is not published yet (polled again next round)
// or one carries flag 2 (the walk ends).
__device__ inline uint32_t look_back(uint32_t* status, uint32_t stride, uint32_t t, uint32_t c, uint32_t* err)
{
    uint32_t excl = 0, spins = 0;
    int j = (int)t - 1;  // the nearest tile not consumed yet
    while (j >= 0) {
        uint32_t s[kLookAhead];
#pragma unroll
        for (int k = 0; k < kLookAhead; ++k)
            s[k] = j - k >= 0 ? status_get(status + (size_t)(j - k) * stride + c) : kFlagInc;
        bool stop = false, done = false;
#pragma unroll
        for (int k = 0; k < kLookAhead; ++k) {
            const uint32_t f = s[k] >> kFlagShift;
            if (stop || f == 0u) {
                stop = true;
                continue;
            }
            excl += s[k] & kCountMask;
            --j;
            if (f == 2u) stop = done = true;
        }
        if (done) break;
        if (j >= 0 && (s[0] >> kFlagShift) == 0u) {  // nothing consumed: wait before the next poll
            if (++spins > kSpinLimit) {
                atomicOr(err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// The same walk over 64-bit scan status words (one per tile).
__device__ inline uint32_t look_back_sum(uint64_t* status, uint32_t t, uint32_t* err)
{
    uint32_t excl = 0, spins = 0;
    int j = (int)t - 1;
    while (j >= 0) {
        uint64_t s[kLookAhead];
#pragma unroll
        for (int k = 0; k < kLookAhead; ++k) s[k] = j - k >= 0 ? status_get(status + (j - k)) : (2ull << 32);
        bool stop = false, done = false;
#pragma unroll
        for (int k = 0; k < kLookAhead; ++k) {
            const uint32_t f = (uint32_t)(s[k] >> 32);
            if (stop || f == 0u) {
                stop = true;
                continue;
            }
            excl += (uint32_t)s[k];
            --j;
            if (f == 2u) stop = done = true;
        }
        if (done) break;
        if (j >= 0 && (uint32_t)(s[0] >> 32) == 0u) {
            if (++spins > kSpinLimit) {
                atomicOr(err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// ---------------------------------------------------------------- scan

// Scan scratch: word 1 the error word, then one 64-bit status word per tile
// of kTile values from word 2.
size_t scan_scratch_words(uint32_t n) { return 2 + 2 * (size_t)((n + kTile - 1) / kTile); }

// Exclusive scan of in[idx[i]] (in[i] when idx is null) over i < n into out,
// one tile of 4096 values per workgroup as four coalesced wave stripes; the
// workgroup of the last tile writes the grand total to *total and, when over
// is given, (total > cap) to *over.
__global__ __launch_bounds__(kTileThreads) void k_scan_lookback(
    const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx, uint32_t n,
    uint32_t* __restrict__ out, uint32_t* total, uint32_t* over, uint32_t cap, uint32_t* scratch,
    uint32_t* err)
{
    __shared__ uint32_t sh[kTileThreads / kWave];
    __shared__ uint32_t carry_sh;
    const uint32_t t = blockIdx.x;
    const uint32_t base = t * (uint32_t)kTile;
    if (base >= n) return;  // the whole workgroup: a tile past the data
    const unsigned lane = __lane_id(), w = threadIdx.x / kWave;
    const uint32_t sbase = base + w * kStripe;
    uint32_t v[kTileItems], ex[kTileItems];
    load_scan_values(in, idx, sbase + lane, kWave, n, v);
    const uint32_t st = stripe_excl_scan(v, ex);
    if (lane == 0) sh[w] = st;
    __syncthreads();
    uint32_t wo = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kTileThreads / kWave; ++k) {
        const uint32_t x = sh[k];
        if (k < (int)w) wo += x;
        tot += x;
    }
    if (threadIdx.x == 0) {
        uint64_t* status = reinterpret_cast<uint64_t*>(scratch + 2);
        uint32_t excl = 0;
        if (t == 0) {
            status_put(status, (2ull << 32) | tot);
        } else {
            status_put(status + t, (1ull << 32) | tot);
            excl = look_back_sum(status, t, err);
            status_put(status + t, (2ull << 32) | (uint32_t)(excl + tot));
        }
        carry_sh = excl;
        if (base + (uint32_t)kTile >= n) {
            *total = excl + tot;
            if (over) *over = excl + tot > cap ? 1u : 0u;
        }
    }
    __syncthreads();
    const uint32_t off = carry_sh + wo;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const uint32_t i = sbase + k * kWave + lane;
        if (i < n) out[i] = off + ex[k];
    }
}

__global__ void k_scan_empty(uint32_t* total, uint32_t* over)
{
    if (total) *total = 0u;
    if (over) *over = 0u;
}

hipError_t launch_excl_scan(const uint32_t* in, const uint32_t* idx, uint32_t n, uint32_t* out,
                            uint32_t* total, uint32_t* over, uint32_t cap, uint32_t* scratch,
                            bool zero_scratch, uint32_t* err, hipStream_t st)
{
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_empty, dim3(1), dim3(1), 0, st, total, over);
        return hipGetLastError();
    }
    if (zero_scratch) {
        hipError_t e = launch_fill_u32(scratch, scan_scratch_words(n), 0u, st);
        if (e != hipSuccess) return e;
    }
    const uint32_t nt = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_scan_lookback, dim3(nt), dim3(kTileThreads), 0, st, in, idx, n, out, total,
                       over, cap, scratch, err ? err : scratch + 1);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix

// Digit counts of every pass from one read of the keys: ghist[p * BINS + d]
// gains the number of keys i < n whose digit p (bits p * width .. p * width +
// width - 1) is d.  Workgroups stride over the key tiles, count in LDS and add
// each non-zero bin with one atomic.
template <int DB>
__global__ __launch_bounds__(kTileThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_dev,
                                                             uint32_t n_cap, int passes, int width,
                                                             uint32_t* __restrict__ ghist)
{
    constexpr int BINS = 1 << DB;
    constexpr int MAXP = (32 + DB - 1) / DB;
    __shared__ uint32_t h[MAXP * BINS];
    const int nbins = passes * BINS;
    for (int k = threadIdx.x; k < nbins; k += kTileThreads) h[k] = 0;
    __syncthreads();
    const uint32_t n = load_count(n_dev, n_cap);
    const uint32_t mask = (1u << width) - 1u;
    for (uint32_t base = blockIdx.x * (uint32_t)kTile; base < n; base += gridDim.x * (uint32_t)kTile) {
        uint32_t key[kTileItems];
#pragma unroll
        for (int k = 0; k < kTileItems; ++k) {
            const uint32_t i = base + k * kTileThreads + threadIdx.x;
            key[k] = keys[i < n ? i : n - 1];
        }
#pragma unroll
        for (int k = 0; k < kTileItems; ++k) {
            if (base + k * kTileThreads + threadIdx.x >= n) continue;
            for (int p = 0; p < passes; ++p) atomicAdd(&h[p * BINS + ((key[k] >> (p * width)) & mask)], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nbins; k += kTileThreads)
        if (h[k]) atomicAdd(&ghist[k], h[k]);
}

// One stable pass over the digit at bits shift .. shift + width - 1.  The
// keys of the workgroup's tile are ranked per digit (wave ballots, then a
// prefix over the waves), the tile's digit counts are published and its
// offsets among the earlier tiles read back by look-back, and the keys and
// values are placed in LDS in their sorted order inside the tile and written
// out from there: consecutive threads store consecutive elements of each
// digit's run, so the global writes are whole runs.
template <int DB, int ITEMS>
__global__ __launch_bounds__(kTileThreads) void k_radix_pass(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ n_dev, uint32_t n_cap, int shift, int width,
    const uint32_t* __restrict__ ghist, uint32_t* status, uint32_t* err)
{
    constexpr int BINS = 1 << DB;
    constexpr int WAVES = kTileThreads / kWave;
    constexpr int TILE = kTileThreads * ITEMS;
    static_assert(BINS == kTileThreads, "one digit per thread");
    // the per-wave digit counts, later (same words) the tile's keys and values
    // in sorted order
    constexpr int UWORDS = WAVES * BINS > 2 * TILE ? WAVES * BINS : 2 * TILE;
    __shared__ uint32_t ubuf[UWORDS];
    __shared__ uint32_t gbase[BINS];   // output position of the tile's first key of each digit
    __shared__ uint32_t dstart[BINS];  // first local position of each digit
    __shared__ uint32_t ssh[4];
    uint32_t(*cnt)[BINS] = reinterpret_cast<uint32_t(*)[BINS]>(ubuf);
    uint32_t* lk = ubuf;
    uint32_t* lv = ubuf + TILE;
    const unsigned lane = __lane_id(), w = threadIdx.x / kWave;
    for (int k = threadIdx.x; k < WAVES * BINS; k += kTileThreads) ubuf[k] = 0;
    __syncthreads();
    const uint32_t t = blockIdx.x;
    const uint32_t n = load_count(n_dev, n_cap);
    if (t * (uint32_t)TILE >= n) return;  // the whole workgroup: a tile past the data

    const uint32_t mask = (1u << width) - 1u;
    const uint32_t span = t * (uint32_t)TILE + w * (kWave * ITEMS);
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
    // all keys and values of the wave's span are requested before the ranking
    // (indices clamped into range; entries past n are never placed)
    const uint32_t nl = n - 1;
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
        const uint32_t dg = (key[s] >> shift) & mask;
        // lanes holding the same digit: intersect the ballots of its bits
        unsigned long long peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            if (b >= width) break;
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
    // (thread q owns digit q)
    const uint32_t d0 = threadIdx.x;
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
        const uint32_t c = cnt[k][d0];
        cnt[k][d0] = tot;
        tot += c;
    }
    // the tile's counts go out first, then the walk over the tiles before it
    uint32_t* my = status + (size_t)t * BINS + d0;
    uint32_t excl = 0;
    if (t == 0) {
        status_put(my, kFlagInc | tot);
    } else {
        status_put(my, kFlagAgg | tot);
        excl = look_back(status, BINS, t, d0, err);
        status_put(my, kFlagInc | ((excl + tot) & kCountMask));
    }
    // output position of each digit's first key in this tile: the keys of all
    // smaller digits (digit counts scanned over the digits) plus this digit's
    // keys in the tiles before
    const uint32_t gv = ghist[d0];
    uint32_t gtot;
    gbase[d0] = block_excl_scan(gv, &gtot, ssh) + excl;
    uint32_t nvalid;
    dstart[d0] = block_excl_scan(tot, &nvalid, ssh);
    __syncthreads();
    // local positions first (they read the counts), then the counts' words
    // take the sorted keys and values
#pragma unroll
    for (int s = 0; s < ITEMS; ++s) {
        if (rank[s] == 0xFFFFFFFFu) continue;
        const uint32_t dg = (key[s] >> shift) & mask;
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
        const uint32_t dg = (k >> shift) & mask;
        const uint32_t pos = gbase[dg] + (i - dstart[dg]);
        if (pos < n) {  // always true for consistent counts; keeps bad ones in bounds
            keys_out[pos] = k;
            vals_out[pos] = lv[i];
        }
    }
}

// Plan of a sort of ``bits`` key bits over at most n_cap keys: 8-bit digits
// (fewer bits when that splits them evenly over the same number of passes)
// over tiles of 4096 keys, or of 1024 keys for wide keys over at most 2^20
// keys (the depth keys of a modest scene: four times the workgroups where
// the key count alone would leave most CUs idle).
struct RadixPlan {
    int passes, width, items;
    uint32_t tiles;
};

constexpr int kDigitBits = 8;
constexpr uint32_t kBins = 1u << kDigitBits;

static RadixPlan radix_plan(int bits, uint32_t n_cap)
{
    bits = bits < 1 ? 1 : (bits > 32 ? 32 : bits);
    RadixPlan r;
    r.passes = (bits + kDigitBits - 1) / kDigitBits;
    r.width = (bits + r.passes - 1) / r.passes;
    r.items = bits > 16 && n_cap <= (1u << 20) ? 4 : kTileItems;
    const uint32_t tile = (uint32_t)(kTileThreads * r.items);
    r.tiles = (uint32_t)(((uint64_t)n_cap + tile - 1) / tile);
    return r;
}

// Radix scratch: word 4 the error word, then from word 8 the digit counts
// (passes x bins) and the tile status words (passes x tiles x bins).
constexpr size_t kRadixHead = 8;

size_t radix_scratch_words(int bits, uint32_t n_cap)
{
    const RadixPlan p = radix_plan(bits, n_cap);
    return kRadixHead + p.passes * (size_t)kBins + (size_t)p.passes * p.tiles * kBins;
}

// Sorts the ``bits`` low bits of the keys, ping-ponging between the A and B
// buffers; *in_b tells where the result ended.  keys_first, when given, is the
// read-only input of the first pass (it is left intact).  With iota_first the
// first pass takes value = input position instead of vals_a.
hipError_t launch_radix_sort(const uint32_t* keys_first, uint32_t* keys_a, uint32_t* vals_a,
                             uint32_t* keys_b, uint32_t* vals_b, bool iota_first,
                             const uint32_t* n_dev, uint32_t n_cap, int bits, uint32_t* scratch,
                             bool zero_scratch, uint32_t* err, bool* in_b, hipStream_t st)
{
    *in_b = false;
    if (n_cap == 0) return hipSuccess;
    if (n_cap >= kMaxSortCount) return hipErrorInvalidValue;
    const RadixPlan plan = radix_plan(bits, n_cap);
    if (zero_scratch) {
        hipError_t e = launch_fill_u32(scratch, radix_scratch_words(bits, n_cap), 0u, st);
        if (e != hipSuccess) return e;
    }
    if (!err) err = scratch + 4;
    uint32_t* gh = scratch + kRadixHead;
    uint32_t* status = gh + (size_t)plan.passes * kBins;
    // one workgroup per 4096 keys for the counts (at most 512, striding
    // beyond): the LDS atomics of keys sharing a digit serialise within a
    // workgroup, so the keys are spread wide; each workgroup then adds its
    // non-zero bins with one atomic each
    const uint32_t hgrid = std::min<uint32_t>((n_cap + kTile - 1) / kTile, 512u);
    hipLaunchKernelGGL((k_radix_hist<kDigitBits>), dim3(hgrid), dim3(kTileThreads), 0, st,
                       keys_first ? keys_first : keys_a, n_dev, n_cap, plan.passes, plan.width, gh);
    uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
    for (int p = 0; p < plan.passes; ++p) {
        const uint32_t* kin = (p == 0 && keys_first) ? keys_first : ki;
        const uint32_t* vin = (p == 0 && iota_first) ? (const uint32_t*)nullptr : vi;
        const uint32_t* ghp = gh + (size_t)p * kBins;
        uint32_t* stp = status + (size_t)p * plan.tiles * kBins;
        const int shift = plan.width * p;
        if (plan.items == 4)
            hipLaunchKernelGGL((k_radix_pass<kDigitBits, 4>), dim3(plan.tiles), dim3(kTileThreads), 0, st,
                               kin, vin, ko, vo, n_dev, n_cap, shift, plan.width, ghp, stp, err);
        else
            hipLaunchKernelGGL((k_radix_pass<kDigitBits, kTileItems>), dim3(plan.tiles), dim3(kTileThreads),
                               0, st, kin, vin, ko, vo, n_dev, n_cap, shift, plan.width, ghp, stp, err);
        uint32_t* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        *in_b = !*in_b;
    }
    return hipGetLastError();
}

int radix_passes(int bits, uint32_t n_cap) { return radix_plan(bits, n_cap).passes; }

}  // namespace lam
