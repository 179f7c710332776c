// The library context: creation, options, and the per-device caches the
// launches share.
#include <ctype.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "common.h"
#include "kernels.h"

// Scratch of lam_decode_forward_noalloc: the prepared dictionary (converted
// K and V, V transposed, K permuted, E4M3 scales).  One copy per GPU, held
// until the process ends; every call on a GPU shares its copy.  In host code
// this name is not a device address: launches use the address
// hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) unsigned char scratch[LAM_NOALLOC_SCRATCH_BYTES];

namespace lam {

void prof_release(lam_ctx* ctx);  // profile.hip

namespace {

// Device address of this GPU's ``scratch`` (resolved once per device, with
// that device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

// The options a context holds, as parsed and validated from JSON.
struct Options {
    int raster_schedule, decode_shape, decode_splits;
};

bool option_ok(const char* key, long v)
{
    if (!strcmp(key, "raster_schedule")) return v >= 0 && v <= 2;
    if (!strcmp(key, "decode_shape")) return v >= 0 && v <= 1;
    if (!strcmp(key, "decode_splits")) return v == 0 || (v >= 8 && v <= 4096 && v % 8 == 0);
    return false;
}

void set_option(Options* o, const char* key, int v)
{
    if (!strcmp(key, "raster_schedule")) o->raster_schedule = v;
    else if (!strcmp(key, "decode_shape")) o->decode_shape = v;
    else o->decode_splits = v;
}

// A flat JSON object of integer fields, e.g. {"decode_shape": 1}.  Unknown
// keys, non-integer values, nesting and values out of range are rejected; on
// rejection ``o`` is left as it was.
bool parse_options(const char* js, Options* o)
{
    if (!js) return true;
    Options t = *o;
    const char* p = js;
    auto ws = [&]() { while (*p && isspace((unsigned char)*p)) ++p; };
    ws();
    if (*p != '{') return false;
    ++p;
    ws();
    if (*p == '}') {
        ++p;
    } else {
        for (;;) {
            ws();
            if (*p != '"') return false;
            ++p;
            char key[32];
            size_t k = 0;
            while (*p && *p != '"') {
                if (k + 1 >= sizeof(key)) return false;
                key[k++] = *p++;
            }
            if (*p != '"') return false;
            key[k] = 0;
            ++p;
            ws();
            if (*p != ':') return false;
            ++p;
            ws();
            const char* q = p;
            if (*q == '-') ++q;
            if (!isdigit((unsigned char)*q)) return false;
            while (isdigit((unsigned char)*q)) ++q;
            if (q - p > 9) return false;
            const long v = strtol(p, nullptr, 10);
            p = q;
            if (!option_ok(key, v)) return false;
            set_option(&t, key, (int)v);
            ws();
            if (*p == ',') {
                ++p;
                continue;
            }
            if (*p != '}') return false;
            ++p;
            break;
        }
    }
    ws();
    if (*p) return false;
    *o = t;
    return true;
}

Options options_of(const lam_ctx* c)
{
    return Options{c->raster_schedule.load(), c->decode_shape.load(), c->decode_splits.load()};
}

void store_options(lam_ctx* c, const Options& o)
{
    c->raster_schedule.store(o.raster_schedule);
    c->decode_shape.store(o.decode_shape);
    c->decode_splits.store(o.decode_splits);
}

}  // namespace

const lam_ctx* ctx_options(const lam_ctx* ctx)
{
    static const lam_ctx defaults;
    return ctx ? ctx : &defaults;
}

bool ctx_ok(const lam_ctx* ctx)
{
    if (!ctx) return false;
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == ctx->device;
}

int ctx_resident_blocks(lam_ctx* ctx, const void* kernel, int threads)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const auto& e : ctx->occ)
        if (e.kernel == kernel && e.threads == threads) return e.blocks;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) per = 1;
    const int n = std::max(1, std::max(ctx->cus, 1) * std::max(per, 1));
    ctx->occ.push_back(lam_ctx::Occ{kernel, threads, n});
    return n;
}

hipError_t ctx_ensure_lds(lam_ctx* ctx, const void* kernel, size_t bytes)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto& e : ctx->lds) {
        if (e.kernel != kernel) continue;
        if (e.bytes >= bytes) return hipSuccess;
        const hipError_t r = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (r == hipSuccess) e.bytes = bytes;
        return r;
    }
    const hipError_t r = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r == hipSuccess) ctx->lds.push_back(lam_ctx::Lds{kernel, bytes});
    return r;
}

}  // namespace lam

using namespace lam;

extern "C" {

lam_status lam_create(int device, const char* options_json, lam_ctx** out)
{
    if (!out) return LAM_ERR_INVALID_ARG;
    *out = nullptr;
    Options o{2, 0, 0};
    if (!parse_options(options_json, &o)) return LAM_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return LAM_ERR_HIP;
    if (device < 0 || device >= count) return LAM_ERR_INVALID_ARG;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return LAM_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return LAM_ERR_HIP;
    lam_ctx* c = new (std::nothrow) lam_ctx();
    lam_status s = LAM_OK;
    if (!c) {
        s = LAM_ERR_INVALID_ARG;
    } else {
        c->device = device;
        store_options(c, o);
        if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
            hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
            scratch_address(device, &c->static_scratch) != hipSuccess)
            s = LAM_ERR_HIP;
        else
            c->static_scratch_bytes = LAM_NOALLOC_SCRATCH_BYTES;
    }
    if (s != LAM_OK && c) {
        if (c->fork) hipEventDestroy(c->fork);
        delete c;
        c = nullptr;
    }
    hipSetDevice(prev);
    *out = c;
    return s;
}

void lam_destroy(lam_ctx* ctx)
{
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        prof_release(ctx);
    }
    if (ctx->fork) hipEventDestroy(ctx->fork);
    delete ctx;
}

lam_status lam_ctx_configure(lam_ctx* ctx, const char* options_json)
{
    if (!ctx || !options_json) return LAM_ERR_INVALID_ARG;
    Options o = options_of(ctx);
    if (!parse_options(options_json, &o)) return LAM_ERR_INVALID_ARG;
    store_options(ctx, o);
    return LAM_OK;
}

lam_status lam_ctx_get(const lam_ctx* ctx, const char* key, int* value)
{
    if (!ctx || !key || !value) return LAM_ERR_INVALID_ARG;
    if (!strcmp(key, "device")) *value = ctx->device;
    else if (!strcmp(key, "raster_schedule")) *value = ctx->raster_schedule.load();
    else if (!strcmp(key, "decode_shape")) *value = ctx->decode_shape.load();
    else if (!strcmp(key, "decode_splits")) *value = ctx->decode_splits.load();
    else return LAM_ERR_INVALID_ARG;
    return LAM_OK;
}

}  // extern "C"
