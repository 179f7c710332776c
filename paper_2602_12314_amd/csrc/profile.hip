// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; when a context has it on, every instrumented launch made
// through that context is bracketed by two events and lam_profile_read sums
// their elapsed times per kernel name.
#include <string.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace lam {

namespace {
hipEvent_t take_event(ProfSlot& s)
{
    if (!s.pool.empty()) {
        hipEvent_t e = s.pool.back();
        s.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfSlot& slot(lam_ctx* ctx, const char* name)
{
    for (auto& s : ctx->prof)
        if (s.name == name) return s;
    ctx->prof.push_back(ProfSlot{name, {}, {}, {}});
    return ctx->prof.back();
}
}  // namespace

void prof_mark(lam_ctx* ctx, const char* name, bool is_begin, hipStream_t st)
{
    if (!ctx || !ctx->profile_on.load()) return;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ProfSlot& s = slot(ctx, name);
    hipEvent_t e = take_event(s);
    if (!e) return;
    hipEventRecord(e, st);
    (is_begin ? s.begin : s.end).push_back(e);
}

void prof_release(lam_ctx* ctx)
{
    for (auto& s : ctx->prof) {
        for (auto e : s.begin) hipEventDestroy(e);
        for (auto e : s.end) hipEventDestroy(e);
        for (auto e : s.pool) hipEventDestroy(e);
    }
    ctx->prof.clear();
}

}  // namespace lam

using namespace lam;

extern "C" {

lam_status lam_profile_enable(lam_ctx* ctx, int on)
{
    if (!ctx) return LAM_ERR_INVALID_ARG;
    ctx->profile_on.store(on != 0 ? 1 : 0);
    return LAM_OK;
}

lam_status lam_profile_read(lam_ctx* ctx, const char* name, double* total_ms, int* count)
{
    if (!ctx || !name || !total_ms || !count) return LAM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    *total_ms = 0.0;
    *count = 0;
    for (auto& s : ctx->prof) {
        if (s.name != name) continue;
        const size_t n = std::min(s.begin.size(), s.end.size());
        for (size_t i = 0; i < n; ++i) {
            if (hipEventSynchronize(s.end[i]) != hipSuccess) return LAM_ERR_HIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s.begin[i], s.end[i]) != hipSuccess) return LAM_ERR_HIP;
            *total_ms += ms;
        }
        *count = (int)n;
        for (auto e : s.begin) s.pool.push_back(e);
        for (auto e : s.end) s.pool.push_back(e);
        s.begin.clear();
        s.end.clear();
    }
    return LAM_OK;
}

}  // extern "C"
