// Optional per-kernel timing with HIP events recorded on the launch stream.
// Off by default; when on, every instrumented launch is bracketed by two
// events and lam_profile_read sums their elapsed times per kernel name.
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace lam {

namespace {
struct Slot {
    std::string name;
    std::vector<hipEvent_t> begin, end;  // recorded pairs
    std::vector<hipEvent_t> pool;        // free events
};
std::mutex g_mu;
bool g_on = false;
std::vector<Slot> g_slots;

hipEvent_t take_event(Slot& s)
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

Slot& slot(const char* name)
{
    for (auto& s : g_slots)
        if (s.name == name) return s;
    g_slots.push_back(Slot{name, {}, {}, {}});
    return g_slots.back();
}
}  // namespace

bool profiling() { return g_on; }

void prof_mark(const char* name, bool is_begin, hipStream_t st)
{
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Slot& s = slot(name);
    hipEvent_t e = take_event(s);
    if (!e) return;
    hipEventRecord(e, st);
    (is_begin ? s.begin : s.end).push_back(e);
}

}  // namespace lam

using namespace lam;

extern "C" {

lam_status lam_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return LAM_OK;
}

lam_status lam_profile_read(const char* name, double* total_ms, int* count)
{
    if (!name || !total_ms || !count) return LAM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    *total_ms = 0.0;
    *count = 0;
    for (auto& s : g_slots) {
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
