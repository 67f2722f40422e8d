// Kernel timing hook: HIP event pairs recorded on the launch stream around
// every launch of one selected kernel family, summed on demand.
#include <mutex>
#include <vector>

#include "helm_internal.h"

namespace helm {

namespace {
struct Prof {
    std::mutex mu;
    int family = HELM_PROF_NONE;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t used = 0;             // events recorded so far
    bool open = false;           // a start without its stop
};
Prof g_prof;
}  // namespace

void prof_mark(int family, hipStream_t s, bool start)
{
    if (g_prof.family != family) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (start == g_prof.open) return;  // unbalanced call: ignore
    if (g_prof.used == g_prof.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        g_prof.ev.push_back(e);
    }
    if (hipEventRecord(g_prof.ev[g_prof.used], s) == hipSuccess) {
        ++g_prof.used;
        g_prof.open = start;
    }
}

}  // namespace helm

using namespace helm;

extern "C" int helm_profile_start(int family)
{
    if (family < HELM_PROF_NONE || family > HELM_PROF_APPLY) {
        set_error("helm_profile_start: unknown kernel family");
        return HELM_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.family = family;
    g_prof.used = 0;
    g_prof.open = false;
    return HELM_OK;
}

extern "C" int helm_profile_stop(double *total_ms, long long *launches)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    double tot = 0.0;
    size_t pairs = g_prof.used / 2;
    for (size_t i = 0; i < pairs; ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(g_prof.ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess) {
            set_error("helm_profile_stop: reading the timing events failed");
            g_prof.family = HELM_PROF_NONE;
            return HELM_E_HIP;
        }
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (long long)pairs;
    g_prof.family = HELM_PROF_NONE;
    g_prof.used = 0;
    g_prof.open = false;
    return HELM_OK;
}
