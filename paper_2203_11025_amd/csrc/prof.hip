// Kernel timing hook: HIP event pairs recorded on the launch stream around
// every launch of the selected kernel families, with the algorithmic work
// (bytes or FLOPs) of each launch, summed on demand.
#include <mutex>
#include <vector>

#include "helm_internal.h"

namespace helm {

namespace {
constexpr int NFAM = HELM_PROF_WGRAD + 1;
struct Family {
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t used = 0;             // events recorded so far
    bool open = false;           // a start without its stop
    long long seen = 0;          // launches since the start (timed or not)
    bool skip = false;           // the open launch is not timed
    double work = 0.0;           // summed algorithmic work of the closed pairs
};
struct Prof {
    std::mutex mu;
    unsigned mask = 0;
    int every = 1;        // time one launch in `every` of each family
    int active_rhs = -1;  // right-hand sides still iterating (set by the solver)
    Family f[NFAM];
};
Prof g_prof;
}  // namespace

// launches of this thread are not timed while positive (callers that must
// not create events)
thread_local int t_prof_suspended = 0;

void prof_suspend(bool on) { t_prof_suspended += on ? 1 : -1; }

bool prof_enabled() { return g_prof.mask != 0; }

void prof_set_active(int nact)
{
    if (!g_prof.mask) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.active_rhs = nact;
}

void prof_mark(int family, hipStream_t s, bool start, double work_per_rhs, int nb, bool masked)
{
    if (!(g_prof.mask & (1u << family)) || t_prof_suspended > 0) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    Family &F = g_prof.f[family];
    if (start == F.open) return;  // unbalanced call: ignore
    if (start) {
        // launch i is timed when a hash of i is divisible by the stride: a
        // fixed subset of about 1 / every of the launches that does not
        // alias with the period of a repeated launch sequence (the layers of
        // a network pass)
        unsigned long long z = (unsigned long long)F.seen++ * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ull;
        F.skip = g_prof.every > 1 && ((z ^ (z >> 29)) % (unsigned long long)g_prof.every) != 0;
        if (F.skip) {
            F.open = true;
            return;
        }
    } else if (F.skip) {
        F.open = false;
        return;
    }
    if (F.used == F.ev.size()) {
        // timing only (read after the caller synchronises): no system-scope
        // fence, whose cache writeback would stall and cool the next kernel
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return;
        F.ev.push_back(e);
    }
    if (hipEventRecord(F.ev[F.used], s) == hipSuccess) {
        ++F.used;
        F.open = start;
        if (!start) {
            // kernels that skip finished right-hand sides do the work of the
            // active ones only
            int cnt = nb;
            if (masked && g_prof.active_rhs >= 0 && g_prof.active_rhs < nb) cnt = g_prof.active_rhs;
            F.work += work_per_rhs * cnt;
        }
    }
}

}  // namespace helm

using namespace helm;

extern "C" int helm_profile_start(unsigned family_mask)
{
    if (family_mask >> NFAM) {
        set_error("helm_profile_start: unknown kernel family in the mask");
        return HELM_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.mask = family_mask;
    g_prof.active_rhs = -1;
    for (auto &F : g_prof.f) {
        F.used = 0;
        F.open = false;
        F.seen = 0;
        F.skip = false;
        F.work = 0.0;
    }
    return HELM_OK;
}

extern "C" int helm_profile_sample(int every)
{
    if (every < 1) {
        set_error("helm_profile_sample: the stride must be at least 1");
        return HELM_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.every = every;
    return HELM_OK;
}

extern "C" int helm_profile_read(int family, double *total_ms, long long *launches, double *work)
{
    if (family <= HELM_PROF_NONE || family >= NFAM) {
        set_error("helm_profile_read: unknown kernel family");
        return HELM_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    Family &F = g_prof.f[family];
    double tot = 0.0;
    size_t pairs = F.used / 2;
    for (size_t i = 0; i < pairs; ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(F.ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, F.ev[2 * i], F.ev[2 * i + 1]) != hipSuccess) {
            set_error("helm_profile_read: reading the timing events failed");
            return HELM_E_HIP;
        }
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (long long)pairs;
    if (work) *work = F.work;
    return HELM_OK;
}

extern "C" int helm_profile_stop(void)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.mask = 0;
    g_prof.active_rhs = -1;
    return HELM_OK;
}
