// Phase profiler behind arborx_profile_enable / arborx_profile_collect.
#include "profile.hpp"

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace ax {

namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
}  // namespace

bool profiling() { return g_on; }

hipEvent_t prof_event()
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

void prof_record(const char *name, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_pending.push_back({name, a, b});
}

}  // namespace ax

using namespace ax;

extern "C" {

arborx_status arborx_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_on = on != 0;
    return ARBORX_OK;
}

arborx_status arborx_profile_collect(char *names, double *ms, int64_t *launches, int32_t cap, int32_t *count)
{
    if (!count || cap < 0 || (cap > 0 && (!names || !ms || !launches)))
        return fail(ARBORX_E_INVALID, "bad arguments");
    std::vector<Pending> todo;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        todo.swap(g_pending);
    }
    std::map<std::string, std::pair<double, int64_t>> acc;
    for (auto &p : todo) {
        float t = 0.0f;
        AX_HIP(hipEventSynchronize(p.b));
        AX_HIP(hipEventElapsedTime(&t, p.a, p.b));
        auto &e = acc[p.name];
        e.first += t;
        e.second += 1;
    }
    {
        std::lock_guard<std::mutex> lock(g_mu);
        for (auto &p : todo) {
            g_free.push_back(p.a);
            g_free.push_back(p.b);
        }
    }
    int i = 0;
    for (auto &kv : acc) {
        if (i >= cap)
            break;
        std::strncpy(names + 32 * i, kv.first.c_str(), 31);
        names[32 * i + 31] = '\0';
        ms[i] = kv.second.first;
        launches[i] = kv.second.second;
        ++i;
    }
    *count = i;
    return ARBORX_OK;
}

}  // extern "C"
