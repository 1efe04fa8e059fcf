// prof.hip -- per-kernel HIP-event timing (include/join_prof.h).
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "join_prof.h"
#include "prof.hpp"

namespace jl {
namespace prof {

namespace {

struct Pending {
    std::string name;
    hipEvent_t a, b;
};

struct Total {
    uint64_t launches = 0;
    double ms = 0;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
std::map<std::string, Total> g_totals;
std::vector<std::string> g_names;  // stable storage for join_prof_entry
thread_local std::vector<Pending> t_open;

hipEvent_t get_event()
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

bool enabled() { return g_on.load(std::memory_order_relaxed); }

void begin(hipStream_t st, const char* name)
{
    Pending p;
    p.name = name;
    p.a = get_event();
    p.b = get_event();
    if (!p.a || !p.b) return;
    hipEventRecord(p.a, st);
    t_open.push_back(p);
}

void end(hipStream_t st)
{
    if (t_open.empty()) return;
    Pending p = t_open.back();
    t_open.pop_back();
    hipEventRecord(p.b, st);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back(p);
}

}  // namespace prof
}  // namespace jl

using namespace jl::prof;

extern "C" {

int join_prof_enable(int on)
{
    if (on) {
        join_prof_collect();
        std::lock_guard<std::mutex> lk(g_mu);
        g_totals.clear();
        g_names.clear();
    }
    g_on.store(on != 0);
    return JOIN_OK;
}

int join_prof_collect(void)
{
    std::vector<Pending> todo;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        todo.swap(g_pending);
    }
    int rc = JOIN_OK;
    for (auto& p : todo) {
        float ms = 0;
        hipError_t e = hipEventSynchronize(p.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) rc = jl::hip_fail(e, "join_prof_collect");
        std::lock_guard<std::mutex> lk(g_mu);
        Total& t = g_totals[p.name];
        t.launches += 1;
        t.ms += ms;
        g_free.push_back(p.a);
        g_free.push_back(p.b);
    }
    return rc;
}

int join_prof_count(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_names.clear();
    for (auto& kv : g_totals) g_names.push_back(kv.first);
    return (int)g_names.size();
}

int join_prof_entry(int i, const char** name, uint64_t* launches, double* total_ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int)g_names.size()) return JOIN_E_INVAL;
    const Total& t = g_totals[g_names[i]];
    if (name) *name = g_names[i].c_str();
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.ms;
    return JOIN_OK;
}

}  // extern "C"
