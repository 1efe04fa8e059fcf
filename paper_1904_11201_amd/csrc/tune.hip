// tune.hip -- process-wide tuning knobs (include/join_tune.h).
#include "tune.hpp"

#include <atomic>
#include <stdlib.h>
#include <string.h>

#include "join_tune.h"

namespace jl {

namespace {

struct KnobDesc {
    const char* name;
    const char* env;
};

const KnobDesc kKnobs[TUNE_COUNT] = {
    {"hash.cap", "JOIN_HASH_CAP"},
    {"hash.slice", "JOIN_HASH_SLICE"},
    {"hash.bits", "JOIN_HASH_BITS"},
    {"hash.single_max_chunks", "JOIN_HASH_SINGLE_MAX_CHUNKS"},
    {"theta.ts", "JOIN_THETA_TS"},
    {"theta.waves", "JOIN_THETA_WAVES"},
    {"theta.stash", "JOIN_THETA_STASH"},
    {"hash.deterministic", "JOIN_HASH_DETERMINISTIC"},
};

constexpr int64_t kUnset = INT64_MIN;

struct Overrides {
    std::atomic<int64_t> v[TUNE_COUNT];
    Overrides()
    {
        for (auto& x : v) x.store(kUnset, std::memory_order_relaxed);
    }
};

Overrides& overrides()
{
    static Overrides o;  // initialised once, thread-safe
    return o;
}

int find(const char* name)
{
    if (!name) return -1;
    for (int i = 0; i < TUNE_COUNT; ++i)
        if (strcmp(name, kKnobs[i].name) == 0) return i;
    return -1;
}

// Values set for the calling thread only (join_tune_set_local); they win over the process-wide
// ones.
struct LocalOverrides {
    int64_t v[TUNE_COUNT];
    LocalOverrides()
    {
        for (auto& x : v) x = kUnset;
    }
};
thread_local LocalOverrides g_local;

}  // namespace

int64_t tune_get(TuneKnob k, int64_t dflt)
{
    if (g_local.v[k] != kUnset) return g_local.v[k];
    const int64_t v = overrides().v[k].load(std::memory_order_relaxed);
    if (v != kUnset) return v;
    const char* s = getenv(kKnobs[k].env);
    if (s && *s) return atoll(s);
    return dflt;
}

}  // namespace jl

extern "C" {

int join_tune_set(const char* name, int64_t value, int clear)
{
    const int i = jl::find(name);
    if (i < 0) return JOIN_TUNE_UNKNOWN;
    jl::overrides().v[i].store(clear ? jl::kUnset : value, std::memory_order_relaxed);
    return 0;
}

int join_tune_set_local(const char* name, int64_t value, int clear)
{
    const int i = jl::find(name);
    if (i < 0) return JOIN_TUNE_UNKNOWN;
    jl::g_local.v[i] = clear ? jl::kUnset : value;
    return 0;
}

int join_tune_get(const char* name, int64_t dflt, int64_t* value)
{
    const int i = jl::find(name);
    if (i < 0 || !value) return JOIN_TUNE_UNKNOWN;
    *value = jl::tune_get(static_cast<jl::TuneKnob>(i), dflt);
    return 0;
}

}  // extern "C"
