// prof.hpp -- opt-in HIP-event timing of each kernel launch (include/join_prof.h).
#pragma once
#include "common.hpp"

namespace jl {
namespace prof {

bool enabled();
void begin(hipStream_t st, const char* name);
void end(hipStream_t st);

// Brackets one launch: records a start event on construction and a stop event on destruction,
// both on the launch stream, when profiling is enabled.
struct Scope {
    hipStream_t st;
    bool on;
    Scope(hipStream_t s, const char* name) : st(s), on(enabled())
    {
        if (on) begin(st, name);
    }
    ~Scope()
    {
        if (on) end(st);
    }
};

}  // namespace prof
}  // namespace jl
