// common.hpp -- device primitives and host plumbing shared by the libjoin kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>

#include "join.h"

namespace jl {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------------------
// Wave-level primitives.  All of them assume every lane of the wave is active.
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `m` in lanes below this one (the wave-aggregated slot rank).
__device__ __forceinline__ uint32_t mask_rank(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// Move a wave-uniform value into a scalar register.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v);
}
__device__ __forceinline__ uint64_t uniform(uint64_t v)
{
    uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int64_t uniform(int64_t v) { return (int64_t)uniform((uint64_t)v); }

// Read-only view of a kernel input through the constant address space: a wave-uniform index
// then becomes a scalar (SMEM) load into SGPRs.  Only for buffers no kernel of the same launch
// writes.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p)
{
    return (cptr<T>)(p);
}

// A pointer known to be in global memory.  Loads through a generic pointer that the compiler
// cannot trace to a kernel argument become FLAT loads, which count against the LDS wait counter
// too: every wait for an LDS result would then also wait for them.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p)
{
    return (gptr<T>)(p);
}

// 16-byte load of four int32 through a global pointer (p 16-byte aligned).
using i32x4 = int32_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ i32x4 load4(gptr<int32_t> p) { return *(const __attribute__((address_space(1))) i32x4*)p; }

// Plan stamps.  Every workspace starts with a 256-byte header.  The count pass records at
// kStampOffset a signature of the plan it ran (sizes, fan-out, capacities, tiles: how the work
// was cut up), and the write pass, which plans again from its own arguments and the tuning
// knobs, writes nothing unless its plan's signature is the one recorded.  A knob changed
// between the two calls therefore cannot make the write pass read a layout the count pass did
// not leave.
constexpr size_t kStampOffset = 64;

inline uint64_t plan_stamp(std::initializer_list<int64_t> fields)
{
    uint64_t h = 0xcbf29ce484222325ull;  // FNV-1a over the fields' bytes
    for (int64_t f : fields)
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((f >> (8 * b)) & 0xff);
            h *= 0x100000001b3ull;
        }
    return h | 1ull;  // never 0 (a cleared header)
}

// Store a join's exact total into the caller's pinned host slot (device-visible address of host
// memory), after every earlier write of this thread: a system-scope release store, so the host
// thread polling the slot can size the output without a copy or a stream synchronisation.
__device__ __forceinline__ void publish_total(uint64_t* pub, uint64_t v)
{
    __hip_atomic_store(pub, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// DPP control codes (GFX9 encoding).
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowShr2 = 0x112;
constexpr int kDppRowShr4 = 0x114;
constexpr int kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

// Inclusive prefix sum across the 64 lanes: Hillis-Steele inside each row of 16 lanes with
// row_shr, then row_bcast:15 / row_bcast:31 carry the row totals upward.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    int v = (int)x;
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr1, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr2, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr4, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr8, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowBcast15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, kDppRowBcast31, 0xc, 0xf, false);
    return (uint32_t)v;
}

// One shift-and-add step of the 64-bit scan: both halves move with the same DPP pattern and
// the sum is formed in 64 bits, so carries between the halves are exact.
template <int CTRL, int RMASK, bool BC>
__device__ __forceinline__ uint64_t dpp_add64(uint64_t v)
{
    int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, RMASK, 0xf, BC);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, RMASK, 0xf, BC);
    return v + (((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x)
{
    x = dpp_add64<kDppRowShr1, 0xf, true>(x);
    x = dpp_add64<kDppRowShr2, 0xf, true>(x);
    x = dpp_add64<kDppRowShr4, 0xf, true>(x);
    x = dpp_add64<kDppRowShr8, 0xf, true>(x);
    x = dpp_add64<kDppRowBcast15, 0xa, false>(x);
    x = dpp_add64<kDppRowBcast31, 0xc, false>(x);
    return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(x), 63);
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x)
{
    uint64_t s = wave_incl_scan64(x);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s, 63);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(s >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// Block-wide exclusive scan of one uint32 per thread.  `lds` holds at least blockDim/64 + 1
// words.  Returns the exclusive prefix; *total receives the block sum (every thread).
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* lds, uint32_t* total)
{
    constexpr int W = BLOCK / kWave;
    const int wv = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(x);
    if (lane_id() == kWave - 1) lds[wv] = inc;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint32_t t = lds[i];
        before += (i < wv) ? t : 0u;
        sum += t;
    }
    __syncthreads();
    *total = sum;
    return before + inc - x;
}

// ---------------------------------------------------------------------------------------------
// Hashing: the 32-bit finaliser of MurmurHash3 (a bijection on 32-bit words).  The partition id
// takes the top bits; the LDS table position takes the bits below them.
// ---------------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t hmix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------------------------
// Host-side error capture.
// ---------------------------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

}  // namespace jl

#define JL_HIP(call)                                                  \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return ::jl::hip_fail(e_, #call);       \
    } while (0)

#define JL_LAUNCH(what)                                               \
    do {                                                              \
        hipError_t e_ = hipGetLastError();                            \
        if (e_ != hipSuccess) return ::jl::hip_fail(e_, what);        \
    } while (0)
