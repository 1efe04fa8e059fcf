// debug.hip -- the checks of the checking build (JL_DEBUG): a fingerprint of device buffers, and
// the comparison of what the write pass wrote per work unit with what the count pass counted.
// The kernels exist in every build; only the checking build calls them (api.hip).
#include "debug.hpp"

namespace jl {
namespace {

constexpr int kFpBlock = 256;

// Order-independent 64-bit fingerprint: every 32-bit word w at index i contributes
// mix(w, i), a SplitMix64-style finaliser of both, and the contributions are summed.
__device__ __forceinline__ uint64_t fp_mix(uint32_t w, uint64_t i)
{
    uint64_t z = ((uint64_t)w << 32 | (uint32_t)i) ^ (i * 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kFpBlock) void fingerprint_k(const uint32_t* __restrict__ p, uint64_t n,
                                                          uint64_t salt, uint64_t* __restrict__ out)
{
    __shared__ uint64_t part[kFpBlock / kWave];
    uint64_t s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kFpBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kFpBlock)
        s += fp_mix(p[i], i + salt);
    s = wave_sum64(s);
    if (lane_id() == 0) part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kFpBlock / kWave; ++w) t += part[w];
        atomicAdd(reinterpret_cast<unsigned long long*>(out), (unsigned long long)t);
    }
}

__global__ void zero_u64_k(uint64_t* __restrict__ p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Units whose written count differs from offsets[u + 1] - offsets[u] (the last unit's end is the
// total) are counted into *bad.
__global__ void check_units_k(const uint64_t* __restrict__ offsets, const uint64_t* __restrict__ total,
                              const uint64_t* __restrict__ written, int64_t units, int64_t nOff,
                              uint32_t* __restrict__ bad)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t end = u + 1 < nOff ? offsets[u + 1] : *total;
        if (written[u] != end - offsets[u]) atomicAdd(bad, 1u);
    }
}

}  // namespace

hipError_t dbg_zero(uint64_t* p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    zero_u64_k<<<(unsigned)(n < 65536 ? ceil_div(n, 256) : 256), 256, 0, st>>>(p, (uint64_t)n);
    return hipGetLastError();
}

hipError_t dbg_fingerprint(const void* p, uint64_t bytes, uint64_t salt, uint64_t* out, hipStream_t st)
{
    const uint64_t n = bytes / 4;
    if (!p || n == 0) return hipSuccess;
    const uint64_t want = (n + kFpBlock - 1) / kFpBlock;
    fingerprint_k<<<(unsigned)(want < 4096 ? want : 4096), kFpBlock, 0, st>>>(
        static_cast<const uint32_t*>(p), n, salt, out);
    return hipGetLastError();
}

hipError_t dbg_check_units(const uint64_t* offsets, const uint64_t* total, const uint64_t* written,
                           int64_t units, int64_t nOff, uint32_t* bad, hipStream_t st)
{
    if (units <= 0) return hipSuccess;
    check_units_k<<<(unsigned)(units < 65536 ? ceil_div(units, 256) : 256), 256, 0, st>>>(
        offsets, total, written, units, nOff, bad);
    return hipGetLastError();
}

}  // namespace jl
