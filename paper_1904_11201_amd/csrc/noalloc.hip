// noalloc.hip -- join_hash_noalloc: the one-shot hash join of join_hash with its workspace in a
// static device array instead of a caller buffer, for callers that cannot allocate device
// memory.  The same kernels run (histogram, scatter, planning, count pass, scan, write pass);
// only where their scratch lives differs, and the exact count stays on the device.
#include <mutex>

#include "hash.hpp"

namespace jl {
namespace {

// The scratch array: one per GPU the library runs on, held until the process ends.  Its name
// is a host-side stand-in in host code; kernels get the device address looked up below.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_addr[kMaxDevices];  // device address of `scratch` per device (NULL: not looked up yet)

// Device address of this device's `scratch`, looked up once per device with that device current
// (the caller's current device).  A failed lookup is reported and tried again on the next call.
hipError_t scratch_address(char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[dev] = static_cast<char*>(p);
    }
    *out = g_addr[dev];
    return hipSuccess;
}

// *dst = *src, or v when src is NULL (the device-side count of an empty join).
__global__ void put_count_k(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src, uint64_t v)
{
    *dst = src ? *src : v;
}

}  // namespace
}  // namespace jl

using namespace jl;

extern "C" {

int join_hash_noalloc(const join_rel_t* R, const join_rel_t* S, int32_t* pairs, uint64_t capacity,
                      uint64_t* count, void* stream)
{
    if (!R || !S || !count) {
        set_error("join_hash_noalloc: R, S and count must not be NULL");
        return JOIN_E_INVAL;
    }
    const join_rel_t* X[2] = {R, S};
    for (const join_rel_t* x : X) {
        if (x->n < 0 || (x->n > 0 && !x->key)) {
            set_error("join_hash_noalloc: n < 0, or key NULL with n > 0");
            return JOIN_E_INVAL;
        }
        if (x->n > 2147483647) {
            set_error("join_hash_noalloc: n = %lld exceeds 2^31 - 1", (long long)x->n);
            return JOIN_E_UNSUPPORTED;
        }
    }
    if (capacity > 0 && !pairs) {
        set_error("join_hash_noalloc: pairs is NULL with capacity %llu", (unsigned long long)capacity);
        return JOIN_E_INVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return hip_fail(e, "join_hash_noalloc: scratch address");
    if (R->n == 0 || S->n == 0) {
        put_count_k<<<1, 1, 0, st>>>(count, nullptr, 0);
        e = hipGetLastError();
        return e == hipSuccess ? JOIN_OK : hip_fail(e, "join_hash_noalloc");
    }
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e, "join_hash_noalloc: device attributes");
    const HashPlan pl = hash_plan(R->n, S->n, cus > 0 ? cus : 256);
    if (pl.bytes > kScratchBytes) {
        set_error("join_hash_noalloc: this join needs %zu bytes of scratch, above the %zu bytes of "
                  "the static array; use join_hash with a workspace", pl.bytes, kScratchBytes);
        return JOIN_E_WORKSPACE;
    }
    // The count pass clears what it accumulates into (partition sizes, arrival counter) and
    // writes every per-unit count and the total before the write pass reads them, so nothing
    // left in the array by an earlier call is read.
    e = hash_count(pl, *R, *S, ws, st, nullptr, nullptr);
    if (e == hipSuccess) {
        put_count_k<<<1, 1, 0, st>>>(count, reinterpret_cast<const uint64_t*>(ws), 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hash_write(pl, *R, *S, ws, pairs, capacity, st);
    return e == hipSuccess ? JOIN_OK : hip_fail(e, "join_hash_noalloc");
}

}  // extern "C"
