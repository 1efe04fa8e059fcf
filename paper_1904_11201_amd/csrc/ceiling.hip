// ceiling.hip -- what the chip sustains, for roofline fractions against measured rather than
// published peaks (include/join_prof.h): streaming copy, read and write kernels, and int32
// VALU spins.
#include "common.hpp"
#include "join_prof.h"
#include "prof.hpp"

namespace jl {
namespace {

constexpr int kStreamBlock = 1024;
constexpr int kStreamPerCU = 2;  // workgroups per compute unit (fastest of 2, 4, 8 and 16)
constexpr int kSpinBlock = 256;
constexpr int kSpinChains = 16;
constexpr uint32_t kSpinWidth = 1u << 20;  // band width of the MIX 1 compares

// Grid-stride streams of 16-byte non-temporal accesses, each lane keeping U of them in flight:
// a copy (U = 4), a read that folds what it reads into one word per lane (U = 8; the word is
// stored, so nothing is dropped) and a write of a lane-dependent pattern (U = 4).  These
// launch shapes were the fastest of a sweep over 1, 2, 4 and 8 accesses in flight, plain and
// non-temporal accesses, and 2 to 16 workgroups of 1024 lanes per compute unit.
template <int U>
__global__ __launch_bounds__(kStreamBlock) void copy_k(const i32x4* __restrict__ src,
                                                       i32x4* __restrict__ dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kStreamBlock;
    uint64_t i = (uint64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        i32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

template <int U>
__global__ __launch_bounds__(kStreamBlock) void read_k(const i32x4* __restrict__ src, uint64_t n,
                                                       int32_t* __restrict__ sink)
{
    const uint64_t stride = (uint64_t)gridDim.x * kStreamBlock;
    uint64_t i = (uint64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    i32x4 acc = {0, 0, 0, 0};
    for (; i + (U - 1) * stride < n; i += U * stride) {
        i32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u];
    }
    for (; i < n; i += stride) acc ^= __builtin_nontemporal_load(src + i);
    sink[(uint64_t)blockIdx.x * kStreamBlock + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

template <int U>
__global__ __launch_bounds__(kStreamBlock) void write_k(i32x4* __restrict__ dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kStreamBlock;
    uint64_t i = (uint64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    const int32_t t = (int32_t)threadIdx.x;
    const i32x4 v = {t, t + 1, t + 2, t + 3};
    for (; i + (U - 1) * stride < n; i += U * stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v, dst + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(v, dst + i);
}

// Workgroups of a stream over n vectors: kStreamPerCU per compute unit, fewer for small n.
uint32_t stream_grid(uint64_t n, int cus, int U)
{
    const uint64_t want = ceil_div((int64_t)n, (int64_t)kStreamBlock * U);
    const uint64_t most = (uint64_t)cus * kStreamPerCU;
    return (uint32_t)(want < most ? (want > 0 ? want : 1) : most);
}

// The VALU instructions are written as assembly so that the compiler can neither fuse nor drop
// them; an iteration issues 2 * kSpinChains of them per lane (MIX 0, 1, 3, 4) or 3 * kSpinChains
// (MIX 2).  MIX 0: kSpinChains independent chains of v_add_u32 + v_xor_b32.  MIX 1: the old band
// test of the nested-loop join, v_sub_u32 of a lane value from a scalar, v_cmp_le_u32 into VCC
// and s_or_b64 of VCC into a scalar mask (on the scalar unit).  MIX 2: the nested-loop join's
// group filter, two v_sub_u32 from a scalar and a v_min3_u32 into one of two running minima, for
// every pair of lane values, twice.  MIX 3 and MIX 4 take that filter's two instructions apart:
// chains of v_sub_u32 from a scalar only, and chains of v_min3_u32 only.  Workgroup 0 reads the
// shader clock counter and the constant-rate real-time counter around its loop.
// One step of the band spin: subtract the next lane value, or the previous mask into %0, compare.
#define SPIN_BAND_STEP(A) "v_sub_u32 %1, %2, " A "\n\ts_or_b64 %0, %0, vcc\n\tv_cmp_le_u32 vcc, %1, %3\n\t"

template <int MIX>
__global__ __launch_bounds__(kSpinBlock) void spin_k(uint32_t seed, uint32_t iters, uint32_t* sink,
                                                     uint64_t* clk)
{
    const uint32_t gid = blockIdx.x * kSpinBlock + threadIdx.x;
    const uint32_t b = seed ^ blockIdx.x;
    const uint32_t wv = kSpinWidth;
    uint32_t a[kSpinChains];
#pragma unroll
    for (int j = 0; j < kSpinChains; ++j) a[j] = gid * kSpinChains + j;
    uint64_t acc = 0;
    uint32_t mn[2] = {~0u, ~0u};
    const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
    uint64_t c0 = 0, r0 = 0;
    if (timer) {
        c0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    for (uint32_t it = 0; it < iters; ++it) {
        if (MIX == 0) {
#pragma unroll
            for (int j = 0; j < kSpinChains; ++j)
                asm volatile("v_add_u32 %0, %0, %1\n\tv_xor_b32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
        } else if (MIX == 3) {
            // subtracts from the scalar only, two per chain
#pragma unroll
            for (int j = 0; j < kSpinChains; ++j)
                asm volatile("v_sub_u32 %0, %1, %0\n\tv_sub_u32 %0, %1, %0" : "+v"(a[j]) : "s"(b));
        } else if (MIX == 4) {
            // three-input minima only, two per chain
#pragma unroll
            for (int j = 0; j < kSpinChains; ++j)
                asm volatile("v_min3_u32 %0, %0, %1, %2\n\tv_min3_u32 %0, %0, %2, %1"
                             : "+v"(a[j]) : "v"(b), "v"(wv));
        } else if (MIX == 2) {
            // twice over the 16 lane values: two subtracts from the scalar, one three-input min
            // into one of two running minima
#pragma unroll
            for (int rep = 0; rep < 2; ++rep)
#pragma unroll
                for (int j = 0; j < kSpinChains; j += 2) {
                    uint32_t t0, t1;
                    asm volatile("v_sub_u32 %1, %3, %4\n\tv_sub_u32 %2, %3, %5\n\tv_min3_u32 %0, %0, %1, %2"
                                 : "+v"(mn[(j >> 1) & 1]), "=&v"(t0), "=&v"(t1)
                                 : "s"(b), "v"(a[j]), "v"(a[j + 1]));
                }
        } else {
            // the nested-loop join's order: each subtract is issued before the previous compare's
            // mask is or-ed in, through one temporary and VCC
            uint32_t t;
            asm volatile(
                "v_sub_u32 %1, %2, %4\n\tv_cmp_le_u32 vcc, %1, %3\n\t"
                SPIN_BAND_STEP("%5") SPIN_BAND_STEP("%6") SPIN_BAND_STEP("%7") SPIN_BAND_STEP("%8")
                SPIN_BAND_STEP("%9") SPIN_BAND_STEP("%10") SPIN_BAND_STEP("%11") SPIN_BAND_STEP("%12")
                SPIN_BAND_STEP("%13") SPIN_BAND_STEP("%14") SPIN_BAND_STEP("%15") SPIN_BAND_STEP("%16")
                SPIN_BAND_STEP("%17") SPIN_BAND_STEP("%18") SPIN_BAND_STEP("%19")
                "s_or_b64 %0, %0, vcc"
                : "+s"(acc), "=&v"(t)
                : "s"(b), "v"(wv), "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]),
                  "v"(a[5]), "v"(a[6]), "v"(a[7]), "v"(a[8]), "v"(a[9]), "v"(a[10]), "v"(a[11]),
                  "v"(a[12]), "v"(a[13]), "v"(a[14]), "v"(a[15])
                : "vcc", "scc");  // s_or_b64 sets SCC
        }
    }
    if (timer) {
        const uint64_t c1 = __builtin_amdgcn_s_memtime();
        const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
        clk[0] = c1 - c0;
        clk[1] = r1 - r0;
    }
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < kSpinChains; ++j) f ^= a[j];
    sink[gid] = MIX == 0 || MIX >= 3 ? f : MIX == 2 ? min(mn[0], mn[1]) : (uint32_t)acc ^ (uint32_t)(acc >> 32);
}

}  // namespace
}  // namespace jl

using namespace jl;

extern "C" {

int join_prof_copy(const void* src, void* dst, uint64_t bytes, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if ((bytes && (!src || !dst)) || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16) {
        set_error("join_prof_copy: bytes must be a multiple of 16 and both pointers 16-byte aligned");
        return JOIN_E_INVAL;
    }
    if (!bytes) return JOIN_OK;
    int dev = 0, cus = 0;
    JL_HIP(hipGetDevice(&dev));
    JL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t n = bytes / 16;
    prof::Scope ps(st, "ceiling.copy");
    copy_k<4><<<stream_grid(n, cus, 4), kStreamBlock, 0, st>>>((const i32x4*)src, (i32x4*)dst, n);
    JL_LAUNCH("copy_k");
    return JOIN_OK;
}

int join_prof_stream(int mode, const void* src, void* dst, uint64_t bytes, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (mode < 1 || mode > 2 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16 ||
        (bytes && (!dst || (mode == 1 && !src)))) {
        set_error("join_prof_stream: mode 1 (read) or 2 (write), bytes a multiple of 16, pointers "
                  "16-byte aligned and non-null");
        return JOIN_E_INVAL;
    }
    if (!bytes) return JOIN_OK;
    int dev = 0, cus = 0;
    JL_HIP(hipGetDevice(&dev));
    JL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t n = bytes / 16;
    if (mode == 1) {
        prof::Scope ps(st, "ceiling.read");
        read_k<8><<<stream_grid(n, cus, 8), kStreamBlock, 0, st>>>((const i32x4*)src, n, (int32_t*)dst);
        JL_LAUNCH("read_k");
    } else {
        prof::Scope ps(st, "ceiling.write");
        write_k<4><<<stream_grid(n, cus, 4), kStreamBlock, 0, st>>>((i32x4*)dst, n);
        JL_LAUNCH("write_k");
    }
    return JOIN_OK;
}

int join_prof_valu(uint32_t blocks, uint32_t iters, int mix, uint32_t* sink, uint64_t* clk,
                   void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (!blocks || blocks > (1u << 22) || !sink || !clk || mix < 0 || mix > 4) {
        set_error("join_prof_valu: blocks must be in [1, 2^22], mix 0 to 4, sink and clk non-null");
        return JOIN_E_INVAL;
    }
    static const char* const names[] = {"ceiling.valu", "ceiling.valu.band", "ceiling.valu.min",
                                        "ceiling.valu.sub", "ceiling.valu.min3"};
    prof::Scope ps(st, names[mix]);
    if (mix == 4) spin_k<4><<<blocks, kSpinBlock, 0, st>>>(0x9e3779b9u, iters, sink, clk);
    else if (mix == 3) spin_k<3><<<blocks, kSpinBlock, 0, st>>>(0x9e3779b9u, iters, sink, clk);
    else if (mix == 2) spin_k<2><<<blocks, kSpinBlock, 0, st>>>(0x9e3779b9u, iters, sink, clk);
    else if (mix) spin_k<1><<<blocks, kSpinBlock, 0, st>>>(0x9e3779b9u, iters, sink, clk);
    else spin_k<0><<<blocks, kSpinBlock, 0, st>>>(0x9e3779b9u, iters, sink, clk);
    JL_LAUNCH("spin_k");
    return JOIN_OK;
}

int join_prof_wall_clock_khz(int* khz)
{
    if (!khz) {
        set_error("join_prof_wall_clock_khz: null pointer");
        return JOIN_E_INVAL;
    }
    int dev = 0;
    JL_HIP(hipGetDevice(&dev));
    JL_HIP(hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, dev));
    return JOIN_OK;
}

}  // extern "C"
