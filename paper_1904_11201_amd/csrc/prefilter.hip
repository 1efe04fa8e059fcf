// prefilter.hip -- the pre-filter of Algorithm 1 (Section 3.1) on the GPU.
//
// The paper's first MapReduce round collects the join keys that occur in both tables and the
// second drops every tuple of either table whose key is not among them, so that only tuples
// that can appear in the result reach the join.  Here each relation sets one bit per key in
// a bit filter (bit = top bits of the key hash); a tuple of R survives if its bit is set in the
// filter of S and vice versa.  A filter only says "maybe present": it never drops a tuple whose
// key occurs on the other side, so the join of the survivors is exactly the join of the inputs
// (the same multiset of (rid_R, rid_S) pairs); keys that merely collide in a filter survive and
// then find no partner.  Survivors keep their rid payload (or their row position).
//
// A filter is built with one atomic OR per row at a random word, which is cheap only while the
// filter stays in the L2 caches: filters get 16 bits per row and at most 2^24 bits (2 MB), and a
// relation of more than 2^21 rows gets no filter (its partner relation is then not filtered).
// So the small side of a join always filters the large one (a semi-join), and both sides are
// filtered, as in the paper, when both are small enough.
#include "prefilter.hpp"

#include "prof.hpp"
#include "scan.hpp"

namespace jl {

namespace {

constexpr int kBlock = 1024;

__device__ __forceinline__ uint32_t filter_bit(int32_t key, int logm)
{
    return hmix((uint32_t)key) >> (32 - logm);
}

__global__ void zero_words_k(uint32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ __launch_bounds__(kBlock) void set_bits_k(const int32_t* __restrict__ key, int64_t n,
                                                     uint32_t* __restrict__ filter, int logm)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const uint32_t b = filter_bit(key[i], logm);
        atomicOr(&filter[b >> 5], 1u << (b & 31));
    }
}

// Keeps the rows whose bit is set in the other relation's filter.  A workgroup takes kPer rows
// per thread per round; waves count their survivors with ballots, one thread reserves the
// workgroup's range of the output with one global atomic, and every wave writes its survivors
// at its offset inside that range.
constexpr int kPer = 8;

__global__ __launch_bounds__(kBlock) void compact_k(const int32_t* __restrict__ key,
                                                    const int32_t* __restrict__ rid, int64_t n,
                                                    const uint32_t* __restrict__ filter, int logm,
                                                    int32_t* __restrict__ okey, int32_t* __restrict__ orid,
                                                    uint32_t* __restrict__ counter)
{
    __shared__ uint32_t wtot[kBlock / kWave];
    __shared__ uint32_t gbase;
    const int wv = threadIdx.x / kWave;
    const int64_t step = (int64_t)kBlock * kPer;
    for (int64_t base = (int64_t)blockIdx.x * step; base < n; base += (int64_t)gridDim.x * step) {
        int32_t k[kPer], r[kPer];
        uint32_t fw[kPer];
        uint64_t m[kPer];
        uint32_t mine = 0;
        // all key and rid loads first, then all filter reads, then the ballots: every load of
        // the round is in flight together
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t i = base + (int64_t)q * kBlock + threadIdx.x;
            k[q] = i < n ? key[i] : 0;
            r[q] = i < n ? (rid ? rid[i] : (int32_t)i) : 0;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) fw[q] = filter[filter_bit(k[q], logm) >> 5];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int64_t i = base + (int64_t)q * kBlock + threadIdx.x;
            const bool keep = i < n && ((fw[q] >> (filter_bit(k[q], logm) & 31)) & 1u);
            m[q] = ballot(keep);
            mine += (uint32_t)__builtin_popcountll(m[q]);
        }
        if (lane_id() == 0) wtot[wv] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < kBlock / kWave; ++w) {
                const uint32_t c = wtot[w];
                wtot[w] = t;
                t += c;
            }
            gbase = t ? atomicAdd(counter, t) : 0u;
        }
        __syncthreads();
        uint32_t at = gbase + wtot[wv];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            if ((m[q] >> lane_id()) & 1u) {
                const uint32_t pos = at + mask_rank(m[q]);
                okey[pos] = k[q];
                orid[pos] = r[q];
            }
            at += (uint32_t)__builtin_popcountll(m[q]);
        }
        __syncthreads();  // wtot and gbase are reused by the next round
    }
}

constexpr int kMinLog = 16, kMaxLog = 24;
constexpr int64_t kMaxFilteredRows = (int64_t)1 << 21;

// log2 of the filter size in bits for a relation of n rows, or 0 for no filter
int log_bits(int64_t n)
{
    if (n <= 0 || n > kMaxFilteredRows) return 0;
    int l = kMinLog;
    while (l < kMaxLog && ((int64_t)1 << l) < 16 * n) ++l;
    return l;
}

}  // namespace

PrefilterPlan prefilter_plan(int64_t nR, int64_t nS, int num_cus)
{
    PrefilterPlan pl{};
    pl.nR = nR;
    pl.nS = nS;
    pl.logR = log_bits(nR);
    pl.logS = log_bits(nS);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off = (off + b + 255) & ~(size_t)255;
        return at;
    };
    pl.off_cnt = take(8);
    pl.off_fR = take(pl.logR ? ((size_t)1 << pl.logR) / 8 : 0);
    pl.off_fS = take(pl.logS ? ((size_t)1 << pl.logS) / 8 : 0);
    // R is compacted when S has a filter, S when R has one
    pl.off_kR = take(pl.logS ? (size_t)nR * 4 : 0);
    pl.off_rR = take(pl.logS ? (size_t)nR * 4 : 0);
    pl.off_kS = take(pl.logR ? (size_t)nS * 4 : 0);
    pl.off_rS = take(pl.logR ? (size_t)nS * 4 : 0);
    // The inner join sees at most nR x nS rows.  Its layout grows with the sizes except the
    // chunk arrays (group shares, and the per-tile counts' last partial tile of every chunk),
    // which a smaller fan-out may lay out for twice the chunks: bounded by 2^11 partitions x 2
    // chunks per CU x 2 sides, twice.
    pl.inner_bytes = hash_plan(nR, nS, num_cus).bytes + ((size_t)1 << 11) * num_cus * 2 * 4 * 2 * 2 + 4096;
    pl.off_inner = take(pl.inner_bytes);
    pl.bytes = off;
    pl.stamp = plan_stamp({JOIN_KIND_HASH_PREFILTER, nR, nS, pl.logR, pl.logS, (int64_t)pl.inner_bytes,
                           (int64_t)hash_plan(nR, nS, num_cus).stamp, (int64_t)pl.bytes});
    return pl;
}

// The relations the inner join sees: the compacted columns of a filtered side, else the input.
static void survivors(const PrefilterPlan& pl, char* ws, const uint32_t* n, const join_rel_t& R,
                      const join_rel_t& S, join_rel_t* R2, join_rel_t* S2)
{
    *R2 = pl.logS ? join_rel_t{reinterpret_cast<const int32_t*>(ws + pl.off_kR), nullptr,
                               reinterpret_cast<const int32_t*>(ws + pl.off_rR), (int64_t)n[0]}
                  : R;
    *S2 = pl.logR ? join_rel_t{reinterpret_cast<const int32_t*>(ws + pl.off_kS), nullptr,
                               reinterpret_cast<const int32_t*>(ws + pl.off_rS), (int64_t)n[1]}
                  : S;
}

static hipError_t read_sizes(const PrefilterPlan& pl, char* ws, hipStream_t st, uint32_t* n)
{
    static thread_local uint32_t* slot = nullptr;
    if (!slot && hipHostMalloc((void**)&slot, 64, hipHostMallocDefault) != hipSuccess) {
        slot = nullptr;
        return hipErrorOutOfMemory;
    }
    hipError_t e = hipMemcpyAsync(slot, ws + pl.off_cnt, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    n[0] = slot[0];
    n[1] = slot[1];
    return e;
}

hipError_t prefilter_count(const PrefilterPlan& pl, const join_rel_t& R, const join_rel_t& S,
                           char* ws, hipStream_t st, int num_cus, uint64_t* pub)
{
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + pl.off_cnt);
    uint32_t* fR = reinterpret_cast<uint32_t*>(ws + pl.off_fR);
    uint32_t* fS = reinterpret_cast<uint32_t*>(ws + pl.off_fS);
    const unsigned grid = (unsigned)num_cus * 8;
    {
        prof::Scope pf(st, "prefilter.filters");
        // the filters and the counters are cleared by kernels (no memset in the stream)
        zero_words_k<<<1, 256, 0, st>>>(cnt, 2);
        if (pl.logR) {
            zero_words_k<<<grid, 256, 0, st>>>(fR, ((int64_t)1 << pl.logR) / 32);
            set_bits_k<<<grid, kBlock, 0, st>>>(R.key, R.n, fR, pl.logR);
        }
        if (pl.logS) {
            zero_words_k<<<grid, 256, 0, st>>>(fS, ((int64_t)1 << pl.logS) / 32);
            set_bits_k<<<grid, kBlock, 0, st>>>(S.key, S.n, fS, pl.logS);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        prof::Scope pc(st, "prefilter.compact");
        if (pl.logS)
            compact_k<<<grid, kBlock, 0, st>>>(R.key, R.rid, R.n, fS, pl.logS,
                                               reinterpret_cast<int32_t*>(ws + pl.off_kR),
                                               reinterpret_cast<int32_t*>(ws + pl.off_rR), cnt);
        if (pl.logR)
            compact_k<<<grid, kBlock, 0, st>>>(S.key, S.rid, S.n, fR, pl.logR,
                                               reinterpret_cast<int32_t*>(ws + pl.off_kS),
                                               reinterpret_cast<int32_t*>(ws + pl.off_rS), cnt + 1);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t n[2] = {0, 0};
    if (pl.logR || pl.logS) {
        e = read_sizes(pl, ws, st, n);
        if (e != hipSuccess) return e;
    }
    join_rel_t R2, S2;
    survivors(pl, ws, n, R, S, &R2, &S2);
    char* inner = ws + pl.off_inner;
    if (R2.n == 0 || S2.n == 0) {
        // nothing survives on one side: the count is 0 (total and unit count cleared)
        zero_words_k<<<1, 256, 0, st>>>(reinterpret_cast<uint32_t*>(inner), 4);
        e = hipGetLastError();
        // a scan of nothing stores the zero total into the host slot
        if (e == hipSuccess && pub) e = exclusive_scan<uint64_t>(nullptr, nullptr, 0, nullptr, nullptr, st, pub);
        return e;
    }
    const HashPlan hp = hash_plan(R2.n, S2.n, num_cus);
    if (hp.bytes > pl.inner_bytes) return hipErrorInvalidValue;  // cannot happen: see the plan
    return hash_count(hp, R2, S2, inner, st, nullptr, pub);
}

hipError_t prefilter_write(const PrefilterPlan& pl, const join_rel_t& R, const join_rel_t& S,
                           char* ws, int32_t* pairs, uint64_t cap, hipStream_t st, int num_cus)
{
    uint32_t n[2] = {0, 0};
    if (pl.logR || pl.logS) {
        hipError_t e = read_sizes(pl, ws, st, n);
        if (e != hipSuccess) return e;
    }
    join_rel_t R2, S2;
    survivors(pl, ws, n, R, S, &R2, &S2);
    if (R2.n == 0 || S2.n == 0) return hipSuccess;
    return hash_write(hash_plan(R2.n, S2.n, num_cus), R2, S2, ws + pl.off_inner, pairs, cap, st);
}

}  // namespace jl
