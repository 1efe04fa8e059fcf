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
#include "tune.hpp"

namespace jl {

namespace {

constexpr int kBlock = 1024;

// A blocked filter with two bits per key: both in one 32-bit word.  The word index takes the top
// bits of the key hash, the two bit positions its lowest ten bits (independent of the top ones
// while the filter has at most 2^24 bits).  At 16 bits per key this leaves about 1.4% false
// positives, where one bit per key leaves about 6%, for the same one word read per lookup.
struct FilterSlot {
    uint32_t word, mask;
};

__device__ __forceinline__ FilterSlot filter_slot(int32_t key, int logm)
{
    const uint32_t h = hmix((uint32_t)key);
    return FilterSlot{h >> (32 - (logm - 5)), (1u << (h & 31)) | (1u << ((h >> 5) & 31))};
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
        const FilterSlot f = filter_slot(key[i], logm);
        atomicOr(&filter[f.word], f.mask);
    }
}

// One round of a compaction: kPer rows per thread (all loads, then all filter reads, in flight
// together) and the ballots of the rows that pass.
constexpr int kPer = 8;

struct Round {
    int32_t k[kPer], r[kPer];
    uint64_t m[kPer];
    uint32_t count;  // wave-uniform: rows of this wave that pass
};

__device__ __forceinline__ void round_of(const int32_t* __restrict__ key, const int32_t* __restrict__ rid,
                                         int64_t base, int64_t end, const uint32_t* __restrict__ filter,
                                         int logm, Round& rd)
{
    uint32_t fw[kPer];
    FilterSlot fs[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t i = base + (int64_t)q * kBlock + threadIdx.x;
        rd.k[q] = i < end ? key[i] : 0;
        rd.r[q] = i < end ? (rid ? rid[i] : (int32_t)i) : 0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        fs[q] = filter_slot(rd.k[q], logm);
        fw[q] = filter[fs[q].word];
    }
    rd.count = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t i = base + (int64_t)q * kBlock + threadIdx.x;
        rd.m[q] = ballot(i < end && (fw[q] & fs[q].mask) == fs[q].mask);
        rd.count += (uint32_t)__builtin_popcountll(rd.m[q]);
    }
}

// This wave's passing rows of a round, the first `skip` of them left out, the next `take` written
// from out position at on (in (q, lane) order).
__device__ __forceinline__ void put_round(const Round& rd, uint32_t skip, uint32_t take, uint32_t at,
                                          int32_t* __restrict__ okey, int32_t* __restrict__ orid)
{
    uint32_t before = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t j = before + mask_rank(rd.m[q]);  // this lane's rank among the passing rows
        if (((rd.m[q] >> lane_id()) & 1u) && j >= skip && j < skip + take) {
            okey[at + j - skip] = rd.k[q];
            orid[at + j - skip] = rd.r[q];
        }
        before += (uint32_t)__builtin_popcountll(rd.m[q]);
    }
}

// Arrival-order compaction: waves append their passing rows to a workgroup stage in LDS (one LDS
// atomic per wave and round, no barrier), and the workgroup writes the stage out in one
// coalesced run at the end, reserved with one global atomic.  Rows that find the stage full go
// straight out with a global atomic of their wave.
constexpr int kStage = 8192;

__global__ __launch_bounds__(kBlock) void compact_k(const int32_t* __restrict__ key,
                                                    const int32_t* __restrict__ rid, int64_t n,
                                                    const uint32_t* __restrict__ filter, int logm,
                                                    int32_t* __restrict__ okey, int32_t* __restrict__ orid,
                                                    uint32_t* __restrict__ counter)
{
    __shared__ int32_t sk[kStage], sr[kStage];
    __shared__ uint32_t sn, gbase;
    if (threadIdx.x == 0) sn = 0;
    __syncthreads();
    const int64_t step = (int64_t)kBlock * kPer;
    for (int64_t base = (int64_t)blockIdx.x * step; base < n; base += (int64_t)gridDim.x * step) {
        Round rd;
        round_of(key, rid, base, n, filter, logm, rd);
        if (rd.count == 0) continue;  // uniform
        uint32_t at = 0;
        if (lane_id() == 0) at = atomicAdd(&sn, rd.count);
        at = uniform(__shfl(at, 0));
        const uint32_t staged = at >= (uint32_t)kStage ? 0u : min(rd.count, (uint32_t)kStage - at);
        if (staged) put_round(rd, 0, staged, at, sk, sr);
        if (staged < rd.count) {  // uniform: the stage is full
            uint32_t g = 0;
            if (lane_id() == 0) g = atomicAdd(counter, rd.count - staged);
            put_round(rd, staged, rd.count - staged, uniform(__shfl(g, 0)), okey, orid);
        }
    }
    __syncthreads();
    const uint32_t ns = min(sn, (uint32_t)kStage);
    if (threadIdx.x == 0) gbase = ns ? atomicAdd(counter, ns) : 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < ns; i += kBlock) {
        okey[gbase + i] = sk[i];
        orid[gbase + i] = sr[i];
    }
}

// Ordered compaction (the deterministic option): workgroup b takes rows [b * per, (b + 1) * per)
// and places its passing rows in (round, wave, q, lane) order.  WRITE = false counts them into
// counts[b]; WRITE = true writes them from offsets[b] (the exclusive scan of the counts).
template <bool WRITE>
__global__ __launch_bounds__(kBlock) void compact_ordered_k(const int32_t* __restrict__ key,
                                                            const int32_t* __restrict__ rid, int64_t n,
                                                            int64_t per, const uint32_t* __restrict__ filter,
                                                            int logm, uint32_t* __restrict__ counts,
                                                            int32_t* __restrict__ okey, int32_t* __restrict__ orid)
{
    __shared__ uint32_t wtot[kBlock / kWave];
    const int wv = threadIdx.x / kWave;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    uint32_t run = WRITE ? counts[blockIdx.x] : 0u;
    for (int64_t base = b0; base < b1; base += (int64_t)kBlock * kPer) {
        Round rd;
        round_of(key, rid, base, b1, filter, logm, rd);
        if (lane_id() == 0) wtot[wv] = rd.count;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            const uint32_t c = wtot[w];
            before += w < wv ? c : 0u;
            tot += c;
        }
        if (WRITE && rd.count) put_round(rd, 0, rd.count, run + before, okey, orid);
        run += tot;
        __syncthreads();  // wtot is reused by the next round
    }
    if (!WRITE && threadIdx.x == 0) counts[blockIdx.x] = run;
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
    // A probe side too large for a filter of its own is also too large to check row by row
    // against R's filter at the rate the caches serve random words: there the hash join's count
    // pass is the filter (the semi-join, exact, from its LDS tables), and its write pass visits
    // only the probe rows it recorded as matching.
    pl.semi = nS > kMaxFilteredRows ? 1 : 0;
    pl.logR = pl.semi ? 0 : log_bits(nR);
    pl.logS = pl.semi ? 0 : log_bits(nS);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off = (off + b + 255) & ~(size_t)255;
        return at;
    };
    pl.ordered = tune_get(TUNE_HASH_DETERMINISTIC, 0) != 0 ? 1 : 0;
    pl.grid = num_cus * 8;
    pl.off_cnt = take(8);
    // the ordered compaction's per-workgroup counts (then offsets) and its scan's storage
    pl.off_wcnt = take(pl.ordered ? (size_t)pl.grid * 4 : 0);
    pl.off_wtmp = take(pl.ordered ? scan_temp_elems<uint32_t>(pl.grid) * 4 : 0);
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
    const HashPlan full = hash_plan(nR, nS, num_cus, -1, pl.semi != 0);
    pl.inner_bytes = pl.semi ? full.bytes
                             : full.bytes + ((size_t)1 << 11) * num_cus * 2 * 4 * 2 * 2 + 4096;
    pl.off_inner = take(pl.inner_bytes);
    pl.bytes = off;
    pl.stamp = plan_stamp({JOIN_KIND_HASH_PREFILTER, nR, nS, pl.semi, pl.logR, pl.logS, pl.ordered, pl.grid,
                           (int64_t)pl.inner_bytes, (int64_t)full.stamp, (int64_t)pl.bytes});
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

// The surviving sizes the last count pass on this thread read, with the workspace and plan they
// belong to: the write pass that follows on the same thread plans from them without a second
// host read (the caller keeps ws and the inputs unchanged between the two).
struct SizesSeen {
    const char* ws;
    uint64_t stamp;
    uint32_t n[2];
};
static thread_local SizesSeen g_seen{nullptr, 0, {0, 0}};

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
    if (pl.semi) return hash_count(hash_plan(pl.nR, pl.nS, num_cus, -1, true), R, S, ws + pl.off_inner, st, nullptr, pub);
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
        auto compact = [&](const join_rel_t& X, const uint32_t* f, int logm, size_t off_k, size_t off_r,
                           uint32_t* total) -> hipError_t {
            int32_t* ok = reinterpret_cast<int32_t*>(ws + off_k);
            int32_t* orr = reinterpret_cast<int32_t*>(ws + off_r);
            if (!pl.ordered) {
                compact_k<<<(unsigned)pl.grid, kBlock, 0, st>>>(X.key, X.rid, X.n, f, logm, ok, orr, total);
                return hipGetLastError();
            }
            uint32_t* wc = reinterpret_cast<uint32_t*>(ws + pl.off_wcnt);
            const int64_t per = (X.n + pl.grid - 1) / pl.grid;
            compact_ordered_k<false><<<(unsigned)pl.grid, kBlock, 0, st>>>(X.key, X.rid, X.n, per, f, logm, wc,
                                                                          nullptr, nullptr);
            hipError_t r = hipGetLastError();
            if (r == hipSuccess)
                r = exclusive_scan<uint32_t>(wc, wc, pl.grid, total, reinterpret_cast<uint32_t*>(ws + pl.off_wtmp), st);
            if (r != hipSuccess) return r;
            compact_ordered_k<true><<<(unsigned)pl.grid, kBlock, 0, st>>>(X.key, X.rid, X.n, per, f, logm, wc, ok, orr);
            return hipGetLastError();
        };
        if (pl.logS) e = compact(R, fS, pl.logS, pl.off_kR, pl.off_rR, cnt);
        if (e == hipSuccess && pl.logR) e = compact(S, fR, pl.logR, pl.off_kS, pl.off_rS, cnt + 1);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t n[2] = {0, 0};
    if (pl.logR || pl.logS) {
        e = read_sizes(pl, ws, st, n);
        if (e != hipSuccess) return e;
    }
    g_seen = SizesSeen{ws, pl.stamp, {n[0], n[1]}};
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
    if (pl.semi)
        return hash_write(hash_plan(pl.nR, pl.nS, num_cus, -1, true), R, S, ws + pl.off_inner, pairs, cap, st);
    uint32_t n[2] = {0, 0};
    if (g_seen.ws == ws && g_seen.stamp == pl.stamp) {
        n[0] = g_seen.n[0];
        n[1] = g_seen.n[1];
    } else if (pl.logR || pl.logS) {
        hipError_t e = read_sizes(pl, ws, st, n);
        if (e != hipSuccess) return e;
    }
    join_rel_t R2, S2;
    survivors(pl, ws, n, R, S, &R2, &S2);
    if (R2.n == 0 || S2.n == 0) return hipSuccess;
    return hash_write(hash_plan(R2.n, S2.n, num_cus), R2, S2, ws + pl.off_inner, pairs, cap, st);
}

}  // namespace jl
