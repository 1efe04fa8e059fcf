// hash.hip -- partitioned hash equi join on gfx950: histogram, scatter, unit planning, and the
// LDS hash-table count and write passes.
//
// The paper's hash join (Section 3.3.2) hashes the smaller table T into fixed-size buckets and
// lets each thread probe a contiguous range of the larger table S (equations NBSJ / IDSJ); its
// MapReduce round first groups tuples by join_key / alpha so that each reducer joins one key
// range (Algorithm 1, Map2 / Reduce2).  The gfx950 design keeps that shape but moves it on chip:
//   1. histogram:   per chunk of input, LDS histogram of pid = hash(key) >> (32 - bits); each
//                   chunk reserves its range inside every partition with one global atomic;
//   2. scan:        exclusive scan of the partition sizes -> partition starts;
//   3. scatter:     per tile, LDS-atomic ranks, the tile sorted by partition in LDS, and
//                   (hash, rid) tuples written partition-major in runs of consecutive
//                   addresses;
//   4. plan:        per partition, work units = (R chunk that fits the LDS table) x (S slice);
//   5. count pass:  per unit, build an LDS hash table from the R chunk and probe the S slice;
//   6. scan:        per-unit counts -> exact output offsets and the total (Section 3.3.3,
//                   computed exactly instead of estimated);
//   7. write pass:  same units, re-probe, each match written inside the unit's output range at
//                   a slot fixed by the count pass's per-wave totals and a wave-wide scan.
// The LDS table is 4-slot buckets with two candidate buckets per key; a lookup reads both with
// predicated compares, so a wave issues its LDS reads together and does not branch per key.
#include "hash.hpp"
#include "debug.hpp"

#include <type_traits>
#include <vector>

#include "prof.hpp"
#include "scan.hpp"
#include "tune.hpp"

namespace jl {

namespace {

constexpr int kHistBlock = 1024;
constexpr int kScatBlock = 1024;
#ifndef JL_SCAT_IT
#define JL_SCAT_IT 16
#endif
constexpr int kScatIt = JL_SCAT_IT;              // tuples per thread per scatter tile (multiple of 4)
constexpr int kScatTile = kScatBlock * kScatIt;  // tuples per scatter tile (sorted in LDS)
constexpr int kChunkAlign = 4 * kScatBlock;      // scatter chunks: whole 16-byte loads per thread
constexpr int kGroups = 8;                       // chunk groups (XCDs) writing through shared cursors
constexpr int64_t kBatchChunk = 65536;           // rows per histogram / scatter item of a batch
constexpr int kJoinBlock = 1024;  // threads of a count or write workgroup of one join
constexpr int kBatchBlock = 512;  // ... of a batch of joins, with tables of at most kBatchCap
constexpr int kBuildItems = 10;   // R chunk entries per thread: cap <= block * kBuildItems
constexpr int kMaxBits = 11;     // scatter: two partitions per thread; 2^11 x 8 B of LDS state
constexpr int kMaxCap = 9728;    // R chunk entries: the write pass's table (15 B an entry) and queue fit 160 KB
// Batches: 512-thread workgroups with tables of up to 4608 entries, so that two write workgroups
// (four count workgroups) share a CU and one's table build overlaps another's probes.
constexpr int kBatchCap = 4608;
static_assert(kBatchCap <= kBatchBlock * kBuildItems, "a batch chunk fits its workgroup's registers");

// Stores of the join's output pairs, which nothing here reads again: optionally non-temporal.
#ifndef JL_NT_PAIRS
#define JL_NT_PAIRS 1
#endif
__device__ __forceinline__ void put(int2* p, int2 v) { *p = v; }
// A pair pointer in the global address space.  A function that is not inlined receives its
// pointer arguments as generic (flat) pointers, and a flat store also counts against the LDS
// wait counter, so every LDS wait after it would wait for the store to reach memory.
typedef __attribute__((address_space(1))) int2 global_int2;

template <typename P>
__device__ __forceinline__ void put_pair(P* p, int2 v)
{
#if JL_NT_PAIRS
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
#else
    *p = v;
#endif
}

__device__ __forceinline__ uint32_t pid_of(int32_t key, int sh)
{
    return sh >= 32 ? 0u : hmix((uint32_t)key) >> sh;
}

__global__ void zero_u32_k(uint32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------------------------------------------- histogram --
// Work items of the histogram and scatter kernels: one chunk of one relation side of one join.
// A single join derives its items from the block index; a batch of joins reads them from a table.
// The second side of a single join, launched together with the first so that one launch covers
// both: workgroups from `split` on take its chunks.  split = the grid size when the launch has
// one side only.
struct SideTwo {
    SideItem one;
    int64_t chunk, n;
    uint32_t* tot;  // histogram: its partition sizes
    uint32_t* grp;  // histogram: its group shares; scatter: its group cursors
    int2* out;      // scatter: its partitioned tuples
    uint32_t* cnt;  // its per-tile counts (histogram), then its run offsets (scatter)
    uint32_t split;
};

// Tiles of a chunk of `len` rows (the scatter sorts one tile at a time; the histogram counts
// each tile separately, so that every run of a tile gets a position of its own).
__host__ __device__ __forceinline__ int64_t tiles_of(int64_t len) { return (len + kScatTile - 1) / kScatTile; }

__device__ __forceinline__ SideItem side_item(const SideItem* __restrict__ items, const SideItem& one,
                                              int64_t chunk, int64_t n, uint32_t blk)
{
    if (items) {
        // scalar loads: the item is the same for the whole workgroup
        const cptr<SideItem> p = as_const(items) + blk;
        SideItem it;
        it.key = p->key;
        it.rid = p->rid;
        it.beg = p->beg;
        it.len = p->len;
        it.bits = p->bits;
        it.part0 = p->part0;
        it.cnt0 = p->cnt0;
        return it;
    }
    SideItem it = one;
    it.beg = (int64_t)blk * chunk;
    const int64_t left = n - it.beg;
    it.len = (uint32_t)(left < chunk ? left : chunk);
    it.cnt0 = ((uint64_t)blk * (uint64_t)tiles_of(chunk)) << it.bits;
    return it;
}

__device__ __forceinline__ bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Chunks are grouped by their workgroup index modulo kGroups, which on this chip is the XCD the
// workgroup runs on: a group's chunks write each partition through one shared cursor (see the
// scatter), so the partially written 64-byte granules of a partition stay in one XCD's L2.
// A chunk counts its tuples per partition in LDS, then adds the counts to tot[part0 + p] (the
// partition's size) and grp[g * stride + part0 + p] (its group's share of the partition).
__device__ __forceinline__ uint32_t group_of_block() { return blockIdx.x % kGroups; }

// Per tile of kScatTile rows of the chunk (the scatter's tiles), the count of every partition
// goes to the tile's row of the side's count array; the chunk's totals then go to the partition
// sizes and to the chunk group's shares with one global atomic each.
__global__ __launch_bounds__(kHistBlock) void hist_k(const SideItem* __restrict__ items, SideItem one,
                                                     int64_t chunk, int64_t n, uint32_t* tot,
                                                     uint32_t* grp, uint32_t stride, uint32_t* cnt,
                                                     SideTwo two)
{
    extern __shared__ uint32_t h[];
    constexpr int V = 4;  // 16-byte loads in flight per thread: one full tile
    static_assert(V * 4 * kHistBlock == kScatTile, "a full tile is one round of loads");
    const bool second = blockIdx.x >= two.split;
    const SideItem it = second ? side_item(nullptr, two.one, two.chunk, two.n, blockIdx.x - two.split)
                               : side_item(items, one, chunk, n, blockIdx.x);
    if (second) {
        tot = two.tot;
        grp = two.grp;
        cnt = two.cnt;
    }
    const int P = 1 << it.bits;
    const int sh = 32 - it.bits;
    for (int i = threadIdx.x; i < P; i += kHistBlock) h[i] = 0;
    uint32_t own[2] = {0u, 0u};  // chunk totals of partitions tid and tid + kHistBlock
    __syncthreads();
    const gptr<int32_t> key = as_global(it.key + it.beg);
    const bool vec = aligned16(it.key + it.beg);
    const int64_t end = it.len;
    // ordered scatter (cnt != NULL): one row per tile; else the chunk is counted as one span
    const int64_t span = cnt ? (int64_t)kScatTile : (end > 0 ? end : 1);
    uint32_t* __restrict__ row = cnt ? cnt + it.cnt0 : nullptr;
    for (int64_t t0 = 0; t0 < end; t0 += span) {
        const int64_t tn = end - t0 < span ? end - t0 : span;
        if (!cnt && vec) {
            int64_t i = 0;
            for (; i + kScatTile <= tn; i += kScatTile) {
                i32x4 k4[V];
#pragma unroll
                for (int v = 0; v < V; ++v) k4[v] = load4(key + t0 + i + v * 4 * kHistBlock + 4 * threadIdx.x);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    atomicAdd(&h[pid_of(k4[v].x, sh)], 1u);
                    atomicAdd(&h[pid_of(k4[v].y, sh)], 1u);
                    atomicAdd(&h[pid_of(k4[v].z, sh)], 1u);
                    atomicAdd(&h[pid_of(k4[v].w, sh)], 1u);
                }
            }
            for (i += threadIdx.x; i < tn; i += kHistBlock) atomicAdd(&h[pid_of(key[t0 + i], sh)], 1u);
        } else if (vec && tn == kScatTile) {
            i32x4 k4[V];
#pragma unroll
            for (int v = 0; v < V; ++v) k4[v] = load4(key + t0 + v * 4 * kHistBlock + 4 * threadIdx.x);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                atomicAdd(&h[pid_of(k4[v].x, sh)], 1u);
                atomicAdd(&h[pid_of(k4[v].y, sh)], 1u);
                atomicAdd(&h[pid_of(k4[v].z, sh)], 1u);
                atomicAdd(&h[pid_of(k4[v].w, sh)], 1u);
            }
        } else {
            for (int64_t i = threadIdx.x; i < tn; i += kHistBlock) atomicAdd(&h[pid_of(key[t0 + i], sh)], 1u);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int p = (int)threadIdx.x + j * kHistBlock;
            if (p < P) {
                const uint32_t v = h[p];
                if (row) row[p] = v;
                own[j] += v;
                h[p] = 0;
            }
        }
        __syncthreads();
        if (row) row += P;
    }
    uint32_t* __restrict__ gs = grp + (size_t)group_of_block() * stride + it.part0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int p = (int)threadIdx.x + j * kHistBlock;
        if (p < P && own[j]) {
            atomicAdd(&tot[it.part0 + p], own[j]);
            atomicAdd(&gs[p], own[j]);
        }
    }
}

// Run offsets.  The runs a group's chunks write into partition p follow each other by tile
// index, then by chunk index: tile t of every chunk of the group, then tile t + 1, and so on.
// The group's workgroups work on about the same tile at the same time, so the runs written at
// about the same time lie next to each other and the 64-byte granules they share are completed
// in that XCD's L2 soon after; and the layout depends on the input alone.  In place, every
// per-tile count becomes the offset of its run from the group's start in the partition.
// Single join: one workgroup per (group, block of 64 partitions) of a side; thread (tl, q) takes
// tiles t = tl, tl + 16, ... of partition p0 + q over the group's chunks c = g0, g0 + 8, ...
// (g0 = the first chunk whose workgroup index falls in group g).  Chunk c has tiles_of(len_c)
// tiles; rows past a chunk's last tile hold nothing.
struct BandSide {
    uint32_t* cnt;
    int64_t chunk, n, nCh;
    int bits;
    uint32_t blockBase;  // workgroup index of chunk 0 in the histogram and scatter launches
};

constexpr int kBandBlock = 1024;
constexpr int kBandQ = 64;                      // partitions per workgroup
constexpr int kBandT = kBandBlock / kBandQ;     // tiles per pass

__device__ void band_side(const BandSide& b, int g, int p0, uint32_t* lds)
{
    const int P = 1 << b.bits;
    const int q = (int)threadIdx.x % kBandQ, tl = (int)threadIdx.x / kBandQ;
    const int p = p0 + q;
    const int64_t T = tiles_of(b.chunk);
    const int64_t c0 = ((int64_t)g - (int64_t)(b.blockBase % kGroups) + kGroups) % kGroups;
    uint32_t carry = 0;  // runs of partition p in earlier tile passes (same in every tile lane)
    for (int64_t tb = 0; tb < T; tb += kBandT) {
        const int64_t t = tb + tl;
        uint32_t sum = 0;
        if (p < P && t < T)
            for (int64_t c = c0; c < b.nCh; c += kGroups) {
                const int64_t len = b.n - c * b.chunk < b.chunk ? b.n - c * b.chunk : b.chunk;
                if (t < tiles_of(len)) sum += b.cnt[((uint64_t)(c * T + t) << b.bits) + p];
            }
        lds[tl * kBandQ + q] = sum;
        __syncthreads();
        uint32_t run = carry, all = 0;
        for (int j = 0; j < kBandT; ++j) {
            const uint32_t v = lds[j * kBandQ + q];
            run += j < tl ? v : 0u;
            all += v;
        }
        __syncthreads();
        if (p < P && t < T)
            for (int64_t c = c0; c < b.nCh; c += kGroups) {
                const int64_t len = b.n - c * b.chunk < b.chunk ? b.n - c * b.chunk : b.chunk;
                if (t < tiles_of(len)) {
                    uint32_t* x = &b.cnt[((uint64_t)(c * T + t) << b.bits) + p];
                    const uint32_t v = *x;
                    *x = run;
                    run += v;
                }
            }
        carry += all;
    }
}

// Batch: one thread per (partition of any join, group) of a side.  A join's chunks are the items
// [item0[j], item0[j + 1]) of the side; item i runs in workgroup i, so its group is i mod 8.
__global__ void band_batch_k(const SideItem* __restrict__ items, const uint32_t* __restrict__ item0,
                             const uint32_t* __restrict__ jpart0, int nJobs, uint32_t nParts,
                             uint32_t* __restrict__ cnt)
{
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (uint64_t)nParts * kGroups) return;
    const uint32_t gp = (uint32_t)(x / kGroups);
    const int g = (int)(x % kGroups);
    int lo = 0, hi = nJobs - 1;  // last job whose first partition is <= gp
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jpart0[mid] <= gp) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t p = gp - jpart0[lo];
    const uint32_t i0 = item0[lo], i1 = item0[lo + 1];
    const uint32_t f = i0 + (uint32_t)((g - (int)(i0 % kGroups) + kGroups) % kGroups);
    uint32_t run = 0;
    for (int64_t t = 0; t < tiles_of(kBatchChunk); ++t)
        for (uint32_t i = f; i < i1; i += kGroups) {
            const SideItem& it = items[i];
            if (t < tiles_of(it.len)) {
                uint32_t* c = &cnt[it.cnt0 + ((uint64_t)t << it.bits) + p];
                const uint32_t v = *c;
                *c = run;
                run += v;
            }
        }
}

// Group shares -> group cursors: the groups' ranges follow each other inside every partition,
// cur[g * stride + p] = base[p] + shares of groups before g.  In place.
__global__ void group_cursors_k(uint32_t* __restrict__ grp, const uint32_t* __restrict__ base,
                                uint32_t stride, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t run = base[p];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const uint32_t c = grp[(size_t)g * stride + p];
        grp[(size_t)g * stride + p] = run;
        run += c;
    }
}

// --------------------------------------------------------------------------------- scatter --
// Partitioned tuples are written as 8-byte (hmix(key), rid) pairs, partition-major.  Two costs
// decide a scatter with 2^11 partitions: memory requests (a store instruction whose 64 lanes
// write 64 partitions makes 64 of them), and 64-byte granules written in part (each is a
// read-modify-write in HBM unless the rest of the granule reaches the L2 while the line is
// still there).  Per tile of kScatTile tuples:
//   1. each wave counts its tuples per partition (LDS atomics on the wave's own counters);
//   2. per partition: the tile's share, its start in the sorted tile (block scan) and each
//      wave's start inside it, and the shift from sorted to output position: the run's output
//      start is the group's start in the partition plus the run offset the band scan computed;
//   3. each tuple takes the next position of its wave in its partition (an LDS atomic on the
//      wave's own counter, so positions follow the waves in order, and inside a wave the lanes
//      of one instruction in order, then the instructions in order): the tile is sorted by
//      partition, and the order depends on the input alone;
//   4. the sorted tile goes through LDS in two halves and is written by consecutive lanes taking
//      consecutive positions, so a store instruction covers runs of about kScatTile / 2^bits
//      tuples and touches a few granules instead of 64.
// Thread t handles partitions 2t and 2t + 1 in the per-partition steps.
// Element of thread tid, item 4v + c: tile position 4 * (v * kScatBlock + tid) + c, so every
// 16-byte load instruction of a wave reads 1 KB of consecutive input.
__device__ __forceinline__ int scat_pos(int q) { return 4 * ((q >> 2) * kScatBlock + (int)threadIdx.x) + (q & 3); }

// Loads of a tile's keys or rids: FULL tiles read whole 16-byte vectors; a partial tile (a
// chunk's last) reads the vectors that lie inside it when the column is 16-byte aligned (vec),
// and the rest element by element.
template <bool FULL>
__device__ __forceinline__ void scat_load(gptr<int32_t> col, int t0, int tn, int32_t (&x)[kScatIt],
                                          bool vec = true)
{
#pragma unroll
    for (int v = 0; v < kScatIt / 4; ++v) {
        const int e = scat_pos(4 * v);
        if (FULL || (vec && e + 4 <= tn)) {
            const i32x4 x4 = load4(col + t0 + e);
            x[4 * v] = x4.x; x[4 * v + 1] = x4.y; x[4 * v + 2] = x4.z; x[4 * v + 3] = x4.w;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) x[4 * v + c] = e + c < tn ? col[t0 + e + c] : 0;
        }
    }
}

// ---- the arrival-order scatter (default) ----
// Each tile's runs go to its chunk group's cursor in every partition (one global atomic per
// partition and tile): consecutive runs of a partition come from the group's chunks in the order
// they arrive, so the granule a run leaves incomplete is completed by the next run of the same
// group soon after, in the same XCD's L2.  The order of a partition's tuples depends on that
// arrival order (and, inside a tile, on the order of the LDS atomics of different waves).
struct ScatLdsA {
    int2* stg;      // [kScatTile] the tile sorted by partition
    uint32_t* cnt;  // [P] tile shares, then sorted starts
    uint32_t* dlt;  // [P] output position - sorted position
    uint32_t* tmp;  // scan scratch
};

// One tile: k holds raw keys (hashed here), r the row ids (RIDS) or nothing (row id = pos0 + tile
// position).  cur: this group's cursors of the join's partitions.
template <bool RIDS, bool FULL>
__device__ __forceinline__ void scat_tile_a(int32_t (&k)[kScatIt], const int32_t (&r)[kScatIt], int tn,
                                          int64_t pos0, int P, int sh, const ScatLdsA& L,
                                          uint32_t* __restrict__ cur, int2* __restrict__ out)
{
    const int tid = threadIdx.x;
    const int pa = 2 * tid, pb = 2 * tid + 1;
    // 1. shares.  Tuples are written as (hmix(key), rid): the hash is a bijection of the key, so
    // the join kernels compare hashes and never hash again.
#pragma unroll
    for (int q = 0; q < kScatIt; ++q) {
        const uint32_t h = hmix((uint32_t)k[q]);
        k[q] = (int32_t)h;
        if (FULL || scat_pos(q) < tn) atomicAdd(&L.cnt[sh >= 32 ? 0u : h >> sh], 1u);
    }
    __syncthreads();
    // 2. output positions from the group cursors; sorted starts (cnt becomes each partition's
    // placing cursor)
    const uint32_t ca = pa < P ? L.cnt[pa] : 0u, cb = pb < P ? L.cnt[pb] : 0u;
    uint32_t oa = 0, ob = 0;
    if (ca) oa = atomicAdd(&cur[pa], ca);
    if (cb) ob = atomicAdd(&cur[pb], cb);
    uint32_t tot;
    const uint32_t sa = block_excl_scan<kScatBlock>(ca + cb, L.tmp, &tot);
    if (pa < P) L.cnt[pa] = sa;
    if (pb < P) L.cnt[pb] = sa + ca;
    __syncthreads();
    // 3. place in sorted order: each tuple takes the next slot of its partition
#pragma unroll
    for (int q = 0; q < kScatIt; ++q) {
        const int e = scat_pos(q);
        if (FULL || e < tn) {
            const uint32_t h = (uint32_t)k[q];
            const uint32_t at = atomicAdd(&L.cnt[sh >= 32 ? 0u : h >> sh], 1u);
            L.stg[at] = make_int2(k[q], RIDS ? r[q] : (int32_t)(pos0 + e));
        }
    }
    // shift from sorted position to output position
    if (pa < P) L.dlt[pa] = oa - sa;
    if (pb < P) L.dlt[pb] = ob - (sa + ca);
    __syncthreads();
    if (pa < P) L.cnt[pa] = 0;  // the next tile's shares (nothing reads the cursors any more)
    if (pb < P) L.cnt[pb] = 0;
    // 4. write the sorted tile, eight LDS reads in flight at a time
    constexpr int G = 8;
#pragma unroll
    for (int g = 0; g < kScatIt; g += G) {
        int2 v[G];
        uint32_t d[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = (g + u) * kScatBlock + tid;
            v[u] = (FULL || i < tn) ? L.stg[i] : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const uint32_t h = (uint32_t)v[u].x;
            d[u] = L.dlt[sh >= 32 ? 0u : h >> sh];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = (g + u) * kScatBlock + tid;
            if (FULL || i < tn) put(&out[d[u] + (uint32_t)i], v[u]);
        }
    }
    __syncthreads();
}

// Full tile t of a chunk: the next tile's keys and rids are loaded into nk, nr while this one is
// worked on, before this tile's stores, so that waiting for them does not wait for the stores
// (the vector memory counter counts loads and stores in one queue).
template <bool RIDS>
__device__ __forceinline__ void scat_full_tile_a(int t, int nfull, gptr<int32_t> key, gptr<int32_t> rid,
                                               int32_t (&nk)[kScatIt], int32_t (&nr)[kScatIt],
                                               int64_t beg, int P, int sh, const ScatLdsA& L,
                                               uint32_t* __restrict__ cur, int2* __restrict__ out)
{
    int32_t k[kScatIt], r[kScatIt];
#pragma unroll
    for (int q = 0; q < kScatIt; ++q) {
        k[q] = nk[q];
        if (RIDS) r[q] = nr[q];
    }
    if (t + 1 < nfull) {
        scat_load<true>(key, (t + 1) * kScatTile, kScatTile, nk);
        if (RIDS) scat_load<true>(rid, (t + 1) * kScatTile, kScatTile, nr);
    }
    scat_tile_a<RIDS, true>(k, r, kScatTile, beg + (int64_t)t * kScatTile, P, sh, L, cur, out);
}

// A chunk: its full tiles, then the partial rest.  The first full tile is peeled off the loop,
// so that every pass through the loop starts in the same state (the loads it needs issued before
// the previous tile's stores) and waiting for those loads does not wait for the stores.
template <bool RIDS>
__device__ __forceinline__ void scat_chunk_a(gptr<int32_t> key, gptr<int32_t> rid, bool vec, int end,
                                           int64_t beg, int P, int sh, const ScatLdsA& L,
                                           uint32_t* __restrict__ cur, int2* __restrict__ out)
{
    const int nfull = vec ? end / kScatTile : 0;
    int32_t nk[kScatIt], nr[kScatIt];
    if (nfull > 0) {
        scat_load<true>(key, 0, kScatTile, nk);
        if (RIDS) scat_load<true>(rid, 0, kScatTile, nr);
        scat_full_tile_a<RIDS>(0, nfull, key, rid, nk, nr, beg, P, sh, L, cur, out);
    }
    for (int t = 1; t < nfull; ++t)
        scat_full_tile_a<RIDS>(t, nfull, key, rid, nk, nr, beg, P, sh, L, cur, out);
    for (int t0 = nfull * kScatTile; t0 < end; t0 += kScatTile) {
        const int tn = end - t0 < kScatTile ? end - t0 : kScatTile;
        int32_t k[kScatIt], r[kScatIt];
        scat_load<false>(key, t0, tn, k, vec);
        if (RIDS) scat_load<false>(rid, t0, tn, r, vec);
        scat_tile_a<RIDS, false>(k, r, tn, beg + t0, P, sh, L, cur, out);
    }
}

// ---- the ordered scatter (plan option hash.deterministic) ----
constexpr int kScatWaves = kScatBlock / kWave;
constexpr int kScatHalf = kScatTile / 2;  // tuples of one half of the sorted tile
static_assert(kScatTile <= 65536, "per-wave positions are 16-bit");

struct ScatLds {
    int2* stg;      // [kScatHalf] one half of the tile, sorted by partition
    uint32_t* wc;   // [kScatWaves / 2][P] per-wave counters: wave w in half (w & 1) of row w / 2
    uint32_t* dlt;  // [P] output position - sorted position
    uint32_t* tmp;  // scan scratch
};

// Where the runs of a chunk's tiles go: the group's start in each of the thread's two
// partitions, and the band scan's run offsets of the current tile.
struct ScatDest {
    uint32_t ga, gb;  // group starts of partitions 2t, 2t + 1
    uint32_t oa, ob;  // run offsets in them of the tile being worked on
};

// One tile: k holds raw keys (hashed here), r the row ids (RIDS) or nothing (row id = pos0 + tile
// position).
template <bool RIDS, bool FULL>
__device__ __forceinline__ void scat_tile(int32_t (&k)[kScatIt], const int32_t (&r)[kScatIt], int tn,
                                          int64_t pos0, int P, int sh, const ScatLds& L,
                                          const ScatDest& d, int2* __restrict__ out)
{
    const int tid = threadIdx.x;
    const int pa = 2 * tid, pb = 2 * tid + 1;
    const int wv = tid / kWave;
    const uint32_t wsh = 16u * (uint32_t)(wv & 1);
    uint32_t* __restrict__ wrow = L.wc + (size_t)(wv >> 1) * P;
    // 1. the wave's shares.  Tuples are written as (hmix(key), rid): the hash is a bijection of
    // the key, so the join kernels compare hashes and never hash again.
#pragma unroll
    for (int q = 0; q < kScatIt; ++q) {
        const uint32_t h = hmix((uint32_t)k[q]);
        k[q] = (int32_t)h;
        if (FULL || scat_pos(q) < tn) atomicAdd(&wrow[sh >= 32 ? 0u : h >> sh], 1u << wsh);
    }
    __syncthreads();
    // 2. tile shares, sorted starts, per-wave starts, shifts
    uint32_t wa[kScatWaves / 2], wb[kScatWaves / 2], ca = 0, cb = 0;
#pragma unroll
    for (int j = 0; j < kScatWaves / 2; ++j) {
        wa[j] = pa < P ? L.wc[(size_t)j * P + pa] : 0u;
        wb[j] = pb < P ? L.wc[(size_t)j * P + pb] : 0u;
        ca += (wa[j] & 0xFFFFu) + (wa[j] >> 16);
        cb += (wb[j] & 0xFFFFu) + (wb[j] >> 16);
    }
    uint32_t tot;
    const uint32_t sa = block_excl_scan<kScatBlock>(ca + cb, L.tmp, &tot);
    uint32_t run = sa;
#pragma unroll
    for (int j = 0; j < kScatWaves / 2; ++j) {
        const uint32_t lo = wa[j] & 0xFFFFu;
        if (pa < P) L.wc[(size_t)j * P + pa] = run | ((run + lo) << 16);
        run += lo + (wa[j] >> 16);
    }
#pragma unroll
    for (int j = 0; j < kScatWaves / 2; ++j) {
        const uint32_t lo = wb[j] & 0xFFFFu;
        if (pb < P) L.wc[(size_t)j * P + pb] = run | ((run + lo) << 16);
        run += lo + (wb[j] >> 16);
    }
    if (pa < P) L.dlt[pa] = d.ga + d.oa - sa;
    if (pb < P) L.dlt[pb] = d.gb + d.ob - (sa + ca);
    __syncthreads();
    // 3. positions in the sorted tile
    uint32_t at[kScatIt];
#pragma unroll
    for (int q = 0; q < kScatIt; ++q) {
        at[q] = ~0u;
        if (FULL || scat_pos(q) < tn) {
            const uint32_t h = (uint32_t)k[q];
            const uint32_t old = atomicAdd(&wrow[sh >= 32 ? 0u : h >> sh], 1u << wsh);
            at[q] = (old >> wsh) & 0xFFFFu;
        }
    }
    // 4. the sorted tile, half by half: placed in LDS, then written by consecutive lanes, eight
    // LDS reads in flight at a time
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int q = 0; q < kScatIt; ++q)
            if (at[q] - (uint32_t)(half * kScatHalf) < (uint32_t)kScatHalf)
                L.stg[at[q] - half * kScatHalf] = make_int2(k[q], RIDS ? r[q] : (int32_t)(pos0 + scat_pos(q)));
        __syncthreads();
        if (half == 0) {  // every position is taken: the next tile's counters start from zero
#pragma unroll
            for (int j = 0; j < kScatWaves / 2; ++j) {
                if (pa < P) L.wc[(size_t)j * P + pa] = 0;
                if (pb < P) L.wc[(size_t)j * P + pb] = 0;
            }
        }
        constexpr int G = 8;
#pragma unroll
        for (int g = 0; g < kScatIt / 2; g += G) {
            int2 v[G];
            uint32_t o[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int i = (g + u) * kScatBlock + tid;
                v[u] = (FULL || half * kScatHalf + i < tn) ? L.stg[i] : make_int2(0, 0);
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const uint32_t h = (uint32_t)v[u].x;
                o[u] = L.dlt[sh >= 32 ? 0u : h >> sh];
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int i = (g + u) * kScatBlock + tid;
                if (FULL || half * kScatHalf + i < tn) put(&out[o[u] + (uint32_t)(half * kScatHalf + i)], v[u]);
            }
        }
        __syncthreads();
    }
}

// The run offsets of tile t of the chunk in the thread's two partitions.
__device__ __forceinline__ void scat_offsets(const uint32_t* __restrict__ cnt0, int t, int P,
                                             uint32_t& oa, uint32_t& ob)
{
    const int pa = 2 * (int)threadIdx.x, pb = pa + 1;
    const uint32_t* row = cnt0 + (size_t)t * P;
    oa = pa < P ? row[pa] : 0u;
    ob = pb < P ? row[pb] : 0u;
}

// Full tile t of a chunk: the next tile's keys, rids and run offsets are loaded into nk, nr, nd
// while this one is worked on, before this tile's stores, so that waiting for them does not wait
// for the stores (the vector memory counter counts loads and stores in one queue).
template <bool RIDS>
__device__ __forceinline__ void scat_full_tile(int t, int nfull, gptr<int32_t> key, gptr<int32_t> rid,
                                               int32_t (&nk)[kScatIt], int32_t (&nr)[kScatIt],
                                               ScatDest& nd, const uint32_t* __restrict__ cnt0,
                                               int64_t beg, int P, int sh, const ScatLds& L,
                                               int2* __restrict__ out)
{
    int32_t k[kScatIt], r[kScatIt];
#pragma unroll
    for (int q = 0; q < kScatIt; ++q) {
        k[q] = nk[q];
        if (RIDS) r[q] = nr[q];
    }
    const ScatDest d = nd;
    if (t + 1 < nfull) {
        scat_offsets(cnt0, t + 1, P, nd.oa, nd.ob);
        scat_load<true>(key, (t + 1) * kScatTile, kScatTile, nk);
        if (RIDS) scat_load<true>(rid, (t + 1) * kScatTile, kScatTile, nr);
    }
    scat_tile<RIDS, true>(k, r, kScatTile, beg + (int64_t)t * kScatTile, P, sh, L, d, out);
}

// A chunk: its full tiles, then the partial rest.  The first full tile is peeled off the loop,
// so that every pass through the loop starts in the same state (the loads it needs issued before
// the previous tile's stores) and waiting for those loads does not wait for the stores.
template <bool RIDS>
__device__ __forceinline__ void scat_chunk(gptr<int32_t> key, gptr<int32_t> rid, bool vec, int end,
                                           int64_t beg, int P, int sh, const ScatLds& L,
                                           ScatDest d, const uint32_t* __restrict__ cnt0,
                                           int2* __restrict__ out)
{
    const int nfull = vec ? end / kScatTile : 0;
    int32_t nk[kScatIt], nr[kScatIt];
    if (nfull > 0) {
        scat_offsets(cnt0, 0, P, d.oa, d.ob);
        scat_load<true>(key, 0, kScatTile, nk);
        if (RIDS) scat_load<true>(rid, 0, kScatTile, nr);
        scat_full_tile<RIDS>(0, nfull, key, rid, nk, nr, d, cnt0, beg, P, sh, L, out);
    }
    for (int t = 1; t < nfull; ++t)
        scat_full_tile<RIDS>(t, nfull, key, rid, nk, nr, d, cnt0, beg, P, sh, L, out);
    for (int t0 = nfull * kScatTile; t0 < end; t0 += kScatTile) {
        const int tn = end - t0 < kScatTile ? end - t0 : kScatTile;
        int32_t k[kScatIt], r[kScatIt];
        scat_offsets(cnt0, t0 / kScatTile, P, d.oa, d.ob);
        scat_load<false>(key, t0, tn, k, vec);
        if (RIDS) scat_load<false>(rid, t0, tn, r, vec);
        scat_tile<RIDS, false>(k, r, tn, beg + t0, P, sh, L, d, out);
    }
}

// ------------------------------------------------------------------------------- planning --
// Per partition: its ranges in the partitioned tuples and its work units.  In a batch the
// partition's join (and so its fan-out) is found by binary search over the joins' first
// partitions jpart0[0..nJobs]; a single join passes jpart0 = NULL and its own fan-out.
// The plan of partition p: its PartInfo and its number of units.
struct PartPlan {
    const uint32_t* baseR;
    const uint32_t* totR;
    const uint32_t* baseS;
    const uint32_t* totS;
    const uint32_t* jpart0;
    const int32_t* jbits;
    int nJobs, bits;
    uint32_t cap, slice;
};

__device__ __forceinline__ uint32_t plan_part(const PartPlan& q, int p, PartInfo& pi)
{
    int bits = q.bits;
    if (q.jpart0) {
        int lo = 0, hi = q.nJobs - 1;  // last job whose first partition is <= p
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (q.jpart0[mid] <= (uint32_t)p) lo = mid;
            else hi = mid - 1;
        }
        bits = q.jbits[lo];
    }
    const uint32_t nr = q.totR[p], ns = q.totS[p];
    const uint32_t nrc = (nr + q.cap - 1) / q.cap;
    uint32_t nss = 0;
    if (nr > 0 && ns > 0) {
        // rounded, not ceiled: a partition a little over the slice stays one slice (an S slice
        // costs a table build, and partitions of a uniform S sit around the mean)
        const uint64_t per = (uint64_t)q.slice * nrc;
        nss = (uint32_t)((ns + per / 2) / per);
        if (nss < 1) nss = 1;
    }
    pi.rStart = q.baseR[p];
    pi.nR = nr;
    pi.sStart = q.baseS[p];
    pi.nS = ns;
    pi.nSs = nss;
    pi.nRc = nrc;
    pi.bits = (uint32_t)bits;
    pi.pad = 0;
    return nrc * nss;
}

// Work unit `local` of a partition (R chunk local / nSs, S slice local % nSs) as one record:
// {first R tuple, R tuples | fan-out << 24, first S tuple, S tuples}.  The planning kernels
// write every unit's record, so the join kernels read a unit with one 16-byte load.
// Bit kRecShared of the second word: the partition has several R chunks, so several units probe
// the same S slice.  Bit kRecOrder: set by the count pass when some probe of the unit has more
// than kEmitSort matches (the write pass then puts the table in canonical order).
constexpr int kRecBitsShift = 24;
constexpr int kRecShared = 28;
constexpr int kRecOrder = 29;
__host__ __device__ __forceinline__ uint4 unit_rec(const PartInfo& pi, uint32_t local, uint32_t cap)
{
    const uint32_t rc = local / pi.nSs;
    const uint32_t sc = local - rc * pi.nSs;
    const uint32_t slen = (pi.nS + pi.nSs - 1) / pi.nSs;
    const uint32_t rN = min(cap, pi.nR - rc * cap);
    const uint32_t sN = sc * slen < pi.nS ? min(slen, pi.nS - sc * slen) : 0u;
    return make_uint4(pi.rStart + rc * cap,
                      rN | (pi.bits << kRecBitsShift) | ((pi.nRc > 1 ? 1u : 0u) << kRecShared),
                      pi.sStart + sc * slen, sN);
}

__global__ void plan_units_k(PartPlan q, int nParts, PartInfo* __restrict__ info,
                             uint32_t* __restrict__ units)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > nParts) return;
    if (p == nParts) {
        units[nParts] = 0;
        return;
    }
    PartInfo pi;
    units[p] = plan_part(q, p, pi);
    info[p] = pi;
}

// Unit -> partition map: partition p owns units [unitStart[p], unitStart[p + 1]).
__global__ void expand_units_k(const uint32_t* __restrict__ unitStart, const PartInfo* __restrict__ info,
                               int P, uint32_t cap, int64_t Umax, uint4* __restrict__ urec)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const PartInfo pi = info[p];
    for (uint32_t u = unitStart[p]; u < unitStart[p + 1] && (int64_t)u < Umax; ++u)
        urec[u] = unit_rec(pi, u - unitStart[p], cap);
}

// One workgroup for up to kFuseParts partitions, in place of several launches of a few
// microseconds each.  part_starts_k: each side's partition starts (exclusive scan of the sizes)
// and group cursors; a NULL tot skips that side.  plan_k: the plans, the units' exclusive scan
// (unitStart[0..nParts], the total also at *Utotal) and the unit -> partition map.
// part_starts_k runs one workgroup per side.
constexpr int kFuseBlock = 1024;
constexpr int kFuseParts = 8192;

__device__ __forceinline__ void group_cursors(uint32_t* __restrict__ grp, uint32_t stride, int p, uint32_t run)
{
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const uint32_t c = grp[(size_t)g * stride + p];
        grp[(size_t)g * stride + p] = run;
        run += c;
    }
}

// Band work of a single join: 8 groups x ceil(P / kBandQ) partition blocks per side with counts
// (cnt != NULL).
__host__ __device__ __forceinline__ int64_t band_blocks(const BandSide& b)
{
    return b.cnt ? (int64_t)kGroups * (((1 << b.bits) + kBandQ - 1) / kBandQ) : 0;
}

// Workgroups 0 and 1: each side's partition starts and group starts (a NULL tot skips that
// side).  Workgroups from 2 on: the run offsets of R's tiles, then of S's (band_side).
__global__ __launch_bounds__(kFuseBlock) void part_starts_k(const uint32_t* __restrict__ totR,
                                                            uint32_t* __restrict__ baseR,
                                                            uint32_t* __restrict__ grpR,
                                                            const uint32_t* __restrict__ totS,
                                                            uint32_t* __restrict__ baseS,
                                                            uint32_t* __restrict__ grpS,
                                                            uint32_t stride, int n, BandSide bR,
                                                            BandSide bS)
{
    static_assert(kFuseBlock == kBandBlock, "one launch shape for both kinds of workgroup");
    __shared__ uint32_t tmp[kBandBlock];
    if (blockIdx.x >= 2) {
        int64_t k = blockIdx.x - 2;
        const bool s = k >= band_blocks(bR);
        if (s) k -= band_blocks(bR);
        const BandSide& b = s ? bS : bR;
        const int64_t nq = ((1 << b.bits) + kBandQ - 1) / kBandQ;
        band_side(b, (int)(k / nq), (int)(k % nq) * kBandQ, tmp);
        return;
    }
    {
        const int side = blockIdx.x;  // workgroup 0: R, workgroup 1: S
        const uint32_t* tot = side ? totS : totR;
        uint32_t* base = side ? baseS : baseR;
        uint32_t* grp = side ? grpS : grpR;
        if (!tot) return;
        uint32_t carry = 0;
        for (int b0 = 0; b0 < n; b0 += 2 * kFuseBlock) {
            const int pa = b0 + 2 * (int)threadIdx.x, pb = pa + 1;
            const uint32_t ca = pa < n ? tot[pa] : 0u, cb = pb < n ? tot[pb] : 0u;
            uint32_t t;
            const uint32_t sa = carry + block_excl_scan<kFuseBlock>(ca + cb, tmp, &t);
            if (pa < n) {
                base[pa] = sa;
                group_cursors(grp, stride, pa, sa);
            }
            if (pb < n) {
                base[pb] = sa + ca;
                group_cursors(grp, stride, pb, sa + ca);
            }
            carry += t;
        }
    }
}

// The plans of all partitions by one workgroup of BLOCK threads, two partitions per thread and
// pass; tmp: BLOCK / 64 + 1 words of LDS.
template <int BLOCK>
__device__ void plan_block(const PartPlan& q, int nParts, PartInfo* __restrict__ info,
                           uint32_t* __restrict__ unitStart, uint32_t* __restrict__ Utotal,
                           int64_t Umax, uint4* __restrict__ urec, uint32_t* tmp)
{
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nParts; b0 += 2 * BLOCK) {
        const int pa = b0 + 2 * (int)threadIdx.x, pb = pa + 1;
        PartInfo ia{}, ib{};
        const uint32_t ua = pa < nParts ? plan_part(q, pa, ia) : 0u;
        const uint32_t ub = pb < nParts ? plan_part(q, pb, ib) : 0u;
        uint32_t t;
        const uint32_t sa = carry + block_excl_scan<BLOCK>(ua + ub, tmp, &t);
        if (pa < nParts) {
            info[pa] = ia;
            unitStart[pa] = sa;
            for (uint32_t u = sa; u < sa + ua && (int64_t)u < Umax; ++u) urec[u] = unit_rec(ia, u - sa, q.cap);
        }
        if (pb < nParts) {
            info[pb] = ib;
            unitStart[pb] = sa + ua;
            for (uint32_t u = sa + ua; u < sa + ua + ub && (int64_t)u < Umax; ++u)
                urec[u] = unit_rec(ib, u - sa - ua, q.cap);
        }
        carry += t;
    }
    if (threadIdx.x == 0) {
        unitStart[nParts] = carry;
        *Utotal = carry;
    }
}

__global__ __launch_bounds__(kFuseBlock) void plan_k(PartPlan q, int nParts, PartInfo* __restrict__ info,
                                                     uint32_t* __restrict__ unitStart,
                                                     uint32_t* __restrict__ Utotal, int64_t Umax,
                                                     uint4* __restrict__ urec)
{
    __shared__ uint32_t tmp[kFuseBlock / kWave + 1];
    plan_block<kFuseBlock>(q, nParts, info, unitStart, Utotal, Umax, urec, tmp);
}

// The per-partition plan can ride along with the scatter of a single join: with pa.info set, the
// last workgroup computes it (the partition starts it reads come from the launch before).
struct PlanArgs {
    PartPlan q;
    int nParts;
    PartInfo* info;
    uint32_t* units;
    uint32_t* Utotal;
    int64_t Umax;
    uint4* urec;
};

// RIDS: the side has a rid column (a batch passes RIDS and may still leave it NULL per item;
// without rids the row ids are positions).  cur: the groups' starts in every partition,
// [kGroups][stride]; cnt: the side's run offsets (band scan).
// ORDERED: the ordered scatter (runs at the band scan's offsets, ranks from per-wave counters),
// else the arrival-order one (runs at the group cursors).
template <bool RIDS, bool ORDERED>
__global__ __launch_bounds__(kScatBlock) void scatter_k(const SideItem* __restrict__ items, SideItem one,
                                                        int64_t chunk, int64_t n, uint32_t* cur,
                                                        uint32_t stride, int2* out,
                                                        const uint32_t* cnt, SideTwo two, PlanArgs pa)
{
    extern __shared__ uint32_t lds[];
    // The chunk of workgroup b is the one the histogram counted in workgroup b: its group shares
    // were counted under the same group, so the plan's workgroup comes after every chunk.
    const uint32_t blk = blockIdx.x;
    if (pa.info && blk == gridDim.x - 1) {
        plan_block<kScatBlock>(pa.q, pa.nParts, pa.info, pa.units, pa.Utotal, pa.Umax, pa.urec, lds);
        return;
    }
    const bool second = blk >= two.split;
    const SideItem it = second ? side_item(nullptr, two.one, two.chunk, two.n, blk - two.split)
                               : side_item(items, one, chunk, n, blk);
    if (second) {
        cur = two.grp;
        out = two.out;
        cnt = two.cnt;
    }
    const int P = 1 << it.bits;
    const int sh = 32 - it.bits;
    const int tid = threadIdx.x;
    if constexpr (!ORDERED) {
        ScatLdsA L;
        L.stg = reinterpret_cast<int2*>(lds);
        L.cnt = lds + 2 * kScatTile;
        L.dlt = L.cnt + P;
        L.tmp = L.dlt + P;
        if (2 * tid < P) L.cnt[2 * tid] = 0;
        if (2 * tid + 1 < P) L.cnt[2 * tid + 1] = 0;
        __syncthreads();
        uint32_t* __restrict__ gc = cur + (size_t)group_of_block() * stride + it.part0;
        const gptr<int32_t> key = as_global(it.key + it.beg);
        const bool kvec = aligned16(it.key + it.beg);
        if (!RIDS || it.rid == nullptr) {
            scat_chunk_a<false>(key, nullptr, kvec, (int)it.len, it.beg, P, sh, L, gc, out);
        } else {
            const bool vec = kvec && aligned16(it.rid + it.beg);
            scat_chunk_a<true>(key, as_global(it.rid + it.beg), vec, (int)it.len, it.beg, P, sh, L, gc, out);
        }
        return;
    }
    ScatLds L;
    L.stg = reinterpret_cast<int2*>(lds);
    L.wc = lds + 2 * kScatHalf;
    L.dlt = L.wc + (size_t)(kScatWaves / 2) * P;
    L.tmp = L.dlt + P;
    for (int i = tid; i < (kScatWaves / 2) * P; i += kScatBlock) L.wc[i] = 0;
    __syncthreads();
    const uint32_t* __restrict__ gc = cur + (size_t)group_of_block() * stride + it.part0;
    ScatDest d{};
    d.ga = 2 * tid < P ? gc[2 * tid] : 0u;
    d.gb = 2 * tid + 1 < P ? gc[2 * tid + 1] : 0u;
    const uint32_t* __restrict__ c0 = cnt + it.cnt0;
    const gptr<int32_t> key = as_global(it.key + it.beg);
    const bool kvec = aligned16(it.key + it.beg);
    if (!RIDS || it.rid == nullptr) {
        scat_chunk<false>(key, nullptr, kvec, (int)it.len, it.beg, P, sh, L, d, c0, out);
    } else {
        const bool vec = kvec && aligned16(it.rid + it.beg);
        scat_chunk<true>(key, as_global(it.rid + it.beg), vec, (int)it.len, it.beg, P, sh, L, d, c0, out);
    }
}

// ------------------------------------------------------------------------- join work units --
struct Unit {
    uint32_t rBeg, rN, sBeg, sN;
    int bits;     // fan-out of the unit's join: the table position uses the hash bits below it
    bool shared;  // other units (other R chunks) probe the same S slice
    bool order;   // partitioned joins, after the count pass: the table needs canonical order
};

__device__ __forceinline__ Unit unit_of(uint4 r)
{
    Unit o;
    o.rBeg = r.x;
    o.rN = r.y & ((1u << kRecBitsShift) - 1);
    o.sBeg = r.z;
    o.sN = r.w;
    o.bits = (int)((r.y >> kRecBitsShift) & ((1u << (kRecShared - kRecBitsShift)) - 1));
    o.shared = ((r.y >> kRecShared) & 1u) != 0;
    o.order = ((r.y >> kRecOrder) & 1u) != 0;
    return o;
}

// Unit u.  PART: a partitioned join (the kernels' AOS instances), whose plan wrote every unit's
// record; otherwise the single partition's units are computed.
template <bool PART>
__device__ __forceinline__ Unit decode_unit(const JoinGeom& g, uint32_t u)
{
    if constexpr (PART) return unit_of(g.urec[u]);
    else return unit_of(unit_rec(g.one, u, g.cap));
}

// Whether two units hash the same chunk (the write pass keeps a table across such units).
__device__ __forceinline__ bool same_chunk(const Unit& a, const Unit& b)
{
    return a.rBeg == b.rBeg && a.rN == b.rN;
}

// ------------------------------------------------------------------------ the LDS table --
// Fixed-size buckets of 4 slots, like the paper's hash buckets with a short search inside the
// bucket (Section 3.3.2).  Bucket b holds 4 keys (one 16-byte LDS read), the 4 matching rids
// (another) and a claim counter; min(claims, 4) slots are filled.  Each key has two candidate
// buckets b1 != b2 from independent bits of its hash.  An insert claims a slot (LDS atomic add)
// in the less loaded of the two, then in the other; a claim past the 4th slot fails.  If both
// fail it walks on from b2 + 1, claiming bucket by bucket.  So every bucket an insert failed in
// ends with more than 4 claims, and a lookup reads b1 and b2 and walks on from b2 + 1 only when
// both hold more than 4 claims, stopping after the first bucket with at most 4.  At load 0.6 the
// two choices keep that walk to about 2 lookups in 10^4, so a lookup is two bucket reads with
// predicated compares.  No empty marker is needed: every int32 key and rid value stays usable.
constexpr int kSlots = 4;
#ifndef JL_HASH_PROBE
#define JL_HASH_PROBE 2
#endif
constexpr int kProbe = JL_HASH_PROBE;  // keys probed together per thread
constexpr int kEmitSort = 8;  // a probe with at most this many matches orders them in registers

__host__ __device__ constexpr uint32_t table_buckets(uint32_t rN)
{
    const uint32_t nb = (rN * 5 + 11) / 12;  // 4 * nb * 0.6 >= rN
    return nb < 2 ? 2u : nb;                 // two distinct candidates need two buckets
}

__device__ __forceinline__ uint32_t next_bucket(uint32_t b, uint32_t nb) { return b + 1 == nb ? 0 : b + 1; }

// The two candidate buckets of hash h.  The partition id took the top `bits` bits of h, so b1
// comes from the bits below it and b2 from a multiplicative remix of all of h.
// (bits <= kMaxBits < 32.)
__device__ __forceinline__ void choices(uint32_t h, int bits, uint32_t nb, uint32_t& b1, uint32_t& b2)
{
    b1 = __umulhi(h << bits, nb);
    b2 = __umulhi(h * 0x9E3779B1u, nb);
    b2 = b2 == b1 ? next_bucket(b1, nb) : b2;
}

// Marked tables.  A partitioned unit with a fan-out of at least 2 bits holds only hashes whose
// two top bits are the partition's.  Its empty slots then hold a marker whose top bit differs
// (no probe of the partition equals it), and a bucket that overflowed (more than 4 claims) has
// bit 30 of its fourth key flipped: lookups read only the two key vectors, with no claim
// counter, and recover the fourth key by comparing the other 31 bits.  Other units (the single
// path's raw keys, batch joins of fan-out 0 or 1) compare against the claim counters.
constexpr uint32_t kOverflow = 1u << 30;

struct Table {
    const uint4* keys;    // [nb]: the 4 keys of each bucket
    const uint4* rids;    // [nb]: their rids (write pass only)
    const uint32_t* cnt;  // [nb]: claims; min(cnt, 4) slots are filled
    uint32_t nb;
    bool marked;          // uniform
};

// LDS bytes of a table for chunks of up to `cap` entries: 16 bytes of keys per bucket, 16 of
// rids when the table keeps them (the count pass does not), and a 4-byte claim counter.
__host__ __device__ constexpr size_t table_lds(uint32_t cap, bool rids)
{
    return (size_t)table_buckets(cap) * (rids ? 36 : 20) + 64;
}

// One R chunk held in registers between its load and its insertion.
template <bool RIDS>
struct Chunk {
    uint32_t k[kBuildItems];
    uint32_t r[RIDS ? kBuildItems : 1];
};

// Issue every load of a chunk before any use (uniform guards only), so the chunk arrives in one
// memory round trip.  AOS: the chunk is partitioned (key, rid) tuples; otherwise it is a range
// of the input columns.
template <bool AOS, bool RIDS, int B>
__device__ __forceinline__ void load_chunk(const JoinGeom& g, const Unit& un, Chunk<RIDS>& c)
{
    const int tid = threadIdx.x;
    const uint32_t nIt = (un.rN + B - 1) / B;
#pragma unroll
    for (int i = 0; i < kBuildItems; ++i) {
        c.k[i] = 0u;
        if constexpr (RIDS) c.r[i] = 0u;
    }
    if (un.rN > 0) {  // every unit has rN >= 1; the guard keeps the clamped index in bounds
#pragma unroll
        for (int i = 0; i < kBuildItems; ++i) {
            const uint32_t e = (uint32_t)(i * B + tid);
            const uint32_t idx = un.rBeg + (e < un.rN ? e : un.rN - 1);
            if ((uint32_t)i < nIt) {
                if constexpr (AOS) {
                    const int2 t = g.rt[idx];
                    c.k[i] = (uint32_t)t.x;
                    if constexpr (RIDS) c.r[i] = (uint32_t)t.y;
                } else {
                    c.k[i] = (uint32_t)g.rk[idx];
                    if constexpr (RIDS) c.r[i] = g.rr ? (uint32_t)g.rr[idx] : idx;
                }
            }
        }
    }
}

// The table of a unit's R chunk in LDS (built by insert_chunk; the same for every unit of that
// chunk).
template <bool RIDS, bool HASHED>
__device__ __forceinline__ Table table_of(const Unit& un, uint4* lds)
{
    const uint32_t nb = table_buckets(un.rN);
    Table t;
    t.keys = lds;
    t.rids = RIDS ? lds + nb : nullptr;
    t.cnt = reinterpret_cast<const uint32_t*>(lds + (RIDS ? 2 : 1) * nb);
    t.nb = nb;
    t.marked = HASHED && un.bits >= 2;
    return t;
}

// Insert a loaded chunk into the LDS table (two barriers: cleared counters, finished table).
// HASHED: the chunk holds hmix(key) values (partitioned tuples), else raw keys.  pos[i]
// receives the LDS word position of item i's slot.
// Clears the table of unit un's chunk: claim counters to zero and, for a marked table, every key
// to the marker (top bit flipped, bit 30 as the partition's, so it never reads as overflowed);
// h: any hash of the partition (read only for a marked table).
template <bool RIDS, bool HASHED, int B>
__device__ __forceinline__ void clear_table(const Unit& un, uint32_t h, uint4* lds)
{
    const uint32_t nb = table_buckets(un.rN);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(lds + (RIDS ? 2 : 1) * nb);
    if (HASHED && un.bits >= 2) {
        const uint32_t m = (h ^ 0x80000000u) & 0xC0000000u;
        for (uint32_t b = threadIdx.x; b < nb; b += B) {
            cnt[b] = 0;
            lds[b] = make_uint4(m, m, m, m);
        }
    } else {
        for (uint32_t b = threadIdx.x; b < nb; b += B) cnt[b] = 0;
    }
}

// A hash of unit un's partition for its table's marker (a scalar load; only for marked tables).
template <bool HASHED>
__device__ __forceinline__ uint32_t marker_hash(const JoinGeom& g, const Unit& un)
{
    return HASHED && un.bits >= 2 ? (uint32_t)g.rt[un.rBeg].x : 0u;
}

template <bool RIDS, bool HASHED, int B, bool CLEARED = false>
__device__ __forceinline__ Table insert_chunk(const JoinGeom& g, const Unit& un, const Chunk<RIDS>& c,
                                              uint4* lds, uint32_t (&pos)[kBuildItems])
{
    const int tid = threadIdx.x;
    const uint32_t nb = table_buckets(un.rN);
    uint32_t* keys = reinterpret_cast<uint32_t*>(lds);
    uint32_t* rids = reinterpret_cast<uint32_t*>(lds + nb);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(lds + (RIDS ? 2 : 1) * nb);
    const bool marked = HASHED && un.bits >= 2;
    if constexpr (!CLEARED) {  // else the caller cleared the table and passed a barrier since
        // The write pass loaded its chunk a unit ahead, and every thread's first entry is a hash
        // of the partition (lanes past the chunk hold its last one).
        clear_table<RIDS, HASHED, B>(un, RIDS ? c.k[0] : marker_hash<HASHED>(g, un), lds);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kBuildItems; ++i) {
        const uint32_t e = (uint32_t)(i * B + tid);
        if (e < un.rN) {
            uint32_t b1, b2;
            choices(HASHED ? c.k[i] : hmix(c.k[i]), un.bits, nb, b1, b2);
            const bool second = cnt[b2] < cnt[b1];  // a racy read only steers the choice
            uint32_t b = second ? b2 : b1;
            uint32_t old = atomicAdd(&cnt[b], 1u);
            if (old >= (uint32_t)kSlots) {
                b = second ? b1 : b2;
                old = atomicAdd(&cnt[b], 1u);
                if (old >= (uint32_t)kSlots) {
                    b = b2;
                    do {  // ends: 4 * nb slots > rN entries
                        b = next_bucket(b, nb);
                        old = atomicAdd(&cnt[b], 1u);
                    } while (old >= (uint32_t)kSlots);
                }
            }
            keys[b * kSlots + old] = c.k[i];
            if constexpr (RIDS) rids[b * kSlots + old] = c.r[i];
            pos[i] = b * kSlots + old;
        }
    }
    __syncthreads();
    if (marked) {  // flag the overflowed buckets, now that every slot is written
        for (uint32_t b = tid; b < nb; b += B)
            if (cnt[b] > (uint32_t)kSlots) keys[b * kSlots + 3] ^= kOverflow;
        __syncthreads();
    }
    return table_of<RIDS, HASHED>(un, lds);
}

// Matches of x among the filled slots of one bucket, as a 4-bit mask (claim-counter tables).
__device__ __forceinline__ uint32_t bucket_hits(const uint4& k, uint32_t c, uint32_t x)
{
    return (uint32_t)(k.x == x && c > 0) | ((uint32_t)(k.y == x && c > 1) << 1) |
           ((uint32_t)(k.z == x && c > 2) << 2) | ((uint32_t)(k.w == x && c > 3) << 3);
}

// The lookup primitives, for marked tables (MARKED) or claim-counter ones; callers choose the
// variant once per unit, by a uniform branch around the whole probe.
// A bucket's claim counter, read only for tables that are not marked.
template <bool MARKED>
__device__ __forceinline__ uint32_t claims(const Table& t, uint32_t b)
{
    if constexpr (MARKED) return 0u;
    else return t.cnt[b];
}

// Matches of x in a bucket (k its keys, c its claims when not marked), as a 4-bit mask.
template <bool MARKED>
__device__ __forceinline__ uint32_t hits(const uint4& k, uint32_t c, uint32_t x)
{
    if constexpr (MARKED)
        return (uint32_t)(k.x == x) | ((uint32_t)(k.y == x) << 1) | ((uint32_t)(k.z == x) << 2) |
               ((uint32_t)(((k.w ^ x) & ~kOverflow) == 0u) << 3);
    else return bucket_hits(k, c, x);
}

// The number of matches of x in a bucket (the popcount of hits), as a sum of comparisons.
template <bool MARKED>
__device__ __forceinline__ uint32_t hit_count(const uint4& k, uint32_t c, uint32_t x)
{
    if constexpr (MARKED)
        return (uint32_t)(k.x == x) + (uint32_t)(k.y == x) + (uint32_t)(k.z == x) +
               (uint32_t)(((k.w ^ x) & ~kOverflow) == 0u);
    else
        return (uint32_t)(k.x == x && c > 0) + (uint32_t)(k.y == x && c > 1) + (uint32_t)(k.z == x && c > 2) +
               (uint32_t)(k.w == x && c > 3);
}

// Whether a bucket holds more than 4 claims, so that lookups go on past it.  In a marked table x
// (a hash of the partition) tells the fourth key's true bit 30.
template <bool MARKED>
__device__ __forceinline__ bool overflowed(const uint4& k, uint32_t c, uint32_t x)
{
    if constexpr (MARKED) return ((k.w ^ x) & 0xC0000000u) == kOverflow;
    else return c > (uint32_t)kSlots;
}

// The walk past b1 and b2 (rare): buckets from b2 + 1 while the previous one overflowed.  A walk
// that wraps onto b1 or b2 skips their slots, which were already counted.
template <bool MARKED, typename Visit>
__device__ __forceinline__ void walk_on(const Table& t, uint32_t x, uint32_t b1, uint32_t b2, Visit visit)
{
    uint32_t b = b2;
    while (true) {
        b = next_bucket(b, t.nb);
        const uint32_t c = claims<MARKED>(t, b);
        const uint4 k = t.keys[b];
        if (b != b1 && b != b2) visit(b, hits<MARKED>(k, c, x));
        if (!overflowed<MARKED>(k, c, x)) break;
    }
}

// Count the entries of N keys: read both candidate buckets of every key (all reads issued
// together), count the matching slots with predicated arithmetic, and walk on only for keys
// whose two buckets both overflowed.  `multi` is set when a key has more than kEmitSort
// entries (the write pass then puts the table's entries in canonical order before it emits
// them; keys with fewer entries are ordered as they are emitted); `many` adds up the entries
// of keys with more than two (the write pass places their pairs apart).
template <int N, bool HASHED, bool MARKED, bool FULL>
__device__ __forceinline__ uint32_t probe_count(const Table& t, int bits, const uint32_t (&x)[N],
                                                const bool (&valid_in)[N], bool& multi, uint32_t& many,
                                                uint32_t (&hout)[N])
{
    bool valid[N];
#pragma unroll
    for (int i = 0; i < N; ++i) valid[i] = FULL || valid_in[i];  // FULL: every key is in range
    uint32_t b1[N], b2[N], c1[N], c2[N];
    uint4 k1[N], k2[N];
#pragma unroll
    for (int i = 0; i < N; ++i) choices(HASHED ? x[i] : hmix(x[i]), bits, t.nb, b1[i], b2[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        k1[i] = t.keys[b1[i]];
        c1[i] = claims<MARKED>(t, b1[i]);
        k2[i] = t.keys[b2[i]];
        c2[i] = claims<MARKED>(t, b2[i]);
    }
    uint32_t n = 0, h[N];
    bool walk[N], any = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        h[i] = hit_count<MARKED>(k1[i], c1[i], x[i]) + hit_count<MARKED>(k2[i], c2[i], x[i]);
        if (!FULL) h[i] = valid[i] ? h[i] : 0u;
        walk[i] = valid[i] && overflowed<MARKED>(k1[i], c1[i], x[i]) && overflowed<MARKED>(k2[i], c2[i], x[i]);
        any = any || walk[i];
    }
    if (ballot(any)) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (walk[i])
                walk_on<MARKED>(t, x[i], b1[i], b2[i], [&](uint32_t, uint32_t hm) { h[i] += __builtin_popcount(hm); });
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        n += h[i];
        many += h[i] > 2 ? h[i] : 0u;
        multi = multi || h[i] > (uint32_t)kEmitSort;
        hout[i] = h[i];
    }
    return n;
}

// Probe N keys for the write pass: per key the number of entries and the LDS word positions of
// the first two, whose rids are read once the output slots are known (a key with more than two
// build matches visits its buckets again when it is written).
template <int N, bool HASHED, bool MARKED>
__device__ __forceinline__ void probe_write(const Table& t, int bits, const uint32_t (&x)[N],
                                            const bool (&valid)[N], uint32_t (&m)[N],
                                            uint32_t (&p1)[N], uint32_t (&p2)[N])
{
    uint32_t b1[N], b2[N], c1[N], c2[N];
    uint4 k1[N], k2[N];
#pragma unroll
    for (int i = 0; i < N; ++i) choices(HASHED ? x[i] : hmix(x[i]), bits, t.nb, b1[i], b2[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        k1[i] = t.keys[b1[i]];
        c1[i] = claims<MARKED>(t, b1[i]);
        k2[i] = t.keys[b2[i]];
        c2[i] = claims<MARKED>(t, b2[i]);
    }
    bool walk[N], any = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint32_t h1 = valid[i] ? hits<MARKED>(k1[i], c1[i], x[i]) : 0u;
        const uint32_t h2 = valid[i] ? hits<MARKED>(k2[i], c2[i], x[i]) : 0u;
        // slots of the two buckets as one 8-bit mask: bit j < 4 is b1's slot j, bit 4 + j b2's
        const uint32_t hm = h1 | (h2 << 4);
        const uint32_t j1 = __builtin_ctz(hm | 256u), j2 = __builtin_ctz((hm & (hm - 1)) | 256u);
        p1[i] = j1 < 4 ? b1[i] * kSlots + j1 : b2[i] * kSlots + (j1 & 3);
        p2[i] = j2 < 4 ? b1[i] * kSlots + j2 : b2[i] * kSlots + (j2 & 3);
        m[i] = __builtin_popcount(hm);
        walk[i] = valid[i] && overflowed<MARKED>(k1[i], c1[i], x[i]) && overflowed<MARKED>(k2[i], c2[i], x[i]);
        any = any || walk[i];
    }
    if (ballot(any)) {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (walk[i])
                walk_on<MARKED>(t, x[i], b1[i], b2[i], [&](uint32_t b, uint32_t hm) {
                    while (hm) {
                        const uint32_t p = b * kSlots + __builtin_ctz(hm);
                        p2[i] = m[i] == 1 ? p : p2[i];
                        p1[i] = m[i] == 0 ? p : p1[i];
                        ++m[i];
                        hm &= hm - 1;
                    }
                });
    }
}

// Every entry of key x in visiting order (b1's slots, b2's, then the walk), as LDS word
// positions; used for keys with more than two build matches.
template <bool HASHED, bool MARKED, typename F>
__device__ __forceinline__ void for_each_match(const Table& t, int bits, uint32_t x, F f)
{
    uint32_t b1, b2;
    choices(HASHED ? x : hmix(x), bits, t.nb, b1, b2);
    const uint32_t c1 = claims<MARKED>(t, b1), c2 = claims<MARKED>(t, b2);
    const uint4 k1 = t.keys[b1], k2 = t.keys[b2];
    auto emit = [&](uint32_t b, uint32_t hm) {
        for (; hm; hm &= hm - 1) f(b * kSlots + __builtin_ctz(hm));
    };
    emit(b1, hits<MARKED>(k1, c1, x));
    emit(b2, hits<MARKED>(k2, c2, x));
    if (overflowed<MARKED>(k1, c1, x) && overflowed<MARKED>(k2, c2, x)) walk_on<MARKED>(t, x, b1, b2, emit);
}

// Sorts 8 values ascending with the 19 compare-exchanges of Batcher's odd-even merge network.
__device__ __forceinline__ void sort8(uint32_t (&v)[8])
{
    constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2},
                                 {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4},
                                 {5, 6}};
#pragma unroll
    for (int c = 0; c < 19; ++c) {
        const uint32_t a = v[kNet[c][0]], b = v[kNet[c][1]];
        v[kNet[c][0]] = min(a, b);
        v[kNet[c][1]] = max(a, b);
    }
}

// The m pairs of probe x (m counted here), at slot .. slot + m - 1, in ascending build rid
// order (as signed int32).
//  * No walk (the two candidate buckets hold every match, so m <= 8): the 8 slots' rids are
//    read at once and sorted by a network, as unsigned keys rid ^ 2^31, the slots that do not
//    match set to all ones; the first m are written.  A matching rid of INT32_MAX has the same
//    key as a slot that does not match, and both turn back into INT32_MAX, so the first m
//    values are the matches in order either way.
//  * A walk with up to kEmitSort matches (rare): gathered in registers, each written at its rank.
//  * More: the table was put in canonical order, so the visiting order is ascending.
template <bool HASHED, bool MARKED, typename P>
__device__ __forceinline__ void emit_many(const Table& t, int bits, uint32_t x, int32_t srid,
                                          uint64_t slot, const uint32_t* rw,
                                          P* __restrict__ out, uint64_t cap)
{
    uint32_t b1, b2;
    choices(HASHED ? x : hmix(x), bits, t.nb, b1, b2);
    const uint4 k1 = t.keys[b1], k2 = t.keys[b2];
    const uint32_t c1 = claims<MARKED>(t, b1), c2 = claims<MARKED>(t, b2);
    if (!(overflowed<MARKED>(k1, c1, x) && overflowed<MARKED>(k2, c2, x))) {
        const uint32_t hm = hits<MARKED>(k1, c1, x) | (hits<MARKED>(k2, c2, x) << 4);
        const uint32_t m = __builtin_popcount(hm);
        const uint4 r1 = t.rids[b1], r2 = t.rids[b2];
        uint32_t v[8] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = ((hm >> j) & 1u) ? v[j] ^ 0x80000000u : ~0u;
        sort8(v);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((uint32_t)k < m && slot + k < cap)
                put_pair(&out[slot + k], make_int2((int32_t)(v[k] ^ 0x80000000u), srid));
        return;
    }
    uint32_t m = 0;
    for_each_match<HASHED, MARKED>(t, bits, x, [&](uint32_t) { ++m; });
    if (m > (uint32_t)kEmitSort) {
        uint32_t seen = 0;
        for_each_match<HASHED, MARKED>(t, bits, x, [&](uint32_t p) {
            if (slot + seen < cap) put_pair(&out[slot + seen], make_int2((int32_t)rw[p], srid));
            ++seen;
        });
        return;
    }
    int32_t r[kEmitSort];
    uint32_t seen = 0;
#pragma unroll
    for (int j = 0; j < kEmitSort; ++j) r[j] = 0;
    for_each_match<HASHED, MARKED>(t, bits, x, [&](uint32_t p) {
        const int32_t v = (int32_t)rw[p];
#pragma unroll
        for (int j = 0; j < kEmitSort; ++j) r[j] = seen == (uint32_t)j ? v : r[j];
        ++seen;
    });
#pragma unroll
    for (int k = 0; k < kEmitSort; ++k) {
        uint32_t rank = 0;
#pragma unroll
        for (int j = 0; j < kEmitSort; ++j)
            rank += ((uint32_t)j < m && (r[j] < r[k] || (r[j] == r[k] && j < k))) ? 1u : 0u;
        if ((uint32_t)k < m && slot + rank < cap) put_pair(&out[slot + rank], make_int2(r[k], srid));
    }
}

// Probes with more than two matches are rare (and scattered over the lanes): each wave queues
// them in LDS, {key, probe rid, matches}, and emits the queue with one probe per lane when the
// next tuple's probes would not fit (and at the end of the unit), instead of running emit_many
// with a few lanes active after every round.  Their pairs form one contiguous block per wave
// and unit, after the wave's other pairs, so each emission writes a contiguous run.  The
// emitting function is not inlined: its registers are needed only while it runs, not across
// the probe loop.
constexpr int kManyQ = 64;  // a whole wave's worth: one tuple index of a round always fits

// The write pass's LDS: its dynamic table, and the queues at file scope, so that the emitting
// function below, which is not inlined, still addresses them as LDS.
extern __shared__ uint4 write_lds[];
__shared__ uint4 write_manyq[kJoinBlock / kWave * kManyQ];       // 1024-thread workgroups
__shared__ uint4 write_manyq_b[kBatchBlock / kWave * kManyQ];    // 512-thread workgroups

// The queues of a B-thread workgroup (each kernel instance references one of the arrays only,
// so its static LDS holds that one).
template <int B>
__device__ __forceinline__ uint4* manyq()
{
    static_assert(B == kJoinBlock || B == kBatchBlock, "two workgroup sizes");
    if constexpr (B == kJoinBlock) return write_manyq;
    else return write_manyq_b;
}

// Emits the qn queued probes of wave wv (one per lane) against the table of a unit whose chunk
// has nb buckets (rids after the keys, claim counters after the rids): their pairs go, in queue
// order, to the contiguous block at `at`.  Returns the end of that block.
template <bool HASHED, bool MARKED, int B>
__device__ __attribute__((noinline)) uint64_t flush_many(uint32_t nb, int bits, int wv, uint32_t qn,
                                                         uint64_t at, int2* __restrict__ out, uint64_t cap)
{
    Table t;
    t.keys = write_lds;
    t.rids = write_lds + nb;
    t.cnt = reinterpret_cast<const uint32_t*>(write_lds + 2 * nb);
    t.nb = nb;
    t.marked = MARKED;
    const uint4* q = manyq<B>() + wv * kManyQ;
    // the queue was written by other lanes of this wave; LDS accesses of a wave complete in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool mine = lane_id() < qn;
    const uint4 e = mine ? q[lane_id()] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t inc = wave_incl_scan(e.z);  // e.z: the probe's matches (0 for no entry)
    const uint64_t total = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
    if (mine)
        emit_many<HASHED, MARKED>(t, bits, e.x, (int32_t)e.y, at + (inc - e.z),
                                  reinterpret_cast<const uint32_t*>(t.rids), (global_int2*)out, cap);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return at + total;
}

// Canonical order of a key's entries.  The inserts race for slots, so which slots a key's
// entries take, and the order in which a probe meets them, can differ between runs; the write
// pass emits the matches of every probe in ascending rid order (as signed int32; equal rids give
// equal pairs, so their order does not matter).  A probe with at most kEmitSort matches sorts
// them in registers as it writes them.  For a table in which some probe has more (the count
// pass records it per unit), the write pass first moves the rids of every key with two or more
// entries so that the key's visiting order (b1's slots, b2's, then the walk) meets them in
// ascending order: each entry finds its rank among its key's entries and the slot of that rank
// in the visiting order, and after a barrier stores its rid there.  Keys stay where they are.
template <bool HASHED, bool MARKED, int B>
__device__ void canonicalize(const Table& t, int bits, const Unit& un, const Chunk<true>& c,
                             const uint32_t (&pos)[kBuildItems], uint32_t* rids)
{
    uint32_t target[kBuildItems];
#pragma unroll
    for (int i = 0; i < kBuildItems; ++i) {
        target[i] = ~0u;
        const uint32_t e = (uint32_t)(i * B + threadIdx.x);
        if (e < un.rN) {
            const int32_t mine = (int32_t)c.r[i];
            uint32_t m = 0, rank = 0;
            bool self = false;
            for_each_match<HASHED, MARKED>(t, bits, c.k[i], [&](uint32_t p) {
                const int32_t r = (int32_t)rids[p];
                if (p == pos[i]) self = true;
                else if (r < mine || (r == mine && !self)) ++rank;
                ++m;
            });
            if (m >= 2) {
                uint32_t k = 0;
                for_each_match<HASHED, MARKED>(t, bits, c.k[i], [&](uint32_t p) {
                    if (k == rank) target[i] = p;
                    ++k;
                });
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kBuildItems; ++i)
        if (target[i] != ~0u && target[i] != pos[i]) rids[target[i]] = c.r[i];
    __syncthreads();
}

// Units of this join.  The device total never exceeds Umax (sum over partitions of
// nRc * nSs <= P + nR / cap + nS / slice); the clamp keeps the counts array in bounds even so.
__device__ __forceinline__ uint32_t unit_total(const JoinGeom& g)
{
    const uint32_t U = g.single ? g.Uhost : *g.Uptr;
    return (int64_t)U < g.Umax ? U : (uint32_t)g.Umax;
}

// A contiguous run [u0, u1) of the unit list per workgroup: the write pass's static share of one
// join.  Units of one partition follow each other R chunk by R chunk, S slice by S slice, so
// consecutive slices of one chunk keep its table (a skewed probe side cuts its hot partitions
// into many slices).  Batches of joins, whose units differ widely in size, and the count pass
// keep the round-robin order, which balances better.
__device__ __forceinline__ void unit_range(uint32_t U, uint32_t& u0, uint32_t& u1)
{
    u0 = (uint32_t)(((uint64_t)U * blockIdx.x) / gridDim.x);
    u1 = (uint32_t)(((uint64_t)U * (blockIdx.x + 1)) / gridDim.x);
}

// The sequence of units a workgroup of the count or write pass takes.  A fixed share per
// workgroup leaves CUs idle at the end of a batch's passes: its units differ widely in size, and
// of the count workgroups sharing a CU the older ones run ahead.  With a ticket counter (words
// of the workspace, zero before the pass; batches), each workgroup takes a static head, half of
// its even share in round-robin order, and then units handed out one at a time after all static
// heads, so that faster workgroups take more.  Without one (one join, whose units are even), the
// whole share is static: round robin, or for the write pass a contiguous run, whose consecutive
// units of one R chunk keep the table.  The unit two places ahead is fixed while a unit runs
// (its ticket taken at the unit's start, read back after the unit's last barrier), so the loads
// the passes issue ahead for the next unit never wait for a ticket.
constexpr uint32_t kTicketed = 0xFFFFFFFFu;

struct Sched {
    uint32_t U;         // units
    uint32_t head;      // static positions
    uint32_t base;      // contig: first unit of the static run
    uint32_t dyn0;      // the first unit handed out by ticket
    uint32_t pos;       // uniform: position of the current unit in this workgroup's sequence
    bool contig;
    uint32_t* ticket;   // NULL: static only

    // Unit at position k: a static one (U or more once the static share is used up and there
    // is no ticket), or kTicketed.
    __device__ __forceinline__ uint32_t at(uint32_t k) const
    {
        if (k >= head) return ticket ? kTicketed : U;
        return contig ? base + k : blockIdx.x + k * gridDim.x;
    }
};

__device__ __forceinline__ Sched make_sched(uint32_t U, bool contig, uint32_t* ticket)
{
    Sched s{};
    s.U = U;
    s.contig = contig;
    s.ticket = ticket;
    if (ticket) {
        const uint32_t h = U / gridDim.x / 2;
        s.head = h;
        s.base = blockIdx.x * h;
        s.dyn0 = gridDim.x * h;
    } else if (contig) {
        uint32_t u0, u1;
        unit_range(U, u0, u1);
        s.head = u1 - u0;
        s.base = u0;
    } else {
        s.head = 0xFFFFFFFFu;  // u = blockIdx.x + k * gridDim.x < U + 2 * gridDim.x: no wrap
    }
    return s;
}

// The first two units of the sequence (U or more: none).  slot: two words of LDS.
__device__ __forceinline__ void sched_start(const Sched& s, uint32_t& u, uint32_t& nxi, uint32_t* slot)
{
    u = s.at(0);
    nxi = s.at(1);
    if (u == kTicketed || nxi == kTicketed) {  // uniform
        if (threadIdx.x == 0) {
            if (u == kTicketed) slot[0] = s.dyn0 + atomicAdd(s.ticket, 1u);
            if (nxi == kTicketed) slot[1] = s.dyn0 + atomicAdd(s.ticket, 1u);
        }
        __syncthreads();
        if (u == kTicketed) u = uniform(slot[0]);
        if (nxi == kTicketed) nxi = uniform(slot[1]);
        __syncthreads();
    }
}

// At the start of the unit at s.pos, with the next one nxi: whether the unit after nxi comes
// from a ticket (then thread 0 takes it now).
__device__ __forceinline__ bool sched_need(const Sched& s, uint32_t nxi)
{
    return nxi < s.U && s.at(s.pos + 2) == kTicketed;
}

// Thread 0 publishes the ticket before the unit's last barrier; every thread reads the unit
// after nxi once past it.  The two LDS slots alternate by position, so a slot is written again
// only after a barrier that every reader of its previous value has passed.
__device__ __forceinline__ void sched_put(const Sched& s, bool need, uint32_t tk, uint32_t* slot)
{
    if (need && threadIdx.x == 0) slot[s.pos & 1] = s.dyn0 + tk;
}

__device__ __forceinline__ uint32_t sched_after(const Sched& s, bool need, uint32_t nxi, const uint32_t* slot)
{
    if (need) return uniform(slot[s.pos & 1]);
    return nxi < s.U ? s.at(s.pos + 2) : s.U;
}

#ifndef JL_HASH_COUNT_BATCH
#define JL_HASH_COUNT_BATCH 2
#endif
// The count kernel's keys-only table lets two 1024-thread workgroups (four of a batch's 512)
// share a CU, so it is compiled for 8 waves per SIMD (64 VGPRs); the write kernel for 4 (128
// VGPRs): one 1024-thread workgroup per CU, or two of a batch's.
#define JL_COUNT_ATTR(B) __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(8)))
#define JL_WRITE_ATTR(B) __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(4)))
constexpr int kCountBatch = JL_HASH_COUNT_BATCH;  // S keys in flight per thread in the count pass
static_assert(kCountBatch % kProbe == 0, "count batch is probed kProbe keys at a time");
#ifndef JL_HASH_WRITE_PROBE
#define JL_HASH_WRITE_PROBE 2
#endif
#ifndef JL_HASH_WRITE_LOAD
#define JL_HASH_WRITE_LOAD 4
#endif
constexpr int kWriteBatch = JL_HASH_WRITE_PROBE;  // S tuples per thread per round of the write pass
// S tuples per thread in flight in the write pass: 4 for one join's 1024-thread workgroups, 2 for
// a batch's 512-thread ones (two share a CU; with 4, a batch's units of about 3K probe rows
// left their second round mostly empty: batch write 22.5 -> 21.7 ms with 2).
template <int B>
constexpr int kWriteLoadOf = B == kBatchBlock ? 2 : JL_HASH_WRITE_LOAD;
static_assert(kWriteLoadOf<kJoinBlock> % kWriteBatch == 0 && kWriteLoadOf<kBatchBlock> % kWriteBatch == 0,
              "write loads are probed kWriteBatch tuples at a time");

template <bool AOS, int B>
__device__ __forceinline__ void load_tuples(const JoinGeom& g, const Unit& un, uint32_t e0,
                                            uint32_t (&x)[kWriteLoadOf<B>], int32_t (&r)[kWriteLoadOf<B>])
{
    const bool full = e0 + (uint32_t)(kWriteLoadOf<B> * B) <= un.sN;  // uniform
    if (un.sN == 0) {  // no tuple to stand in for the out-of-range lanes
#pragma unroll
        for (int i = 0; i < kWriteLoadOf<B>; ++i) x[i] = 0u, r[i] = 0;
        return;
    }
#pragma unroll
    for (int i = 0; i < kWriteLoadOf<B>; ++i) {
        const uint32_t e = e0 + i * B + threadIdx.x;
        const bool ok = full || e < un.sN;
        uint32_t idx = un.sBeg + (ok ? e : 0u);
        // computed where the load is issued: hoisted out of the probe loop, the addresses of the
        // next unit's first loads would occupy registers through it
        asm volatile("" : "+v"(idx));
        // no select on the loaded values: the probe masks the out-of-range lanes, and a select
        // here would wait for the loads
        if constexpr (AOS) {
            const int2 t = g.st[idx];
            x[i] = (uint32_t)t.x;
            r[i] = t.y;
        } else {
            x[i] = (uint32_t)g.sk[idx];
            r[i] = g.sr ? g.sr[idx] : (int32_t)idx;
        }
    }
}

// A batch of S keys of a unit with un.sN > 0.  Out-of-range lanes read the unit's first tuple and
// drop it (the probe masks them), so the loads carry no branch.
template <bool AOS, int B>
__device__ __forceinline__ void load_keys_of(const JoinGeom& g, const Unit& un, uint32_t e0,
                                             uint32_t (&xs)[kCountBatch])
{
    const bool full = e0 + (uint32_t)(kCountBatch * B) <= un.sN;  // uniform
#pragma unroll
    for (int i = 0; i < kCountBatch; ++i) {
        const uint32_t e = e0 + i * B + threadIdx.x;
        const bool ok = full || e < un.sN;
        const uint32_t idx = un.sBeg + (ok ? e : 0u);
        // no select on the loaded value: the probe masks the out-of-range lanes
        if constexpr (AOS) xs[i] = (uint32_t)g.st[idx].x;
        else xs[i] = (uint32_t)g.sk[idx];
    }
}

// The same for any unit: a unit without probes loads nothing.
template <bool AOS, int B>
__device__ __forceinline__ void load_keys(const JoinGeom& g, const Unit& un, uint32_t e0,
                                          uint32_t (&xs)[kCountBatch])
{
    if (un.sN == 0) {
#pragma unroll
        for (int i = 0; i < kCountBatch; ++i) xs[i] = 0u;
        return;
    }
    load_keys_of<AOS, B>(g, un, e0, xs);
}

// Count pass.  A workgroup walks the units of its sequence (Sched).  The S keys come in
// batches of kCountBatch per thread through two register buffers used in turn: while one batch
// is probed the next is in flight, and the next unit's first batch while the last one probes.
// Every half of the loop issues the same loads (a batch past the unit reloads a valid one), and
// the buffers swap roles instead of being copied, so the wait before a probe is for that
// batch's loads alone, never for the loads issued after them.
// A batch's matches fit 32 bits (kCountBatch keys of at most kMaxCap entries each); the lane's
// total over a unit is kept in 64 bits.
// The probe rows of a wave that have matches (the semi-join), recorded by the count pass when
// the write pass is to visit only them: the k-th such row of wave wv in a unit is stored, as its
// index in the partitioned probe tuples, at the place of the wave's k-th own row
// (unit start + (k / 64) * kJoinBlock + wv * 64 + k % 64), which lies inside the unit because
// the wave has at least k + 1 rows there.  A unit whose S slice other units also probe (its
// partition has several R chunks) records nothing (rows == NULL) and is written in full.
struct Semi {
    uint32_t* rows;  // [probe rows]
    uint32_t sBeg;   // the unit's first probe row
    uint32_t k;      // uniform: matching rows of this wave in the unit so far
};

__device__ __forceinline__ uint32_t semi_slot(uint32_t sBeg, uint32_t k, int wv)
{
    return sBeg + (k / kWave) * kJoinBlock + (uint32_t)wv * kWave + (k % kWave);
}

template <bool AOS, bool MARKED, bool FULL, bool SEMI, int B>
__device__ __forceinline__ uint32_t count_batch_of(const Table& t, const Unit& un, uint32_t e0,
                                                   const uint32_t (&xs)[kCountBatch], bool& multi,
                                                   uint32_t& many, Semi& sm)
{
    static_assert(!SEMI || B == kJoinBlock, "the semi-join record is laid out for 1024 threads");
    uint32_t cnt = 0;
#pragma unroll
    for (int h = 0; h < kCountBatch; h += kProbe) {
        uint32_t x[kProbe], hv[kProbe];
        bool ok[kProbe];
#pragma unroll
        for (int i = 0; i < kProbe; ++i) {
            x[i] = xs[h + i];
            ok[i] = e0 + (h + i) * B + threadIdx.x < un.sN;
        }
        cnt += probe_count<kProbe, AOS, MARKED, FULL>(t, un.bits, x, ok, multi, many, hv);
        if (SEMI && sm.rows) {  // uniform
            const int wv = (int)(threadIdx.x / kWave);
#pragma unroll
            for (int i = 0; i < kProbe; ++i) {
                const bool hit = hv[i] > 0;  // zero for rows past the unit
                const uint64_t bm = ballot(hit);
                if (hit) sm.rows[semi_slot(sm.sBeg, sm.k + mask_rank(bm), wv)] = un.sBeg + e0 + (h + i) * B + threadIdx.x;
                sm.k += (uint32_t)__builtin_popcountll(bm);
            }
        }
    }
    return cnt;
}

// A batch wholly inside the unit (the common case) probes without per-key range checks.
template <bool AOS, bool MARKED, bool SEMI, int B>
__device__ __forceinline__ uint32_t count_batch(const Table& t, const Unit& un, uint32_t e0,
                                                const uint32_t (&xs)[kCountBatch], bool& multi,
                                                uint32_t& many, Semi& sm)
{
    if (e0 + (uint32_t)(kCountBatch * B) <= un.sN)  // uniform
        return count_batch_of<AOS, MARKED, true, SEMI, B>(t, un, e0, xs, multi, many, sm);
    return count_batch_of<AOS, MARKED, false, SEMI, B>(t, un, e0, xs, multi, many, sm);
}

// Each wave of the count and write passes takes the same probe tuples of a unit: those at
// positions e with (e mod kJoinBlock) / 64 equal to its index.  The count pass records, per
// unit and wave, where the wave's pairs start inside the unit's output range, so the write pass
// needs no shared cursor and every pair lands at a position that depends on the input and the
// plan alone.  Entry 0 of a unit (wave 0 starts at 0) instead holds 1 when some probe of the
// unit has more than kEmitSort entries in its table.  Inside a wave's range the pairs of probes
// with at most two matches come first, in (batch, tuple, lane) order, then those of probes with
// more, in the order the wave queued them; the second half of the unit's record holds, per wave,
// where that second block starts inside the wave's range.
constexpr int kJoinWaves = kJoinBlock / kWave;
constexpr int kWaveRec = 2 * kJoinWaves;  // uint64 entries per unit in the wave record
constexpr int kWaveHalf = kJoinWaves;     // its second half (a 512-thread workgroup uses 8 + 8)
// the write pass's queues of probes with many matches, beside its dynamic table
constexpr size_t kWriteStaticLds = (size_t)kJoinWaves * kManyQ * 16;
constexpr size_t kBatchStaticLds = (size_t)(kBatchBlock / kWave) * kManyQ * 16;
static_assert(table_lds(kMaxCap, true) + kWriteStaticLds <= 160 * 1024, "write pass LDS");
static_assert(2 * (table_lds(kBatchCap, true) + kBatchStaticLds + 256) <= 160 * 1024,
              "two batch write workgroups per CU");

// End of a unit in the count pass: lane totals -> wave totals -> the unit's total in counts[u],
// the waves' starts in wave_off[u][1..kJoinWaves) and, in wave_off[u][kJoinWaves + w], each
// wave's count of pairs before its block of many-match pairs (low 32 bits: at most two pairs per
// probe row of the wave) and its count of probe rows with matches when the semi-join is recorded
// (high 32 bits, else 0); sh: kJoinWaves + 1 words of LDS.  rec_word (partitioned joins): the
// second word of the unit's record, which receives the canonical-order flag as well.  between:
// run by every thread after all waves have finished the unit, before the closing barrier.
template <int B, typename Between>
__device__ __forceinline__ void unit_totals(uint64_t lane_total, uint64_t lane_many, bool multi,
                                            uint32_t semi_rows, uint32_t u, uint64_t* __restrict__ counts,
                                            uint64_t* __restrict__ wave_off, uint64_t* sh, uint32_t* rec_word,
                                            Between between)
{
    const uint64_t wt = wave_sum64(lane_total);
    const uint64_t wmany = wave_sum64(lane_many);
    const bool wm = ballot(multi) != 0;
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) {
        sh[wv] = wt | (wm ? (1ull << 63) : 0ull);
        wave_off[(size_t)u * kWaveRec + kWaveHalf + wv] = (wt - wmany) | ((uint64_t)semi_rows << 32);
    }
    __syncthreads();
    if (threadIdx.x < (B / kWave)) {
        uint64_t before = 0, sum = 0, any = 0;
#pragma unroll
        for (int w = 0; w < (B / kWave); ++w) {
            const uint64_t v = sh[w];
            const uint64_t c = v & ~(1ull << 63);
            before += w < (int)threadIdx.x ? c : 0ull;
            sum += c;
            any |= v >> 63;
        }
        wave_off[(size_t)u * kWaveRec + threadIdx.x] = threadIdx.x == 0 ? any : before;
        if (threadIdx.x == 0) {
            counts[u] = sum;
            if (any && rec_word) atomicOr(rec_word, 1u << kRecOrder);
        }
    }
    between();  // every wave has finished the unit's probes
    __syncthreads();
}

// Up to kFuseScanMax units, the count kernel's last workgroup to finish also scans the counts,
// instead of a separate scan kernel after the count kernel.
constexpr int kFuseScanPer = 8;
constexpr int64_t kFuseScanMax = (int64_t)kJoinBlock * kFuseScanPer;

// Exclusive scan of counts[0, U) in place by one workgroup, kFuseScanPer consecutive counts per
// thread; entries U..Umax-1 are set to the sum, and *total receives it.  wsum: kJoinBlock / 64
// words of LDS.
template <int B>
__device__ void scan_counts_block(uint64_t* counts, uint32_t U, int64_t Umax, uint64_t* total,
                                  uint64_t* pub, uint64_t* wsum)
{
    const int64_t i0 = (int64_t)threadIdx.x * kFuseScanPer;
    uint64_t v[kFuseScanPer];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kFuseScanPer; ++k) {
        v[k] = i0 + k < (int64_t)U ? counts[i0 + k] : 0;
        s += v[k];
    }
    const uint64_t inc = wave_incl_scan64(s);
    const int wv = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[wv] = inc;
    __syncthreads();
    uint64_t run = inc - s, sum = 0;
#pragma unroll
    for (int w = 0; w < B / kWave; ++w) {
        const uint64_t t = wsum[w];
        run += w < wv ? t : 0;
        sum += t;
    }
#pragma unroll
    for (int k = 0; k < kFuseScanPer; ++k) {
        if (i0 + k < Umax) counts[i0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) {
        *total = sum;
        if (pub) publish_total(pub, sum);
    }
}

// done: NULL, or a zeroed arrival counter; then the last workgroup to arrive scans the counts
// (Umax <= kFuseScanMax) and writes the sum to *total and, when pub is not NULL, to that pinned
// host slot.
template <bool AOS, bool SEMI, int B>
__global__ JL_COUNT_ATTR(B) void join_count_k(JoinGeom g, uint64_t* __restrict__ counts,
                                           uint64_t* __restrict__ wave_off,
                                           uint32_t* __restrict__ done, uint64_t* __restrict__ total,
                                           uint64_t* pub)
{
    extern __shared__ uint4 tab[];
    __shared__ uint64_t wsum[B / kWave + 1];
    constexpr uint32_t kB = B * kCountBatch;  // keys per batch
    const uint32_t U = unit_total(g);
    if (g.stamp_at && blockIdx.x == 0 && threadIdx.x == 0) *g.stamp_at = g.stamp;  // for the write pass
    __shared__ uint32_t slot[2];
    Sched sc = make_sched(U, false, g.sched);
    uint32_t u, nxi;
    sched_start(sc, u, nxi, slot);
    uint32_t xa[kCountBatch], xb[kCountBatch];
    Unit un{};
    if (u < U) {
        un = decode_unit<AOS>(g, u);
        load_keys<AOS, B>(g, un, 0, xa);
        // each unit's table is cleared in the previous unit's closing step; the first one here
        clear_table<false, AOS, B>(un, marker_hash<AOS>(g, un), tab);
        __syncthreads();
    }
    while (u < U) {
        const bool need = sched_need(sc, nxi);
        uint32_t tk = 0;
        if (need && threadIdx.x == 0) tk = atomicAdd(sc.ticket, 1u);
        Chunk<false> ch;
        load_chunk<AOS, false, B>(g, un, ch);
        uint32_t pos[kBuildItems];
        const Table t = insert_chunk<false, AOS, B, true>(g, un, ch, tab, pos);
        __builtin_amdgcn_s_waitcnt(0);  // nothing in flight enters the batch loop
        const bool more = nxi < U;
        const Unit nx = more ? decode_unit<AOS>(g, nxi) : Unit{};
        uint64_t cnt = 0, many = 0;
        bool multi = false;
        Semi sm{SEMI && !un.shared ? g.semi : nullptr, un.sBeg, 0u};
        auto batches = [&](auto marked) {
            constexpr bool M = decltype(marked)::value;
            for (uint32_t e0 = 0; e0 < un.sN; e0 += 2 * kB) {
                const uint32_t e1 = e0 + kB, e2 = e1 + kB;
                uint32_t ma = 0, mb = 0;
                load_keys_of<AOS, B>(g, un, e1 < un.sN ? e1 : e0, xb);
                cnt += count_batch<AOS, M, SEMI, B>(t, un, e0, xa, multi, ma, sm);
                const bool here = e2 < un.sN, there = !here && more && nx.sN > 0;
                load_keys_of<AOS, B>(g, there ? nx : un, here ? e2 : (there ? 0u : e0), xa);
                cnt += count_batch<AOS, M, SEMI, B>(t, un, e1, xb, multi, mb, sm);  // every lane masked past the unit
                many += (uint64_t)ma + mb;
            }
        };
        if (AOS && t.marked) batches(std::true_type{});
        else batches(std::false_type{});
        if (un.sN == 0 && more) load_keys<AOS, B>(g, nx, 0, xa);
        sched_put(sc, need, tk, slot);
        // a partitioned join's record is read only by this workgroup in this pass (it decoded it
        // before), so the flag can go into it
        uint32_t* rec_word = AOS ? const_cast<uint32_t*>(&g.urec[u].y) : nullptr;
        // The next unit's table is cleared once every wave is done with this one.  Its marker
        // comes from the next unit's first probe keys, loaded during the last batch: every hash
        // of a partition has the partition's top bits (a unit without probe keys never reads
        // its table, so its marker does not matter).
        unit_totals<B>(cnt, many, multi, sm.k, u, counts, wave_off, wsum, rec_word, [&] {
            if (more) clear_table<false, AOS, B>(nx, xa[0], tab);
        });  // ends with a barrier
        const uint32_t nn = sched_after(sc, need, nxi, slot);
        u = nxi;
        nxi = nn;
        ++sc.pos;
        un = nx;
    }
    if (done) {
        // Thread 0 wrote every count of this workgroup: a device-scope release orders them before
        // its arrival.  Only the last to arrive acquires (an acquire also drops the L2 lines that
        // workgroups still running on this XCD are reading).
        __shared__ uint32_t last;
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            last = atomicAdd(done, 1u) == gridDim.x - 1;
        }
        __syncthreads();
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            scan_counts_block<B>(counts, U, g.Umax, total, pub, wsum);
        }
        return;
    }
    // units past the device-side total must read as zero for the scan over Umax entries
    for (int64_t i = (int64_t)U + (int64_t)blockIdx.x * B + threadIdx.x; i < g.Umax;
         i += (int64_t)gridDim.x * B)
        counts[i] = 0;
}

// Whether unit v (record n) had a probe with more than kEmitSort matches: the flag the count pass
// put into a partitioned join's record, else entry 0 of the unit's wave_off record.
template <bool PART>
__device__ __forceinline__ bool unit_order(const uint64_t* wave_off, uint32_t v, const Unit& n)
{
    if constexpr (PART) return n.order;
    else return as_const(wave_off)[(size_t)v * kWaveRec] != 0;
}

// Whether any unit of [u, end) that shares unit u's R chunk had a probe with more than
// kEmitSort matches: then the chunk's table is put in canonical order.  end: the end of the
// contiguous run u is in, 0 for a unit outside a run (which builds its own table).
template <bool PART>
__device__ __forceinline__ bool chunk_needs_order(const JoinGeom& g, const uint64_t* wave_off, uint32_t u,
                                                  uint32_t end, const Unit& un)
{
    bool any = unit_order<PART>(wave_off, u, un);
    for (uint32_t v = u + 1; v < end && !any; ++v) {
        const Unit n = decode_unit<PART>(g, v);
        if (!same_chunk(n, un)) break;
        any = unit_order<PART>(wave_off, v, n);
    }
    return any;
}

// Write pass.  Units are walked in a Sched sequence (for one join a contiguous run per
// workgroup, for batches a round-robin head, then tickets); each wave writes the pairs of its probe
// tuples from the start the count pass recorded for it, in (batch, tuple, lane) order, with one
// wave-wide scan per round and no shared cursor: the output depends on the input and the plan
// only, not on which workgroup takes a unit.
template <bool AOS, bool SEMI, int B>
__global__ JL_WRITE_ATTR(B) void join_write_k(JoinGeom g, const uint64_t* __restrict__ offsets,
                                           const uint64_t* __restrict__ wave_off,
                                           const uint64_t* __restrict__ total,
                                           int2* __restrict__ out, uint64_t cap)
{
    uint4* const tab = write_lds;
    // an output too small for the exact count, or a plan other than the count pass's, receives
    // nothing
    if (*total > cap || (g.stamp_at && *g.stamp_at != g.stamp)) return;
    const uint32_t U = unit_total(g);
    const bool contig = g.contig != 0;  // uniform
    const int wv = uniform((int32_t)(threadIdx.x / kWave));
    uint4* q = manyq<B>() + wv * kManyQ;  // this wave's queue of probes with many matches
    uint32_t qn = 0;                 // uniform: its length
    __shared__ uint32_t slot[2];
    Sched sc = make_sched(U, contig, g.sched ? g.sched + 1 : nullptr);
    uint32_t u, nxi;
    sched_start(sc, u, nxi, slot);
    // Units of the static run of one join follow each other, so a unit whose R chunk is the
    // previous unit's keeps the table; other units build their own.
    const uint32_t run_end = contig ? sc.base + sc.head : 0u;
    // The next unit's R chunk (when it needs a new table) is loaded into registers while the
    // current unit probes, and the next unit's first S batch while its last batch probes.
    Unit un{};
    Chunk<true> ch;
    uint32_t pos[kBuildItems];
    constexpr int kWriteLoad = kWriteLoadOf<B>;
    uint32_t nx[kWriteLoad];
    int32_t nr[kWriteLoad];
    if (u < U) {
        un = decode_unit<AOS>(g, u);
        load_chunk<AOS, true, B>(g, un, ch);
        if constexpr (!SEMI) load_tuples<AOS, B>(g, un, 0, nx, nr);
    }
    Unit tu{};  // the unit whose chunk is in the table (rN == 0: none yet)
    const cptr<uint64_t> offs = as_const(offsets);
    const cptr<uint64_t> wo = as_const(wave_off);
    while (u < U) {
        const bool need = sched_need(sc, nxi);
        uint32_t tk = 0;
        if (need && threadIdx.x == 0) tk = atomicAdd(sc.ticket, 1u);
        const bool more = nxi < U;
        const bool in_run = contig && sc.pos < sc.head;            // uniform
        const bool next_in_run = contig && sc.pos + 1 < sc.head;  // uniform
        if (!in_run || tu.rN == 0 || !same_chunk(un, tu)) {  // uniform: a new chunk (loaded in ch)
            const bool order = chunk_needs_order<AOS>(g, wave_off, u, in_run ? run_end : 0u, un);
            const Table tb = insert_chunk<true, AOS, B>(g, un, ch, tab, pos);
            if (order) {
                uint32_t* rids = reinterpret_cast<uint32_t*>(tab + tb.nb);
                if (AOS && tb.marked) canonicalize<AOS, true, B>(tb, un.bits, un, ch, pos, rids);
                else canonicalize<AOS, false, B>(tb, un.bits, un, ch, pos, rids);
            }
            tu = un;
        }
        // this wave's first output slot in unit u, and the start of its block of many-match pairs
        uint64_t cursor = uniform(offs[u]) + (wv ? uniform(wo[(size_t)u * kWaveRec + wv]) : 0ull);
        const uint64_t wrec = uniform(wo[(size_t)u * kWaveRec + kWaveHalf + wv]);
        uint64_t cmany = cursor + (uint32_t)wrec;
        const uint32_t semi_rows = (uint32_t)(wrec >> 32);  // the semi-join's rows of this wave
#if JL_DEBUG
        const uint64_t cursor0 = cursor, cmany0 = cmany;
#endif
        const Table t = table_of<true, AOS>(un, tab);
        const Unit nxt = more ? decode_unit<AOS>(g, nxi) : Unit{};
        if (more && (!next_in_run || !same_chunk(nxt, un))) load_chunk<AOS, true, B>(g, nxt, ch);
        const uint32_t* rw = reinterpret_cast<const uint32_t*>(t.rids);
        auto batches = [&](auto marked) {
            constexpr bool M = decltype(marked)::value;
            // kWriteLoad probe tuples per lane (lanes and tuples in range where ok_of(j) holds):
            // probed kWriteBatch at a time, pairs written
            auto round = [&](const uint32_t (&cx)[kWriteLoad], const int32_t (&cr)[kWriteLoad], auto ok_of) {
#pragma unroll
                for (int h = 0; h < kWriteLoad; h += kWriteBatch) {
                    uint32_t x[kWriteBatch], m[kWriteBatch], p1[kWriteBatch], p2[kWriteBatch];
                    int32_t srid[kWriteBatch];
                    bool ok[kWriteBatch];
#pragma unroll
                    for (int i = 0; i < kWriteBatch; ++i) {
                        x[i] = cx[h + i];
                        srid[i] = cr[h + i];
                        ok[i] = ok_of(h + i);
                    }
                    probe_write<kWriteBatch, AOS, M>(t, un.bits, x, ok, m, p1, p2);
                    // Slots of probes with one or two matches: the wave's cursor plus an
                    // exclusive scan over (tuple i, lane); the pairs of the i-th tuple of every
                    // lane are contiguous, so each store instruction writes one coalesced run.
                    uint32_t excl[kWriteBatch], wtot = 0;
#pragma unroll
                    for (int i = 0; i < kWriteBatch; ++i) {
                        const uint32_t ms = m[i] <= 2 ? m[i] : 0u;
                        const uint32_t inc = wave_incl_scan(ms);
                        excl[i] = wtot + inc - ms;
                        wtot += (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
                    }
#pragma unroll
                    for (int i = 0; i < kWriteBatch; ++i) {
                        const uint64_t slot = cursor + excl[i];
                        // two matches leave in ascending rid order
                        const int32_t ra = (int32_t)rw[p1[i]], rb = (int32_t)rw[p2[i]];
                        const bool sw = m[i] == 2 && rb < ra;
                        if (m[i] >= 1 && m[i] <= 2 && slot < cap)
                            put_pair(&out[slot], make_int2(sw ? rb : ra, srid[i]));
                        if (m[i] == 2 && slot + 1 < cap)
                            put_pair(&out[slot + 1], make_int2(sw ? ra : rb, srid[i]));
                        const bool many = m[i] > 2;
                        const uint64_t bm = ballot(many);
                        if (bm) {  // uniform
                            const uint32_t c = (uint32_t)__builtin_popcountll(bm);
                            if (qn + c > (uint32_t)kManyQ) {
                                cmany = flush_many<AOS, M, B>(t.nb, un.bits, wv, qn, cmany, out, cap);
                                qn = 0;
                            }
                            if (many) q[qn + mask_rank(bm)] = make_uint4(x[i], (uint32_t)srid[i], m[i], 0u);
                            qn += c;
                        }
                    }
                    cursor += wtot;
                }
            };
            if (SEMI && !un.shared) {  // uniform
                // only this wave's probe rows with matches, as the count pass recorded them
                for (uint32_t k0 = 0; k0 < semi_rows; k0 += kWave * kWriteLoad) {  // wave-uniform
                    uint32_t cx[kWriteLoad];
                    int32_t cr[kWriteLoad];
#pragma unroll
                    for (int j = 0; j < kWriteLoad; ++j) {
                        const uint32_t k = k0 + j * kWave + lane_id();
                        const uint32_t row = g.semi[semi_slot(un.sBeg, k < semi_rows ? k : 0u, wv)];
                        const int2 tp = g.st[row];
                        cx[j] = (uint32_t)tp.x;
                        cr[j] = tp.y;
                    }
                    round(cx, cr, [&](int j) { return k0 + j * kWave + lane_id() < semi_rows; });
                }
            } else {
                if (SEMI) load_tuples<AOS, B>(g, un, 0, nx, nr);  // not loaded ahead in this mode
                for (uint32_t e0 = 0; e0 < un.sN; e0 += B * kWriteLoad) {
                    uint32_t cx[kWriteLoad];
                    int32_t cr[kWriteLoad];
#pragma unroll
                    for (int i = 0; i < kWriteLoad; ++i) {
                        cx[i] = nx[i];
                        cr[i] = nr[i];
                    }
                    if (e0 + B * kWriteLoad < un.sN)
                        load_tuples<AOS, B>(g, un, e0 + B * kWriteLoad, nx, nr);
                    else if (more)
                        load_tuples<AOS, B>(g, nxt, 0, nx, nr);
                    round(cx, cr, [&](int j) { return e0 + j * B + threadIdx.x < un.sN; });
                }
            }
        };
        if (AOS && t.marked) batches(std::true_type{});
        else batches(std::false_type{});
        if (qn) {  // uniform: the queue must be empty before the table changes
            if (AOS && t.marked) cmany = flush_many<AOS, true, B>(t.nb, un.bits, wv, qn, cmany, out, cap);
            else cmany = flush_many<AOS, false, B>(t.nb, un.bits, wv, qn, cmany, out, cap);
            qn = 0;
        }
#if JL_DEBUG
        const uint64_t wrote = (cursor - cursor0) + (cmany - cmany0);
        if (g.dbg && lane_id() == 0 && wrote > 0)
            atomicAdd(reinterpret_cast<unsigned long long*>(&g.dbg[u]), (unsigned long long)wrote);
#endif
        if constexpr (!SEMI)
            if (un.sN == 0 && more) load_tuples<AOS, B>(g, nxt, 0, nx, nr);
        sched_put(sc, need, tk, slot);
        __syncthreads();
        const uint32_t nn = sched_after(sc, need, nxi, slot);
        u = nxi;
        nxi = nn;
        ++sc.pos;
        un = nxt;
    }
    // The last workgroup to finish resets the ticket counter for the next write from this
    // workspace (every workgroup took its last ticket before it arrives here).
    if (sc.ticket && threadIdx.x == 0 && atomicAdd(g.sched + 2, 1u) == gridDim.x - 1) {
        atomicExch(g.sched + 1, 0u);
        atomicExch(g.sched + 2, 0u);
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace


// Arrival order: the sorted tile, shares/starts and shifts per partition, scan scratch.
// Ordered: half of the sorted tile, per-wave counters and shifts per partition, scan scratch.
static size_t scatter_lds(int P, bool ordered)
{
    if (!ordered) return (size_t)kScatTile * sizeof(int2) + (size_t)P * 8 + (kScatBlock / kWave + 1) * 4;
    return (size_t)kScatHalf * sizeof(int2) + (size_t)(kScatWaves / 2) * P * 4 + (size_t)P * 4 +
           (kScatWaves + 1) * 4;
}

static bool ordered_knob() { return tune_get(TUNE_HASH_DETERMINISTIC, 0) != 0; }

// Default fan-out: mean partition size <= 0.9 * cap keeps the largest partitions (mean + 6 sigma
// for hashed unique keys) under cap; past 2^kMaxBits partitions R chunks repeat per S slice.
static int default_bits(int64_t nR, int cap)
{
    const double target = cap * 0.9;
    int bits = 0;
    while (bits < kMaxBits && (double)nR / (double)(1 << bits) > target) ++bits;
    return bits;
}

static int env_cap()
{
    int64_t cap = tune_get(TUNE_HASH_CAP, 9216);
    if (cap < 64) cap = 64;
    if (cap > kMaxCap) cap = kMaxCap;
    return (int)cap;
}

// Persistent grid of one join's count (rids false) or write kernel: as many 1024-thread
// workgroups per CU as the LDS table allows, at most 2.
static int join_grid(int num_cus, int cap, bool rids)
{
    int per_cu = (int)((160 * 1024) / (table_lds((uint32_t)cap, rids) + 128));
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 2) per_cu = 2;
    return num_cus * per_cu;
}

HashPlan hash_plan(int64_t nR, int64_t nS, int num_cus, int prebuilt_bits, bool semi)
{
    HashPlan pl{};
    pl.nR = nR;
    pl.nS = nS;
    const int cap = env_cap();
    pl.cap = cap;
    pl.slice = (int)tune_get(TUNE_HASH_SLICE, 32768);
    if (pl.slice < 1024) pl.slice = 1024;
    const int64_t single_max = tune_get(TUNE_HASH_SINGLE_MAX, 16) * cap;
    pl.prebuilt = prebuilt_bits >= 0;
    pl.ordered = ordered_knob();
    const int forced_bits = pl.prebuilt ? prebuilt_bits : (int)tune_get(TUNE_HASH_BITS, -1);
    pl.single = !pl.prebuilt && (forced_bits == 0 || (forced_bits < 0 && nR <= single_max));
    if (semi && !pl.single) {
        // The semi-join's write pass visits about the matching probe rows only, so its units pay
        // their fixed costs (table build, per-unit loads) for few rows: S slices up to one unit
        // per count workgroup, at most 128K rows (1M x 64M, 1% matching: write 56 -> 32 us, the
        // count pass unchanged).
        int64_t sl = nS / join_grid(num_cus, cap, false) / 1024 * 1024;
        if (sl > 131072) sl = 131072;
        if (sl > pl.slice) pl.slice = (int)sl;
    }
    size_t off = 256;  // header: [0] uint64 total, [8] uint32 units
    if (pl.single) {
        pl.bits = 0;
        pl.P = 1;
        const int64_t nrc = nR > 0 ? ceil_div(nR, cap) : 0;
        // S slices: enough units to cover the chip, each at least 1024 probes
        int64_t nss = 1;
        if (nR > 0 && nS > 0) {
            const int64_t want = (int64_t)num_cus * 2;
            nss = ceil_div(want, nrc);
            const int64_t max_ss = ceil_div(nS, 1024);
            if (nss > max_ss) nss = max_ss;
            if (nss < 1) nss = 1;
        }
        pl.nSs = nss;
        pl.Umax = (nR > 0 && nS > 0) ? nrc * nss : 0;
    } else {
        int bits = forced_bits;
        if (bits < 0) bits = default_bits(nR, cap) < 1 ? 1 : default_bits(nR, cap);
        if (bits > kMaxBits) bits = kMaxBits;
        pl.bits = bits;
        pl.P = 1 << bits;
        // scatter chunks: one per resident scatter workgroup (the sorted tile decides how many
        // fit a CU), each a multiple of kChunkAlign rows
        int per_cu = (int)((160 * 1024) / scatter_lds(pl.P, pl.ordered));
        if (per_cu < 1) per_cu = 1;
        if (per_cu > 2) per_cu = 2;
        auto chunk_for = [&](int64_t n) {
            int64_t c = ceil_div(n, (int64_t)num_cus * per_cu);
            c = ceil_div(c, kChunkAlign) * kChunkAlign;
            if (c < kChunkAlign) c = kChunkAlign;
            return c;
        };
        pl.chR = chunk_for(nR);
        pl.chS = chunk_for(nS);
        pl.nChR = nR > 0 && !pl.prebuilt ? ceil_div(nR, pl.chR) : 0;  // a prebuilt R has its own
        pl.nChS = nS > 0 ? ceil_div(nS, pl.chS) : 0;
        pl.Umax = pl.P + ceil_div(nR, cap) + ceil_div(nS, pl.slice) + 2;
        // totR[P], totS[P], group shares of S [kGroups][P], of R [kGroups][P]: cleared together
        // (only the S half, from totS on, for a prebuilt R)
        pl.off_tot = off;
        pl.off_grpS = off + (size_t)2 * pl.P * 4;
        pl.off_grpR = pl.off_grpS + (size_t)kGroups * pl.P * 4;
        pl.off_done = pl.off_grpR + (size_t)kGroups * pl.P * 4;  // cleared with the sizes and shares
        off = align_up(pl.off_done + 4);
        pl.off_baseR = off;
        off = align_up(off + (size_t)(pl.P + 1) * 4);
        pl.off_baseS = off;
        off = align_up(off + (size_t)(pl.P + 1) * 4);
        pl.off_tupR = off;
        off = align_up(off + (size_t)(pl.prebuilt ? 0 : nR) * 8);
        pl.off_tupS = off;
        off = align_up(off + (size_t)nS * 8);
        pl.off_info = off;
        off = align_up(off + (size_t)pl.P * sizeof(PartInfo));
        pl.off_units = off;
        off = align_up(off + (size_t)(pl.P + 1) * 4);
        pl.off_umap = off;  // the unit records
        off = align_up(off + (size_t)pl.Umax * 16);
        // ordered scatter: per-tile counts, then run offsets, of each side (chunks x tiles per
        // chunk x P)
        const size_t on = pl.ordered ? 1 : 0;
        pl.off_cntR = off;
        off = align_up(off + ((on * (size_t)pl.nChR * (size_t)tiles_of(pl.chR) * 4) << pl.bits));
        pl.off_cntS = off;
        off = align_up(off + ((on * (size_t)pl.nChS * (size_t)tiles_of(pl.chS) * 4) << pl.bits));
    }
    pl.off_counts = off;
    off = align_up(off + (size_t)(pl.Umax > 0 ? pl.Umax : 1) * 8);
    pl.off_wave = off;
    off = align_up(off + (size_t)(pl.Umax > 0 ? pl.Umax : 1) * kWaveRec * 8);
    size_t temp = scan_temp_elems<uint64_t>(pl.Umax) * 8;
    if (!pl.single) {
        const size_t t1 = scan_temp_elems<uint32_t>(pl.P + 1) * 4;
        temp = temp > t1 ? temp : t1;
    }
    pl.off_temp = off;
    off = align_up(off + temp + 8);
    pl.semi = semi && !pl.single ? 1 : 0;
    pl.off_semi = off;  // the semi-join's probe rows: one slot per probe row
    off = align_up(off + (pl.semi ? (size_t)nS * 4 : 0));
    pl.off_dbg = off;  // last: the checking build's per-unit written counts
    off = align_up(off + (JL_DEBUG ? (size_t)(pl.Umax > 0 ? pl.Umax : 1) * 8 : 0));
    pl.bytes = off;
    pl.gridCount = join_grid(num_cus, cap, false);
    pl.gridWrite = join_grid(num_cus, cap, true);
    pl.stamp = plan_stamp({JOIN_KIND_HASH, pl.nR, pl.nS, pl.single, pl.prebuilt, pl.ordered, pl.semi, pl.bits, pl.P, pl.cap,
                           pl.slice, pl.nSs, pl.chR, pl.chS, pl.Umax, pl.gridCount, pl.gridWrite,
                           (int64_t)pl.bytes});
    return pl;
}

static bool g_attr_done = false;

static hipError_t set_attrs()
{
    if (g_attr_done) return hipSuccess;
    const int big = 160 * 1024 - 4096;
    const int write_max = (int)(160 * 1024 - kWriteStaticLds - 256);  // beside its static queue
    const int write_max_b = (int)(160 * 1024 - kBatchStaticLds - 256);
    const void* fns[] = {
        (const void*)scatter_k<true, false>, (const void*)scatter_k<false, false>,
        (const void*)scatter_k<true, true>, (const void*)scatter_k<false, true>, (const void*)hist_k,
        (const void*)join_count_k<true, false, kJoinBlock>, (const void*)join_count_k<false, false, kJoinBlock>,
        (const void*)join_count_k<true, true, kJoinBlock>, (const void*)join_count_k<true, false, kBatchBlock>,
    };
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big);
        if (e != hipSuccess) return e;
    }
    for (const void* f : {(const void*)join_write_k<true, false, kJoinBlock>, (const void*)join_write_k<false, false, kJoinBlock>,
                          (const void*)join_write_k<true, true, kJoinBlock>}) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, write_max);
        if (e != hipSuccess) return e;
    }
    {
        const hipError_t e = hipFuncSetAttribute((const void*)join_write_k<true, false, kBatchBlock>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, write_max_b);
        if (e != hipSuccess) return e;
    }
    g_attr_done = true;
    return hipSuccess;
}

static SideItem whole_side(const join_rel_t& X, int bits)
{
    SideItem it{};
    it.key = X.key;
    it.rid = X.rid;
    it.bits = bits;
    return it;
}

static hipError_t hist_side(const SideItem* items, const SideItem& one, int64_t ch, int64_t n,
                            int64_t grid, int maxBits, uint32_t* tot, uint32_t* grp, int64_t stride,
                            uint32_t* cnt, hipStream_t st, bool is_r)
{
    if (grid <= 0) return hipSuccess;
    const size_t hl = (size_t)4 << maxBits;
    SideTwo none{};
    none.split = (uint32_t)grid;
    prof::Scope ph(st, is_r ? "hash.hist.R" : "hash.hist.S");
    hist_k<<<(unsigned)grid, kHistBlock, hl, st>>>(items, one, ch, n, tot, grp, (uint32_t)stride, cnt, none);
    return hipGetLastError();
}

// Both sides of a single join in one launch, R's chunks first.
static hipError_t hist_pair(const SideItem& oneR, int64_t chR, int64_t nR, int64_t gridR,
                            uint32_t* totR, uint32_t* grpR, uint32_t* cntR, const SideItem& oneS,
                            int64_t chS, int64_t nS, int64_t gridS, uint32_t* totS, uint32_t* grpS,
                            uint32_t* cntS, int bits, int64_t stride, hipStream_t st)
{
    if (gridR + gridS <= 0) return hipSuccess;
    SideTwo two{};
    two.one = oneS;
    two.chunk = chS;
    two.n = nS;
    two.tot = totS;
    two.grp = grpS;
    two.cnt = cntS;
    two.split = (uint32_t)gridR;
    prof::Scope ph(st, "hash.hist");
    hist_k<<<(unsigned)(gridR + gridS), kHistBlock, (size_t)4 << bits, st>>>(
        nullptr, oneR, chR, nR, totR, grpR, (uint32_t)stride, cntR, two);
    return hipGetLastError();
}

// group shares -> group cursors, after the partition starts are known
static hipError_t cursors_side(uint32_t* grp, const uint32_t* base, int64_t stride, hipStream_t st)
{
    if (stride <= 0) return hipSuccess;
    prof::Scope pc(st, "hash.plan");
    group_cursors_k<<<(unsigned)ceil_div(stride, 256), 256, 0, st>>>(grp, base, (uint32_t)stride, stride);
    return hipGetLastError();
}

// Partition starts and group starts of both sides (a NULL totR or totS skips that side), and
// the run offsets of the sides' tiles given by bR and bS (cnt NULL: none): one launch up to
// kFuseParts partitions, else a scan and a cursor kernel per side (then no run offsets: batches
// compute theirs with band_batch_k).
static hipError_t starts_sides(const uint32_t* totR, uint32_t* baseR, uint32_t* grpR,
                               const uint32_t* totS, uint32_t* baseS, uint32_t* grpS, int64_t n,
                               uint32_t* temp, hipStream_t st, const BandSide& bR = BandSide{},
                               const BandSide& bS = BandSide{})
{
    if (n <= kFuseParts) {
        prof::Scope pc(st, "hash.plan");
        const int64_t blocks = 2 + band_blocks(bR) + band_blocks(bS);
        part_starts_k<<<(unsigned)blocks, kFuseBlock, 0, st>>>(totR, baseR, grpR, totS, baseS, grpS,
                                                               (uint32_t)n, (int)n, bR, bS);
        return hipGetLastError();
    }
    if (bR.cnt || bS.cnt) return hipErrorInvalidValue;  // band work rides only on the fused launch
    hipError_t e = hipSuccess;
    if (totR) {
        e = exclusive_scan<uint32_t>(totR, baseR, n, nullptr, temp, st);
        if (e == hipSuccess) e = cursors_side(grpR, baseR, n, st);
    }
    if (e == hipSuccess && totS) {
        e = exclusive_scan<uint32_t>(totS, baseS, n, nullptr, temp, st);
        if (e == hipSuccess) e = cursors_side(grpS, baseS, n, st);
    }
    return e;
}

// The band work of one side of a single join: its chunks start at workgroup `base` of the
// histogram and scatter launches.
static BandSide band_of(uint32_t* cnt, int64_t chunk, int64_t n, int64_t nCh, int bits, int64_t base)
{
    BandSide b{};
    if (nCh <= 0 || !cnt) return b;
    b.cnt = cnt;
    b.chunk = chunk;
    b.n = n;
    b.nCh = nCh;
    b.bits = bits;
    b.blockBase = (uint32_t)base;
    return b;
}

// Per-partition plans, unit starts (total at *Utotal) and the unit -> partition map.
static hipError_t plan_parts(const PartPlan& q, int64_t nParts, PartInfo* info, uint32_t* units,
                             uint32_t* Utotal, int64_t Umax, uint4* urec, uint32_t* temp,
                             hipStream_t st)
{
    if (nParts <= kFuseParts) {
        prof::Scope pp(st, "hash.plan");
        plan_k<<<1, kFuseBlock, 0, st>>>(q, (int)nParts, info, units, Utotal, Umax, urec);
        return hipGetLastError();
    }
    {
        prof::Scope pp(st, "hash.plan");
        plan_units_k<<<(unsigned)ceil_div(nParts + 1, 256), 256, 0, st>>>(q, (int)nParts, info, units);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = exclusive_scan<uint32_t>(units, units, nParts + 1, Utotal, temp, st);
    if (e != hipSuccess) return e;
    {
        prof::Scope pe(st, "hash.plan");
        expand_units_k<<<(unsigned)ceil_div(nParts, 256), 256, 0, st>>>(units, info, (int)nParts, q.cap, Umax, urec);
    }
    return hipGetLastError();
}

static hipError_t scatter_side(const SideItem* items, const SideItem& one, int64_t ch, int64_t n,
                               int64_t grid, int maxBits, uint32_t* cur, int64_t stride,
                               int2* out, const uint32_t* cnt, hipStream_t st, bool is_r,
                               const PlanArgs* plan = nullptr)
{
    const PlanArgs pa = plan ? *plan : PlanArgs{};
    const int64_t all = grid + (plan ? 1 : 0);
    if (all <= 0) return hipSuccess;
    const size_t sl = scatter_lds(1 << maxBits, cnt != nullptr);
    SideTwo none{};
    none.split = (uint32_t)grid;
    prof::Scope ps(st, is_r ? "hash.scatter.R" : "hash.scatter.S");
    const bool rids = items != nullptr || one.rid != nullptr;
    if (cnt) {
        if (rids) scatter_k<true, true><<<(unsigned)all, kScatBlock, sl, st>>>(items, one, ch, n, cur, (uint32_t)stride, out, cnt, none, pa);
        else scatter_k<false, true><<<(unsigned)all, kScatBlock, sl, st>>>(items, one, ch, n, cur, (uint32_t)stride, out, cnt, none, pa);
    } else {
        if (rids) scatter_k<true, false><<<(unsigned)all, kScatBlock, sl, st>>>(items, one, ch, n, cur, (uint32_t)stride, out, cnt, none, pa);
        else scatter_k<false, false><<<(unsigned)all, kScatBlock, sl, st>>>(items, one, ch, n, cur, (uint32_t)stride, out, cnt, none, pa);
    }
    return hipGetLastError();
}

// Both sides of a single join in one launch, R's chunks first (the plan's workgroup last).
static hipError_t scatter_pair(const SideItem& oneR, int64_t chR, int64_t nR, int64_t gridR,
                               uint32_t* curR, int2* outR, const uint32_t* cntR,
                               const SideItem& oneS, int64_t chS, int64_t nS, int64_t gridS,
                               uint32_t* curS, int2* outS, uint32_t* cntS, int bits,
                               int64_t stride, hipStream_t st, const PlanArgs* plan)
{
    const PlanArgs pa = plan ? *plan : PlanArgs{};
    const int64_t all = gridR + gridS + (plan ? 1 : 0);
    if (all <= 0) return hipSuccess;
    SideTwo two{};
    two.one = oneS;
    two.chunk = chS;
    two.n = nS;
    two.grp = curS;
    two.out = outS;
    two.cnt = cntS;
    two.split = (uint32_t)gridR;
    const bool ordered = cntR != nullptr || cntS != nullptr;
    const size_t sl = scatter_lds(1 << bits, ordered);
    prof::Scope ps(st, "hash.scatter");
    const bool rids = oneR.rid != nullptr || oneS.rid != nullptr;
    if (ordered) {
        if (rids) scatter_k<true, true><<<(unsigned)all, kScatBlock, sl, st>>>(nullptr, oneR, chR, nR, curR, (uint32_t)stride, outR, cntR, two, pa);
        else scatter_k<false, true><<<(unsigned)all, kScatBlock, sl, st>>>(nullptr, oneR, chR, nR, curR, (uint32_t)stride, outR, cntR, two, pa);
    } else {
        if (rids) scatter_k<true, false><<<(unsigned)all, kScatBlock, sl, st>>>(nullptr, oneR, chR, nR, curR, (uint32_t)stride, outR, cntR, two, pa);
        else scatter_k<false, false><<<(unsigned)all, kScatBlock, sl, st>>>(nullptr, oneR, chR, nR, curR, (uint32_t)stride, outR, cntR, two, pa);
    }
    return hipGetLastError();
}

static JoinGeom make_geom(const HashPlan& pl, const join_rel_t& R, const join_rel_t& S, char* ws,
                          const RView* pre)
{
    JoinGeom g{};
    g.bits = pl.bits;
    g.cap = (uint32_t)pl.cap;
    g.Umax = pl.Umax;
    g.stamp_at = reinterpret_cast<uint64_t*>(ws + kStampOffset);
    g.stamp = pl.stamp;
    g.dbg = JL_DEBUG ? reinterpret_cast<uint64_t*>(ws + pl.off_dbg) : nullptr;
    g.semi = pl.semi ? reinterpret_cast<uint32_t*>(ws + pl.off_semi) : nullptr;
    if (pl.single) {
        g.single = 1;
        g.rk = R.key;
        g.rr = R.rid;
        g.sk = S.key;
        g.sr = S.rid;
        g.one.rStart = 0;
        g.one.nR = (uint32_t)R.n;
        g.one.sStart = 0;
        g.one.nS = (uint32_t)S.n;
        g.one.nSs = (uint32_t)pl.nSs;
        g.one.nRc = (uint32_t)ceil_div(R.n, pl.cap);
        g.Uhost = (uint32_t)pl.Umax;
        g.P = 1;
    } else {
        g.single = 0;
        g.contig = 1;
        g.rt = pre ? pre->tup : reinterpret_cast<const int2*>(ws + pl.off_tupR);
        g.st = reinterpret_cast<const int2*>(ws + pl.off_tupS);
        g.part = reinterpret_cast<const PartInfo*>(ws + pl.off_info);
        g.unitStart = reinterpret_cast<const uint32_t*>(ws + pl.off_units);
        g.urec = reinterpret_cast<const uint4*>(ws + pl.off_umap);
        g.Uptr = reinterpret_cast<const uint32_t*>(ws + 8);
        g.P = pl.P;
        // one join's units are even and its write pass keeps a table across consecutive units of
        // one R chunk: static shares (tickets measured slower on 16M x 64M and 1M x 64M)
        g.sched = nullptr;
    }
    return g;
}

hipError_t hash_count(const HashPlan& pl, const join_rel_t& R, const join_rel_t& S, char* ws,
                      hipStream_t st, const RView* pre, uint64_t* pub)
{
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    uint64_t* total = reinterpret_cast<uint64_t*>(ws);
    uint64_t* counts = reinterpret_cast<uint64_t*>(ws + pl.off_counts);
    char* temp = ws + pl.off_temp;
    if (!pl.single) {
        uint32_t* totR = reinterpret_cast<uint32_t*>(ws + pl.off_tot);
        uint32_t* totS = totR + pl.P;
        uint32_t* baseR = reinterpret_cast<uint32_t*>(ws + pl.off_baseR);
        uint32_t* baseS = reinterpret_cast<uint32_t*>(ws + pl.off_baseS);
        uint32_t* grpR = reinterpret_cast<uint32_t*>(ws + pl.off_grpR);
        uint32_t* grpS = reinterpret_cast<uint32_t*>(ws + pl.off_grpS);
        int2* tupR = reinterpret_cast<int2*>(ws + pl.off_tupR);
        int2* tupS = reinterpret_cast<int2*>(ws + pl.off_tupS);
        {
            // a prebuilt R keeps its sizes: only the S sizes and shares are cleared
            prof::Scope pz(st, "hash.plan");
            uint32_t* z = pre ? totS : totR;
            const int64_t nz = reinterpret_cast<uint32_t*>(ws + pl.off_done) + 1 - z;
            zero_u32_k<<<(unsigned)ceil_div(nz, 256), 256, 0, st>>>(z, nz);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const SideItem oneR = whole_side(R, pl.bits), oneS = whole_side(S, pl.bits);
        uint32_t* cntR = pl.ordered ? reinterpret_cast<uint32_t*>(ws + pl.off_cntR) : nullptr;
        uint32_t* cntS = pl.ordered ? reinterpret_cast<uint32_t*>(ws + pl.off_cntS) : nullptr;
        if (pre)
            e = hist_side(nullptr, oneS, pl.chS, S.n, pl.nChS, pl.bits, totS, grpS, pl.P, cntS, st, false);
        else
            e = hist_pair(oneR, pl.chR, R.n, pl.nChR, totR, grpR, cntR, oneS, pl.chS, S.n, pl.nChS,
                          totS, grpS, cntS, pl.bits, pl.P, st);
        if (e != hipSuccess) return e;
        // the scatter launch puts R's chunks first (none for a prebuilt R)
        const int64_t sBase = pre ? 0 : pl.nChR;
        e = starts_sides(pre ? nullptr : totR, baseR, grpR, totS, baseS, grpS, pl.P,
                         reinterpret_cast<uint32_t*>(temp), st,
                         pre ? BandSide{} : band_of(cntR, pl.chR, R.n, pl.nChR, pl.bits, 0),
                         band_of(cntS, pl.chS, S.n, pl.nChS, pl.bits, sBase));
        if (e != hipSuccess) return e;
        const uint32_t* pbaseR = pre ? pre->base : baseR;
        const uint32_t* ptotR = pre ? pre->tot : totR;
        PlanArgs pa{};
        pa.q = PartPlan{pbaseR, ptotR, baseS, totS, nullptr, nullptr, 0, pl.bits, (uint32_t)pl.cap,
                        (uint32_t)pl.slice};
        pa.nParts = (int)pl.P;
        pa.info = reinterpret_cast<PartInfo*>(ws + pl.off_info);
        pa.units = reinterpret_cast<uint32_t*>(ws + pl.off_units);
        pa.Utotal = reinterpret_cast<uint32_t*>(ws + 8);
        pa.Umax = pl.Umax;
        pa.urec = reinterpret_cast<uint4*>(ws + pl.off_umap);
        // up to kFuseParts partitions the plan is one workgroup of the scatter launch
        const PlanArgs* fused = pl.P <= kFuseParts ? &pa : nullptr;
        if (pre)
            e = scatter_side(nullptr, oneS, pl.chS, S.n, pl.nChS, pl.bits, grpS, pl.P, tupS, cntS, st,
                             false, fused);
        else
            e = scatter_pair(oneR, pl.chR, R.n, pl.nChR, grpR, tupR, cntR, oneS, pl.chS, S.n, pl.nChS,
                             grpS, tupS, cntS, pl.bits, pl.P, st, fused);
        if (e != hipSuccess) return e;
        if (!fused) {
            e = plan_parts(pa.q, pl.P, pa.info, pa.units, pa.Utotal, pl.Umax, pa.urec,
                           reinterpret_cast<uint32_t*>(temp), st);
            if (e != hipSuccess) return e;
        }
    }
    if (pl.Umax > 0) {
        const JoinGeom g = make_geom(pl, R, S, ws, pre);
        const unsigned grid = (unsigned)(pl.single ? pl.Umax : pl.gridCount);
        const size_t lds = table_lds((uint32_t)pl.cap, false);
        // the partitioned path cleared the arrival counter with the partition sizes
        uint32_t* done = !pl.single && pl.Umax <= kFuseScanMax
                             ? reinterpret_cast<uint32_t*>(ws + pl.off_done) : nullptr;
        uint64_t* wave_off = reinterpret_cast<uint64_t*>(ws + pl.off_wave);
        prof::Scope pc(st, "hash.count");
        if (pl.single) join_count_k<false, false, kJoinBlock><<<grid, kJoinBlock, lds, st>>>(g, counts, wave_off, nullptr, total, nullptr);
        else if (pl.semi) join_count_k<true, true, kJoinBlock><<<grid, kJoinBlock, lds, st>>>(g, counts, wave_off, done, total, pub);
        else join_count_k<true, false, kJoinBlock><<<grid, kJoinBlock, lds, st>>>(g, counts, wave_off, done, total, pub);
        e = hipGetLastError();
        if (e != hipSuccess || done) return e;
    }
    return exclusive_scan<uint64_t>(counts, counts, pl.Umax, total, reinterpret_cast<uint64_t*>(temp), st,
                                    pub);
}

hipError_t hash_write(const HashPlan& pl, const join_rel_t& R, const join_rel_t& S, char* ws,
                      int32_t* pairs, uint64_t cap, hipStream_t st, const RView* pre)
{
    if (pl.Umax <= 0) return hipSuccess;
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    const uint64_t* offsets = reinterpret_cast<const uint64_t*>(ws + pl.off_counts);
    const uint64_t* wave_off = reinterpret_cast<const uint64_t*>(ws + pl.off_wave);
    const uint64_t* total = reinterpret_cast<const uint64_t*>(ws);
    const JoinGeom g = make_geom(pl, R, S, ws, pre);
    const unsigned grid = (unsigned)(pl.single ? pl.Umax : pl.gridWrite);
    const size_t lds = table_lds((uint32_t)pl.cap, true);
    int2* out = reinterpret_cast<int2*>(pairs);
    prof::Scope pw(st, "hash.write");
    if (pl.single) join_write_k<false, false, kJoinBlock><<<grid, kJoinBlock, lds, st>>>(g, offsets, wave_off, total, out, cap);
    else if (pl.semi) join_write_k<true, true, kJoinBlock><<<grid, kJoinBlock, lds, st>>>(g, offsets, wave_off, total, out, cap);
    else join_write_k<true, false, kJoinBlock><<<grid, kJoinBlock, lds, st>>>(g, offsets, wave_off, total, out, cap);
    return hipGetLastError();
}

static size_t take(size_t& off, size_t bytes)
{
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
}

// ------------------------------------------------------------------------ resident builds --
// The partitioned form of a build relation (its tuples, partition sizes and starts), kept by the
// caller and probed by many probe relations: only the probe side is partitioned per join.

BuildPlan hash_build_plan(int64_t nR, int num_cus)
{
    BuildPlan b{};
    b.nR = nR;
    const int cap = env_cap();
    int bits = default_bits(nR, cap);
    if (bits < 1) bits = 1;
    if (bits > kMaxBits) bits = kMaxBits;
    b.bits = bits;
    b.P = 1 << bits;
    b.ordered = ordered_knob();
    int per_cu = (int)((160 * 1024) / scatter_lds(b.P, b.ordered));
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 2) per_cu = 2;
    int64_t c = ceil_div(nR > 0 ? nR : 1, (int64_t)num_cus * per_cu);
    c = ceil_div(c, kChunkAlign) * kChunkAlign;
    b.chR = c < kChunkAlign ? kChunkAlign : c;
    b.nChR = nR > 0 ? ceil_div(nR, b.chR) : 0;
    size_t off = 256;
    b.off_tot = take(off, (size_t)b.P * 4 * (1 + kGroups));  // sizes, then group shares: cleared together
    b.off_base = take(off, (size_t)(b.P + 1) * 4);
    b.off_tup = take(off, (size_t)nR * 8);
    b.off_temp = take(off, scan_temp_elems<uint32_t>(b.P + 1) * 4 + 8);
    b.off_cnt = take(off, ((b.ordered ? (size_t)b.nChR * (size_t)tiles_of(b.chR) * 4 : 0)) << b.bits);
    b.bytes = off;
    return b;
}

hipError_t hash_build(const BuildPlan& b, const join_rel_t& R, char* build, hipStream_t st)
{
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    uint32_t* tot = reinterpret_cast<uint32_t*>(build + b.off_tot);
    uint32_t* base = reinterpret_cast<uint32_t*>(build + b.off_base);
    uint32_t* grp = tot + b.P;
    int2* tup = reinterpret_cast<int2*>(build + b.off_tup);
    {
        prof::Scope pz(st, "hash.plan");
        const int64_t nz = (int64_t)b.P * (1 + kGroups);
        zero_u32_k<<<(unsigned)ceil_div(nz, 256), 256, 0, st>>>(tot, nz);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const SideItem one = whole_side(R, b.bits);
    uint32_t* cnt = b.ordered ? reinterpret_cast<uint32_t*>(build + b.off_cnt) : nullptr;
    e = hist_side(nullptr, one, b.chR, R.n, b.nChR, b.bits, tot, grp, b.P, cnt, st, true);
    if (e != hipSuccess) return e;
    e = starts_sides(tot, base, grp, nullptr, nullptr, nullptr, b.P,
                     reinterpret_cast<uint32_t*>(build + b.off_temp), st,
                     band_of(cnt, b.chR, R.n, b.nChR, b.bits, 0));
    if (e != hipSuccess) return e;
    return scatter_side(nullptr, one, b.chR, R.n, b.nChR, b.bits, grp, b.P, tup, cnt, st, true);
}

RView build_view(const BuildPlan& b, const void* build)
{
    const char* p = static_cast<const char*>(build);
    RView v;
    v.tot = reinterpret_cast<const uint32_t*>(p + b.off_tot);
    v.base = reinterpret_cast<const uint32_t*>(p + b.off_base);
    v.tup = reinterpret_cast<const int2*>(p + b.off_tup);
    return v;
}

// ------------------------------------------------------------------------- batched joins --
// Many independent joins go through the same kernels as one: every join gets its own fan-out
// and a contiguous block of partitions in shared partition arrays; histogram and scatter items
// are chunks of any join's sides; units of all joins form one list, so the count pass, the scan
// of unit counts and the write pass are one launch each, and join j's pairs land contiguously,
// in join order, in one output array.


static int job_bits(const join_job_t& j, int cap)
{
    int b = j.bits >= 0 ? j.bits : default_bits(j.R.n, cap);
    return b > kMaxBits ? kMaxBits : b;
}

static int64_t side_items(int64_t n) { return n > 0 ? ceil_div(n, kBatchChunk) : 0; }

// Tiles of all items of a side of n rows (every item but the last is kBatchChunk rows).
static int64_t side_tiles(int64_t n)
{
    if (n <= 0) return 0;
    const int64_t full = n / kBatchChunk, rest = n - full * kBatchChunk;
    return full * tiles_of(kBatchChunk) + tiles_of(rest);
}

int hash_batch_plan(int njobs, const join_job_t* jobs, int num_cus, BatchPlan* out)
{
    BatchPlan bp{};
    bp.njobs = njobs;
    bp.cap = env_cap() < kBatchCap ? env_cap() : kBatchCap;  // the batch kernels' tables
    bp.slice = (int)tune_get(TUNE_HASH_SLICE, 32768);
    if (bp.slice < 1024) bp.slice = 1024;
    bp.ordered = ordered_knob();
    int64_t umax = 0;
    uint64_t cntR = 0, cntS = 0;  // per-tile count entries of each side
    for (int j = 0; j < njobs; ++j) {
        const int b = job_bits(jobs[j], bp.cap);
        if (b > bp.maxBits) bp.maxBits = b;
        const int64_t P = (int64_t)1 << b;
        bp.nParts += P;
        bp.nItemsR += side_items(jobs[j].R.n);
        bp.nItemsS += side_items(jobs[j].S.n);
        cntR += (uint64_t)side_tiles(jobs[j].R.n) << b;
        cntS += (uint64_t)side_tiles(jobs[j].S.n) << b;
        bp.sumR += jobs[j].R.n;
        bp.sumS += jobs[j].S.n;
        umax += P + ceil_div(jobs[j].R.n, bp.cap) + ceil_div(jobs[j].S.n, bp.slice) + 1;
    }
    // partition starts, unit indices and item fields are 32-bit
    if (bp.sumR >= ((int64_t)1 << 32) || bp.sumS >= ((int64_t)1 << 32) || umax >= ((int64_t)1 << 31) ||
        bp.nParts * kGroups >= ((int64_t)1 << 32))
        return -1;
    bp.Umax = umax;
    size_t off = 256;  // header: [0] uint64 total, [8] uint32 units
    bp.off_jpart0 = take(off, (size_t)(njobs + 1) * 4);
    bp.off_jbits = take(off, (size_t)njobs * 4);
    bp.off_itemsR = take(off, (size_t)bp.nItemsR * sizeof(SideItem));
    bp.off_itemsS = take(off, (size_t)bp.nItemsS * sizeof(SideItem));
    // totR, totS, then the group shares of R and S: cleared together
    // sizes, group shares, then the count and write passes' unit tickets (Sched), cleared together
    bp.off_tot = take(off, ((size_t)(2 + 2 * kGroups) * bp.nParts + 4) * 4);
    bp.off_baseR = take(off, (size_t)(bp.nParts + 1) * 4);
    bp.off_baseS = take(off, (size_t)(bp.nParts + 1) * 4);
    bp.off_tupR = take(off, (size_t)bp.sumR * 8);
    bp.off_tupS = take(off, (size_t)bp.sumS * 8);
    bp.off_info = take(off, (size_t)bp.nParts * sizeof(PartInfo));
    bp.off_units = take(off, (size_t)(bp.nParts + 1) * 4);
    bp.off_umap = take(off, (size_t)(bp.Umax > 0 ? bp.Umax : 1) * 16);
    bp.off_counts = take(off, (size_t)(bp.Umax > 0 ? bp.Umax : 1) * 8);
    bp.off_wave = take(off, (size_t)(bp.Umax > 0 ? bp.Umax : 1) * kWaveRec * 8);
    bp.off_item0R = take(off, (size_t)(njobs + 1) * 4);
    bp.off_item0S = take(off, (size_t)(njobs + 1) * 4);
    bp.off_cntR = take(off, bp.ordered ? (size_t)cntR * 4 : 0);
    bp.off_cntS = take(off, bp.ordered ? (size_t)cntS * 4 : 0);
    size_t temp = scan_temp_elems<uint64_t>(bp.Umax) * 8;
    const size_t t1 = scan_temp_elems<uint32_t>(bp.nParts + 1) * 4;
    temp = temp > t1 ? temp : t1;
    bp.off_temp = take(off, temp + 8);
    bp.bytes = off;
    // 512-thread workgroups: four count workgroups (64 VGPRs) or two write workgroups (128
    // VGPRs, and their static queues) fit a CU when their tables do
    auto grid_for = [&](bool rids) {
        const size_t lds = table_lds((uint32_t)bp.cap, rids) + (rids ? kBatchStaticLds : 0) + 256;
        int per_cu = (int)((160 * 1024) / lds);
        if (per_cu < 1) per_cu = 1;
        if (per_cu > (rids ? 2 : 4)) per_cu = rids ? 2 : 4;
        return num_cus * per_cu;
    };
    bp.gridCount = grid_for(false);
    bp.gridWrite = grid_for(true);
    *out = bp;
    return 0;
}

hipError_t hash_batch_upload(const BatchPlan& bp, const join_job_t* jobs, char* ws, hipStream_t st)
{
    std::vector<uint32_t> jpart0((size_t)bp.njobs + 1), item0R((size_t)bp.njobs + 1), item0S((size_t)bp.njobs + 1);
    std::vector<int32_t> jbits((size_t)bp.njobs);
    std::vector<SideItem> itemsR((size_t)bp.nItemsR), itemsS((size_t)bp.nItemsS);
    uint32_t part0 = 0;
    size_t iR = 0, iS = 0;
    uint64_t cR = 0, cS = 0;
    for (int j = 0; j < bp.njobs; ++j) {
        const int b = job_bits(jobs[j], bp.cap);
        jpart0[j] = part0;
        jbits[j] = b;
        item0R[j] = (uint32_t)iR;
        item0S[j] = (uint32_t)iS;
        auto add = [&](const join_rel_t& X, std::vector<SideItem>& items, size_t& i, uint64_t& c) {
            for (int64_t beg = 0; beg < X.n; beg += kBatchChunk) {
                SideItem it{};
                it.key = X.key;
                it.rid = X.rid;
                it.beg = beg;
                it.len = (uint32_t)(X.n - beg < kBatchChunk ? X.n - beg : kBatchChunk);
                it.bits = b;
                it.part0 = part0;
                it.cnt0 = c;
                c += (uint64_t)tiles_of(it.len) << b;
                items[i++] = it;
            }
        };
        add(jobs[j].R, itemsR, iR, cR);
        add(jobs[j].S, itemsS, iS, cS);
        part0 += 1u << b;
    }
    jpart0[bp.njobs] = part0;
    item0R[bp.njobs] = (uint32_t)iR;
    item0S[bp.njobs] = (uint32_t)iS;
    hipError_t e;
    e = hipMemcpyAsync(ws + bp.off_jpart0, jpart0.data(), jpart0.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && bp.njobs > 0)
        e = hipMemcpyAsync(ws + bp.off_jbits, jbits.data(), jbits.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + bp.off_item0R, item0R.data(), item0R.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + bp.off_item0S, item0S.data(), item0S.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !itemsR.empty())
        e = hipMemcpyAsync(ws + bp.off_itemsR, itemsR.data(), itemsR.size() * sizeof(SideItem), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !itemsS.empty())
        e = hipMemcpyAsync(ws + bp.off_itemsS, itemsS.data(), itemsS.size() * sizeof(SideItem), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host tables go out of scope
    return e;
}

static JoinGeom batch_geom(const BatchPlan& bp, char* ws)
{
    JoinGeom g{};
    g.cap = (uint32_t)bp.cap;
    g.Umax = bp.Umax;
    g.single = 0;
    g.rt = reinterpret_cast<const int2*>(ws + bp.off_tupR);
    g.st = reinterpret_cast<const int2*>(ws + bp.off_tupS);
    g.part = reinterpret_cast<const PartInfo*>(ws + bp.off_info);
    g.unitStart = reinterpret_cast<const uint32_t*>(ws + bp.off_units);
    g.urec = reinterpret_cast<const uint4*>(ws + bp.off_umap);
    g.Uptr = reinterpret_cast<const uint32_t*>(ws + 8);
    g.P = (int)bp.nParts;
    g.sched = reinterpret_cast<uint32_t*>(ws + bp.off_tot) + (2 + 2 * kGroups) * bp.nParts;
    return g;
}

namespace {
// offsets[j] = first output slot of join j (its first unit's scanned offset); offsets[njobs] =
// the total.  A join without units starts where the next one does.
__global__ void job_offsets_k(const uint32_t* __restrict__ jpart0, int njobs,
                              const uint32_t* __restrict__ unitStart, const uint64_t* __restrict__ scanned,
                              int64_t Umax, const uint64_t* __restrict__ total, uint64_t* __restrict__ offsets)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > njobs) return;
    if (j == njobs) {
        offsets[j] = *total;
        return;
    }
    const uint32_t u = unitStart[jpart0[j]];
    offsets[j] = (int64_t)u < Umax ? scanned[u] : *total;
}
}  // namespace

hipError_t hash_batch_count(const BatchPlan& bp, char* ws, uint64_t* offsets, hipStream_t st)
{
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    uint64_t* total = reinterpret_cast<uint64_t*>(ws);
    uint64_t* counts = reinterpret_cast<uint64_t*>(ws + bp.off_counts);
    char* temp = ws + bp.off_temp;
    const uint32_t* jpart0 = reinterpret_cast<const uint32_t*>(ws + bp.off_jpart0);
    const int32_t* jbits = reinterpret_cast<const int32_t*>(ws + bp.off_jbits);
    const SideItem* itemsR = reinterpret_cast<const SideItem*>(ws + bp.off_itemsR);
    const SideItem* itemsS = reinterpret_cast<const SideItem*>(ws + bp.off_itemsS);
    uint32_t* totR = reinterpret_cast<uint32_t*>(ws + bp.off_tot);
    uint32_t* totS = totR + bp.nParts;
    uint32_t* baseR = reinterpret_cast<uint32_t*>(ws + bp.off_baseR);
    uint32_t* baseS = reinterpret_cast<uint32_t*>(ws + bp.off_baseS);
    uint32_t* grpR = totS + bp.nParts;
    uint32_t* grpS = grpR + kGroups * bp.nParts;
    int2* tupR = reinterpret_cast<int2*>(ws + bp.off_tupR);
    int2* tupS = reinterpret_cast<int2*>(ws + bp.off_tupS);
    uint32_t* units = reinterpret_cast<uint32_t*>(ws + bp.off_units);
    const SideItem none{};
    if (bp.nParts > 0) {
        prof::Scope pz(st, "hash.plan");
        const int64_t nz = (2 + 2 * kGroups) * bp.nParts + 4;
        zero_u32_k<<<(unsigned)ceil_div(nz, 256), 256, 0, st>>>(totR, nz);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* cntR = bp.ordered ? reinterpret_cast<uint32_t*>(ws + bp.off_cntR) : nullptr;
    uint32_t* cntS = bp.ordered ? reinterpret_cast<uint32_t*>(ws + bp.off_cntS) : nullptr;
    e = hist_side(itemsR, none, 0, 0, bp.nItemsR, bp.maxBits, totR, grpR, bp.nParts, cntR, st, true);
    if (e != hipSuccess) return e;
    e = hist_side(itemsS, none, 0, 0, bp.nItemsS, bp.maxBits, totS, grpS, bp.nParts, cntS, st, false);
    if (e != hipSuccess) return e;
    e = starts_sides(totR, baseR, grpR, totS, baseS, grpS, bp.nParts, reinterpret_cast<uint32_t*>(temp), st);
    if (e != hipSuccess) return e;
    if (bp.ordered && bp.nParts > 0) {
        prof::Scope pb(st, "hash.plan");
        const unsigned grid = (unsigned)ceil_div(bp.nParts * kGroups, 256);
        band_batch_k<<<grid, 256, 0, st>>>(itemsR, reinterpret_cast<const uint32_t*>(ws + bp.off_item0R),
                                           jpart0, bp.njobs, (uint32_t)bp.nParts, cntR);
        band_batch_k<<<grid, 256, 0, st>>>(itemsS, reinterpret_cast<const uint32_t*>(ws + bp.off_item0S),
                                           jpart0, bp.njobs, (uint32_t)bp.nParts, cntS);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    e = scatter_side(itemsR, none, 0, 0, bp.nItemsR, bp.maxBits, grpR, bp.nParts, tupR, cntR, st, true);
    if (e != hipSuccess) return e;
    e = scatter_side(itemsS, none, 0, 0, bp.nItemsS, bp.maxBits, grpS, bp.nParts, tupS, cntS, st, false);
    if (e != hipSuccess) return e;
    PartPlan q{baseR, totR, baseS, totS, jpart0, jbits, bp.njobs, 0, (uint32_t)bp.cap, (uint32_t)bp.slice};
    e = plan_parts(q, bp.nParts, reinterpret_cast<PartInfo*>(ws + bp.off_info), units,
                   reinterpret_cast<uint32_t*>(ws + 8), bp.Umax, reinterpret_cast<uint4*>(ws + bp.off_umap),
                   reinterpret_cast<uint32_t*>(temp), st);
    if (e != hipSuccess) return e;
    if (bp.Umax > 0) {
        const JoinGeom g = batch_geom(bp, ws);
        prof::Scope pc(st, "hash.count");
        join_count_k<true, false, kBatchBlock><<<(unsigned)bp.gridCount, kBatchBlock, table_lds((uint32_t)bp.cap, false), st>>>(
            g, counts, reinterpret_cast<uint64_t*>(ws + bp.off_wave), nullptr, nullptr, nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    e = exclusive_scan<uint64_t>(counts, counts, bp.Umax, total, reinterpret_cast<uint64_t*>(temp), st);
    if (e != hipSuccess) return e;
    {
        prof::Scope po(st, "hash.plan");
        job_offsets_k<<<(unsigned)ceil_div(bp.njobs + 1, 256), 256, 0, st>>>(
            jpart0, bp.njobs, units, counts, bp.Umax, total, offsets);
    }
    return hipGetLastError();
}

hipError_t hash_batch_write(const BatchPlan& bp, char* ws, int32_t* pairs, uint64_t cap, hipStream_t st)
{
    if (bp.Umax <= 0) return hipSuccess;
    hipError_t e = set_attrs();
    if (e != hipSuccess) return e;
    const JoinGeom g = batch_geom(bp, ws);
    prof::Scope pw(st, "hash.write");
    join_write_k<true, false, kBatchBlock><<<(unsigned)bp.gridWrite, kBatchBlock, table_lds((uint32_t)bp.cap, true), st>>>(
        g, reinterpret_cast<const uint64_t*>(ws + bp.off_counts),
        reinterpret_cast<const uint64_t*>(ws + bp.off_wave), reinterpret_cast<const uint64_t*>(ws),
        reinterpret_cast<int2*>(pairs), cap);
    return hipGetLastError();
}

}  // namespace jl
