// region.hip -- theta join with region pruning on gfx950 (the paper's improved theta join).
//
// Section 4.2 cuts the |T| x |S| matrix into square regions of join-key ranges, with the same
// range boundaries on both axes (k quantiles, figure "classb"), and classifies each region from
// its ranges alone (figures "greena"/"greenb"/"greenc"): in a green region every pair satisfies
// the condition, in a white region none does, and only the red regions need pair-by-pair
// evaluation on the GPU (Algorithm 3: red = the diagonal, sent to GPU_theta_join; green =
// cross join).  Here:
//   1. range:      min and max of column a over R and S;
//   2. fine bins:  2^14 power-of-two bins over [min, max], histogram of each side;
//   3. buckets:    B buckets (quantiles of the union) made of whole bins, so both sides share
//                  the same boundaries; each bucket knows its value range [lo_b, hi_b];
//   4. partition:  R and S are scattered by bucket (columns a, c, rid);
//   5. classify:   for each R bucket i and S bucket j, the pair of value ranges decides white,
//                  green or red for op_a; a condition on column c turns green into red;
//   6. red:        the red S buckets of R bucket i are contiguous: their rows become units
//                  (512 R rows x <= 8 S tiles) of the tiled nested-loop kernels;
//   7. green:      counted as |R_i| * |S rows| with no evaluation, written as a cross product.
// The result is exactly the nested-loop result: every pair is either in a red unit (evaluated),
// in a green span (holds by the range argument) or in a white span (cannot hold).
#include "region.hpp"
#include "debug.hpp"

#include "prof.hpp"
#include "scan.hpp"
#include "theta.hpp"

namespace jl {

namespace {

constexpr int kBinBits = 14;
constexpr int kBins = 1 << kBinBits;
constexpr int kBlk = 256;
constexpr int kTile = 2048;        // tuples staged per scatter step
constexpr int kRBlockRows = 512;   // R rows per unit (one wave, 8 rows per lane)
#ifndef JL_REGION_TILE
#define JL_REGION_TILE 128
#endif
constexpr int kTileRows = JL_REGION_TILE;     // S rows per unit, at least
constexpr int kMaxTiles = 8;       // S tiles per R block, at most (the tile grows beyond)
constexpr int kCrossWaves = 4;
constexpr int kSortCap = 2048;     // S rows of a bucket split in LDS for band trimming, at most
constexpr int kSortBlk = 256;

enum : int { kWhite = 0, kGreen = 1, kRed = 2 };

struct Hdr {
    uint64_t total;
    uint32_t U;     // red units
    uint32_t pad;
    int32_t lo, hi; // range of column a over R and S
    uint32_t shift; // bin = (uint32)(a - lo) >> shift
    uint32_t pad2;
};

struct BucketInfo {
    uint32_t rStart, nR;      // R rows of the bucket (bucketed order)
    uint32_t red0, red1;      // S rows evaluated pair by pair
    uint32_t gl0, gl1;        // S rows of the green span left of the red span
    uint32_t gr0, gr1;        // S rows of the green span right of it
    uint32_t tiles, ts;       // S tiles per R block and their length
    uint32_t pad0, pad1;
};

__device__ __forceinline__ uint32_t bin_of(int32_t a, const Hdr& h)
{
    return (uint32_t)((uint32_t)a - (uint32_t)h.lo) >> h.shift;
}

// ---------------------------------------------------------------------------- range + bins --
__global__ void init_k(Hdr* h, uint32_t* hist2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        h->lo = INT32_MAX;
        h->hi = INT32_MIN;
    }
    if (i < 2 * kBins) hist2[i] = 0;
}

__global__ __launch_bounds__(kBlk) void range_k(const int32_t* __restrict__ Ra, int64_t nR,
                                                const int32_t* __restrict__ Sa, int64_t nS,
                                                Hdr* h)
{
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    const int64_t n = nR + nS;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlk) {
        const int32_t a = i < nR ? Ra[i] : Sa[i - nR];
        lo = a < lo ? a : lo;
        hi = a > hi ? a : hi;
    }
    __shared__ int32_t slo, shi;
    if (threadIdx.x == 0) {
        slo = INT32_MAX;
        shi = INT32_MIN;
    }
    __syncthreads();
    atomicMin(&slo, lo);
    atomicMax(&shi, hi);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMin(&h->lo, slo);
        atomicMax(&h->hi, shi);
    }
}

__global__ void shift_k(Hdr* h)
{
    const uint32_t span = (uint32_t)h->hi - (uint32_t)h->lo;  // hi >= lo
    const int len = span ? 32 - __builtin_clz(span) : 0;
    h->shift = len > kBinBits ? (uint32_t)(len - kBinBits) : 0u;
}

__global__ __launch_bounds__(kBlk) void finehist_k(const int32_t* __restrict__ a, int64_t n,
                                                   const Hdr* __restrict__ h,
                                                   uint32_t* __restrict__ hist)
{
    __shared__ uint32_t lh[kBins];
    for (int i = threadIdx.x; i < kBins; i += kBlk) lh[i] = 0;
    __syncthreads();
    const Hdr hh = *h;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlk)
        atomicAdd(&lh[bin_of(a[i], hh)], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kBlk)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// Bucket of every bin: buckets of about (|R| + |S|) / B tuples made of whole bins, so the
// bucket ids are non-decreasing in the value; and each bucket's value range.
__global__ __launch_bounds__(1024) void buckets_k(const uint32_t* __restrict__ hR,
                                                  const uint32_t* __restrict__ hS, const Hdr* h,
                                                  int B, uint64_t N, uint16_t* __restrict__ lut,
                                                  int64_t* __restrict__ vlo,
                                                  int64_t* __restrict__ vhi)
{
    constexpr int PER = kBins / 1024;
    __shared__ uint32_t wsum[1024 / kWave + 1];
    __shared__ uint32_t first[4096], last[4096];
    const int t = threadIdx.x;
    for (int b = t; b < B; b += 1024) {
        first[b] = kBins;
        last[b] = 0;
    }
    uint32_t c[PER], s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        c[k] = hR[t * PER + k] + hS[t * PER + k];
        s += c[k];
    }
    uint32_t tot;
    uint64_t run = block_excl_scan<1024>(s, wsum, &tot);
    uint16_t id[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        uint64_t b = run * (uint64_t)B / (N ? N : 1);
        id[k] = (uint16_t)(b < (uint64_t)B ? b : (uint64_t)(B - 1));
        lut[t * PER + k] = id[k];
        run += c[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        atomicMin(&first[id[k]], (uint32_t)(t * PER + k));
        atomicMax(&last[id[k]], (uint32_t)(t * PER + k));
    }
    __syncthreads();
    const Hdr hh = *h;
    for (int b = t; b < B; b += 1024) {
        if (first[b] == (uint32_t)kBins) {  // no bin maps here: an empty bucket
            vlo[b] = 1;
            vhi[b] = 0;
        } else {
            int64_t lo = (int64_t)hh.lo + ((int64_t)first[b] << hh.shift);
            int64_t hi = (int64_t)hh.lo + (((int64_t)last[b] + 1) << hh.shift) - 1;
            vlo[b] = lo;
            vhi[b] = hi < (int64_t)hh.hi ? hi : (int64_t)hh.hi;
        }
    }
}

// ------------------------------------------------------------------------ bucket partition --
__global__ __launch_bounds__(kBlk) void bhist_k(const int32_t* __restrict__ a, int64_t n,
                                                int64_t chunk, const Hdr* __restrict__ h,
                                                const uint16_t* __restrict__ lut, int B,
                                                uint32_t* __restrict__ hist, int64_t nCh)
{
    extern __shared__ uint32_t lh[];
    for (int i = threadIdx.x; i < B; i += kBlk) lh[i] = 0;
    __syncthreads();
    const Hdr hh = *h;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlk) atomicAdd(&lh[lut[bin_of(a[i], hh)]], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += kBlk) hist[(int64_t)b * nCh + blockIdx.x] = lh[b];
}

// LDS: cursor[B] | tstart[B + 1] | sa[T] | sc[T] | sr[T] | sp[T] (uint16)
template <bool HAS_C, bool HAS_RID>
__global__ __launch_bounds__(kBlk) void bscatter_k(const int32_t* __restrict__ a,
                                                   const int32_t* __restrict__ c,
                                                   const int32_t* __restrict__ rid, int64_t n,
                                                   int64_t chunk, const Hdr* __restrict__ h,
                                                   const uint16_t* __restrict__ lut, int B,
                                                   const uint32_t* __restrict__ off, int64_t nCh,
                                                   int32_t* __restrict__ oa, int32_t* __restrict__ oc,
                                                   int32_t* __restrict__ orid)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t wsum[kBlk / kWave + 1];
    constexpr int IT = kTile / kBlk;
    uint32_t* cursor = lds;
    uint32_t* tstart = lds + B;
    int32_t* sa = reinterpret_cast<int32_t*>(tstart + B + 1);
    int32_t* sc = sa + kTile;
    int32_t* sr = sc + kTile;
    uint16_t* sp = reinterpret_cast<uint16_t*>(sr + kTile);
    const int tid = threadIdx.x;
    const Hdr hh = *h;
    for (int b = tid; b < B; b += kBlk) {
        cursor[b] = off[(int64_t)b * nCh + blockIdx.x];
        tstart[b] = 0;
    }
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    const int seg = (B + kBlk - 1) / kBlk;
    for (int64_t t0 = beg; t0 < end; t0 += kTile) {
        const int tn = (int)(end - t0 < kTile ? end - t0 : kTile);
        int32_t va[IT], vc[IT], vr[IT];
        uint32_t p[IT], rank[IT];
#pragma unroll
        for (int q = 0; q < IT; ++q) {
            const int e = q * kBlk + tid;
            const bool ok = e < tn;
            va[q] = ok ? a[t0 + e] : 0;
            vc[q] = (HAS_C && ok) ? c[t0 + e] : 0;
            vr[q] = ok ? (HAS_RID ? rid[t0 + e] : (int32_t)(t0 + e)) : 0;
        }
#pragma unroll
        for (int q = 0; q < IT; ++q) {
            const int e = q * kBlk + tid;
            p[q] = e < tn ? lut[bin_of(va[q], hh)] : 0u;
            rank[q] = e < tn ? atomicAdd(&tstart[p[q]], 1u) : 0u;
        }
        __syncthreads();
        {
            uint32_t s = 0;
            for (int i = 0; i < seg; ++i) {
                const int b = tid * seg + i;
                s += b < B ? tstart[b] : 0u;
            }
            uint32_t tot;
            uint32_t run = block_excl_scan<kBlk>(s, wsum, &tot);
            for (int i = 0; i < seg; ++i) {
                const int b = tid * seg + i;
                if (b < B) {
                    const uint32_t x = tstart[b];
                    tstart[b] = run;
                    run += x;
                }
            }
            if (tid == 0) tstart[B] = (uint32_t)tn;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < IT; ++q) {
            const int e = q * kBlk + tid;
            if (e < tn) {
                const uint32_t pos = tstart[p[q]] + rank[q];
                sa[pos] = va[q];
                if (HAS_C) sc[pos] = vc[q];
                sr[pos] = vr[q];
                sp[pos] = (uint16_t)p[q];
            }
        }
        __syncthreads();
        for (int e = tid; e < tn; e += kBlk) {
            const uint32_t b = sp[e];
            const uint32_t gidx = cursor[b] + ((uint32_t)e - tstart[b]);
            oa[gidx] = sa[e];
            if (HAS_C) oc[gidx] = sc[e];
            orid[gidx] = sr[e];
        }
        __syncthreads();
        for (int b = tid; b < B; b += kBlk) cursor[b] += tstart[b + 1] - tstart[b];
        __syncthreads();
        for (int b = tid; b < B; b += kBlk) tstart[b] = 0;
        __syncthreads();
    }
}

// --------------------------------------------------------------------------- classification --
// Class of the region (R values in [rlo, rhi]) x (S values in [slo, shi]) for R.a op S.a.
__device__ __forceinline__ int region_class(int op, int64_t w, int64_t rlo, int64_t rhi,
                                            int64_t slo, int64_t shi)
{
    switch (op) {
    case JOIN_OP_EQ:
        if (rhi < slo || shi < rlo) return kWhite;
        return (rlo == rhi && slo == shi) ? kGreen : kRed;
    case JOIN_OP_NE:
        if (rhi < slo || shi < rlo) return kGreen;
        return (rlo == rhi && slo == shi) ? kWhite : kRed;
    case JOIN_OP_LT:
        if (rhi < slo) return kGreen;
        if (rlo >= shi) return kWhite;
        return kRed;
    case JOIN_OP_LE:
        if (rhi <= slo) return kGreen;
        if (rlo > shi) return kWhite;
        return kRed;
    case JOIN_OP_GT:
        if (rlo > shi) return kGreen;
        if (rhi <= slo) return kWhite;
        return kRed;
    case JOIN_OP_GE:
        if (rlo >= shi) return kGreen;
        if (rhi < slo) return kWhite;
        return kRed;
    case JOIN_OP_BAND: {
        int64_t dmin = slo - rhi > rlo - shi ? slo - rhi : rlo - shi;
        if (dmin < 0) dmin = 0;
        const int64_t dmax = shi - rlo > rhi - slo ? shi - rlo : rhi - slo;
        if (dmin > w) return kWhite;
        if (dmax <= w) return kGreen;
        return kRed;
    }
    default: return kRed;
    }
}

__device__ __forceinline__ int wave_min_i(int v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Band joins: the S rows of every bucket of at most kSortCap rows are split three ways by a:
// low (a < vlo + w), middle, high (a > vhi - w), each keeping its c and rid, and the two split
// points are recorded.  An R bucket's band reaches into a neighbouring S bucket only through that
// bucket's near edge: a left neighbour contributes only its high rows, a right neighbour only
// its low rows, so classify_k trims the red span to them.  A bucket that is not split (larger
// than kSortCap, or narrower than 2w, where the parts would overlap) records split points that
// trim nothing.  One workgroup per bucket, the rows staged in LDS, kSplitRows per thread.
constexpr int kSplitRows = kSortCap / kSortBlk;

__global__ __launch_bounds__(kSortBlk) void bsplit_k(const uint32_t* __restrict__ offS, int64_t nChS,
                                                     uint32_t nS, int B, const int64_t* __restrict__ vlo,
                                                     const int64_t* __restrict__ vhi, int64_t w,
                                                     int32_t* __restrict__ Sa, int32_t* __restrict__ Sc,
                                                     int32_t* __restrict__ Sr, uint32_t* __restrict__ split)
{
    __shared__ int32_t ta[kSortCap], tc[kSortCap], tr[kSortCap];
    __shared__ uint32_t tmp[kSortBlk / kWave + 1];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const uint32_t s0 = offS[(int64_t)b * nChS];
    const uint32_t s1 = b + 1 < B ? offS[(int64_t)(b + 1) * nChS] : nS;
    const uint32_t n = s1 - s0;
    const int64_t lo = vlo[b], hi = vhi[b];
    if (n == 0 || n > (uint32_t)kSortCap || hi - lo < 2 * w) {  // uniform
        if (tid == 0) {
            split[2 * b] = s1;      // low rows end: the whole bucket
            split[2 * b + 1] = s0;  // high rows start: the whole bucket
        }
        return;
    }
    for (uint32_t i = tid; i < n; i += kSortBlk) {
        ta[i] = Sa[s0 + i];
        if (Sc) tc[i] = Sc[s0 + i];
        tr[i] = Sr[s0 + i];
    }
    __syncthreads();
    // thread t holds rows [t * kSplitRows, ...): category 0 low, 1 middle, 2 high
    const uint32_t r0 = (uint32_t)tid * kSplitRows;
    uint32_t cl = 0, cm = 0;
    uint8_t cat[kSplitRows];
#pragma unroll
    for (int k = 0; k < kSplitRows; ++k) {
        const uint32_t i = r0 + k;
        const int64_t a = i < n ? (int64_t)ta[i] : 0;
        cat[k] = a < lo + w ? 0 : (a > hi - w ? 2 : 1);
        if (i < n) {
            cl += cat[k] == 0;
            cm += cat[k] == 1;
        }
    }
    uint32_t L, M;
    const uint32_t pl = block_excl_scan<kSortBlk>(cl, tmp, &L);
    const uint32_t pm = block_excl_scan<kSortBlk>(cm, tmp, &M);
    uint32_t ql = pl, qm = L + pm, qh = L + M + ((r0 < n ? r0 : n) - pl - pm);
#pragma unroll
    for (int k = 0; k < kSplitRows; ++k) {
        const uint32_t i = r0 + k;
        if (i < n) {
            const uint32_t d = cat[k] == 0 ? ql++ : (cat[k] == 1 ? qm++ : qh++);
            Sa[s0 + d] = ta[i];
            if (Sc) Sc[s0 + d] = tc[i];
            Sr[s0 + d] = tr[i];
        }
    }
    if (tid == 0) {
        split[2 * b] = s0 + L;
        split[2 * b + 1] = s0 + L + M;
    }
}

// One wave per R bucket: red span, adjacent green spans, units and green pair counts.  The S
// buckets are classified by the wave's lanes together; every span end is a wave-wide min or max.
__global__ __launch_bounds__(kWave) void classify_k(const uint32_t* __restrict__ offR, int64_t nChR,
                                                    const uint32_t* __restrict__ offS, int64_t nChS,
                                                    uint32_t nR, uint32_t nS,
                                                    const int64_t* __restrict__ vlo,
                                                    const int64_t* __restrict__ vhi, int B, int op,
                                                    int64_t w, int has_c, const uint32_t* __restrict__ split,
                                                    BucketInfo* __restrict__ info,
                                                    uint32_t* __restrict__ units,
                                                    uint64_t* __restrict__ green)
{
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= B) {
        if (lane == 0) units[B] = 0;
        return;
    }
    auto rs = [&](int b) { return b < B ? offR[(int64_t)b * nChR] : nR; };
    auto ss = [&](int b) { return b < B ? offS[(int64_t)b * nChS] : nS; };
    BucketInfo bi{};
    bi.rStart = rs(i);
    bi.nR = rs(i + 1) - bi.rStart;
    const int64_t lo_i = vlo[i], hi_i = vhi[i];
    auto cls = [&](int j) -> int {
        if (ss(j + 1) == ss(j)) return -1;  // an empty S bucket: any class
        int c = region_class(op, w, lo_i, hi_i, vlo[j], vhi[j]);
        if (c == kGreen && has_c) c = kRed;  // a condition on c must still be checked
        return c;
    };
    int jr0 = B, jr1 = 0, jg0 = B, jg1 = 0;
    if (bi.nR > 0) {
        for (int j = lane; j < B; j += kWave) {
            const int c = cls(j);
            if (c == kRed) {
                jr0 = min(jr0, j);
                jr1 = max(jr1, j + 1);
            } else if (c == kGreen) {
                jg0 = min(jg0, j);
                jg1 = max(jg1, j + 1);
            }
        }
        jr0 = wave_min_i(jr0);
        jr1 = wave_max_i(jr1);
        jg0 = wave_min_i(jg0);
        jg1 = wave_max_i(jg1);
    }
    // Spans of S buckets: red [jr0, jr1), green [gl, jr0) and [jr1, gr); every bucket outside
    // them is white or empty.  Empty buckets may join any span.
    if (jr0 >= jr1) jr0 = jr1 = 0;
    int gl = jr0, gr = jr1;
    if (jg0 < jg1) {
        if (jr0 == jr1) {
            int white = 0;  // no red region: the greens must form one run without whites
            for (int j = jg0 + lane; j < jg1; j += kWave) white |= cls(j) == kWhite;
            if (!wave_max_i(white)) {
                jr0 = jr1 = gl = jg0;
                gr = jg1;
            } else {
                jr0 = gl = jg0;
                jr1 = gr = jg1;
            }
        } else {
            // greens reach from the red span to the nearest white on each side (no red lies
            // outside [jr0, jr1))
            int lw = -1, fw = B;
            for (int j = lane; j < jr0; j += kWave)
                if (cls(j) == kWhite) lw = max(lw, j);
            for (int j = jr1 + lane; j < B; j += kWave)
                if (cls(j) == kWhite) fw = min(fw, j);
            gl = wave_max_i(lw) + 1;
            gr = wave_min_i(fw);
            if (jg0 < gl || jg1 > gr) {  // greens cut off by whites: evaluate them as red
                jr0 = gl = (jg0 < jr0 ? jg0 : jr0);
                jr1 = gr = (jg1 > jr1 ? jg1 : jr1);
            }
        }
    }
    if (lane != 0) return;
    bi.red0 = ss(jr0);
    bi.red1 = jr1 > jr0 ? ss(jr1) : bi.red0;
    if (split && jr1 > jr0) {
        // band: a left neighbour of the R bucket contributes only its high rows, a right one only
        // its low rows (bsplit_k); not next to a green span, which must stay adjacent
        if (gl == jr0 && jr0 < i) bi.red0 = split[2 * jr0 + 1];
        if (gr == jr1 && jr1 - 1 > i) bi.red1 = split[2 * (jr1 - 1)];
        if (bi.red1 < bi.red0) bi.red1 = bi.red0;
    }
    bi.gl0 = ss(gl);
    bi.gl1 = jr0 > gl ? ss(jr0) : bi.gl0;
    bi.gr0 = ss(jr1);
    bi.gr1 = gr > jr1 ? ss(gr) : bi.gr0;
    const uint32_t span = bi.red1 - bi.red0;
    uint32_t tiles = 0, ts = 0;
    if (span > 0 && bi.nR > 0) {
        tiles = (span + kTileRows - 1) / kTileRows;
        if (tiles > (uint32_t)kMaxTiles) tiles = kMaxTiles;
        ts = (span + tiles - 1) / tiles;
    }
    bi.tiles = tiles;
    bi.ts = ts;
    info[i] = bi;
    const uint32_t blocks = (bi.nR + kRBlockRows - 1) / kRBlockRows;
    units[i] = blocks * tiles;
    green[2 * i] = (uint64_t)bi.nR * (bi.gl1 - bi.gl0);
    green[2 * i + 1] = (uint64_t)bi.nR * (bi.gr1 - bi.gr0);
}

__global__ void expand_k(const BucketInfo* __restrict__ info, const uint32_t* __restrict__ ustart,
                         int B, int64_t Umax, uint4* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const BucketInfo bi = info[i];
    const uint32_t u0 = ustart[i], u1 = ustart[i + 1];
    for (uint32_t u = u0; u < u1 && (int64_t)u < Umax; ++u) {
        const uint32_t k = u - u0;
        const uint32_t b = k / bi.tiles, t = k - b * bi.tiles;
        const uint32_t r0 = bi.rStart + b * kRBlockRows;
        const uint32_t rEnd = r0 + kRBlockRows < bi.rStart + bi.nR ? r0 + kRBlockRows : bi.rStart + bi.nR;
        const uint32_t s0 = bi.red0 + t * bi.ts;
        const uint32_t s1 = s0 + bi.ts < bi.red1 ? s0 + bi.ts : bi.red1;
        out[u] = make_uint4(r0, rEnd, s0, s1);
    }
}

__global__ void fill_u64_k(uint64_t* p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Green spans: item k = (R row r, side) writes |span| pairs (rid_R[r], rid_S[s]) at
// green offset + (r - rStart) * |span| + (s - span start); one wave per item.
__global__ __launch_bounds__(kCrossWaves * kWave) void cross_k(
    const BucketInfo* __restrict__ info, int B, uint32_t nR, const int32_t* __restrict__ rrid,
    const int32_t* __restrict__ srid, const uint64_t* __restrict__ goff,
    const uint64_t* __restrict__ total, int2* __restrict__ out, uint64_t cap,
    const uint64_t* __restrict__ stamp_at, uint64_t stamp)
{
    (void)nR;
    if (*total > cap || *stamp_at != stamp) return;  // see theta_write_k
    const int lane = (int)lane_id();
    const int wv = uniform((int32_t)(threadIdx.x >> 6));
    // one workgroup per (R bucket, side) item; its waves take the bucket's rows in turn, and a
    // row's pairs with the green span are written by the wave's lanes, consecutive in S
    for (int64_t item = blockIdx.x; item < 2 * (int64_t)B; item += gridDim.x) {
        const int i = (int)(item >> 1);
        const int side = (int)(item & 1);
        const BucketInfo bi = info[i];
        const uint32_t g0 = side ? bi.gr0 : bi.gl0, g1 = side ? bi.gr1 : bi.gl1;
        if (g1 <= g0 || bi.nR == 0) continue;
        const uint64_t len = g1 - g0;
        const uint64_t base0 = goff[2 * i + side];
        for (uint32_t r = (uint32_t)wv; r < bi.nR; r += kCrossWaves) {
            const int32_t rr = rrid[bi.rStart + r];
            const uint64_t base = base0 + (uint64_t)r * len;
            for (uint64_t s2 = lane; s2 < len; s2 += kWave)
                if (base + s2 < cap) out[base + s2] = make_int2(rr, srid[g0 + s2]);
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t chunk_for(int64_t n)
{
    int64_t c = ceil_div(n, 512);
    c = ceil_div(c, kTile) * kTile;
    return c < kTile ? kTile : c;
}

size_t bscatter_lds(int B) { return (size_t)(2 * B + 1) * 4 + (size_t)kTile * 14; }

}  // namespace

RegionPlan region_plan(int64_t nR, int64_t nS, int op_a, int64_t stash_k)
{
    RegionPlan pl{};
    int bits = 1;
    const int64_t n = nR + nS;
    while (bits < 12 && (n >> bits) > 1024) ++bits;
    pl.bits = bits;
    pl.B = 1 << bits;
    pl.chR = chunk_for(nR);
    pl.chS = chunk_for(nS);
    pl.nChR = nR > 0 ? ceil_div(nR, pl.chR) : 0;
    pl.nChS = nS > 0 ? ceil_div(nS, pl.chS) : 0;
    pl.Umax = (int64_t)kMaxTiles * (ceil_div(nR, kRBlockRows) + pl.B);
    const bool sel = op_a == JOIN_OP_BAND || op_a == JOIN_OP_EQ || op_a == JOIN_OP_NONE;
#ifndef JL_REGION_STASH_MULT
#define JL_REGION_STASH_MULT 2
#endif
    pl.K = sel && stash_k > 0 ? stash_k * JL_REGION_STASH_MULT : 0;
    pl.nOff = pl.Umax + 2 * (int64_t)pl.B;
    size_t off = 256;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    pl.off_hist2 = take((size_t)2 * kBins * 4);
    pl.off_lut = take((size_t)kBins * 2);
    pl.off_vlo = take((size_t)pl.B * 8);
    pl.off_vhi = take((size_t)pl.B * 8);
    pl.off_hR = take((size_t)pl.B * pl.nChR * 4);
    pl.off_hS = take((size_t)pl.B * pl.nChS * 4);
    pl.off_Ra = take((size_t)nR * 4);
    pl.off_Rc = take((size_t)nR * 4);
    pl.off_Rr = take((size_t)nR * 4);
    pl.off_Sa = take((size_t)nS * 4);
    pl.off_Sc = take((size_t)nS * 4);
    pl.off_Sr = take((size_t)nS * 4);
    pl.off_info = take((size_t)pl.B * sizeof(BucketInfo));
    pl.off_split = take((size_t)pl.B * 8);
    pl.off_units = take((size_t)(pl.B + 1) * 4);
    pl.off_table = take((size_t)pl.Umax * sizeof(uint4));
    pl.off_counts = take((size_t)pl.nOff * 8);
    pl.off_stash = take((size_t)pl.Umax * pl.K * 8);
    size_t temp = scan_temp_elems<uint64_t>(pl.nOff) * 8;
    const size_t t1 = scan_temp_elems<uint32_t>((int64_t)pl.B * pl.nChR) * 4;
    const size_t t2 = scan_temp_elems<uint32_t>((int64_t)pl.B * pl.nChS) * 4;
    const size_t t3 = scan_temp_elems<uint32_t>(pl.B + 1) * 4;
    temp = temp > t1 ? temp : t1;
    temp = temp > t2 ? temp : t2;
    temp = temp > t3 ? temp : t3;
    pl.off_temp = take(temp + 8);
    pl.off_dbg = take(JL_DEBUG ? (size_t)(pl.Umax > 0 ? pl.Umax : 1) * 8 : 0);  // last (checking build)
    pl.bytes = off;
    pl.stamp = plan_stamp({JOIN_KIND_THETA_REGION, nR, nS, op_a, pl.bits, pl.B, pl.chR, pl.chS, pl.Umax,
                           pl.K, pl.nOff, (int64_t)pl.bytes});
    return pl;
}

static bool g_region_attr = false;

static hipError_t region_attrs()
{
    if (g_region_attr) return hipSuccess;
    const int big = 160 * 1024 - 4096;
    hipError_t e;
    e = hipFuncSetAttribute((const void*)bscatter_k<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)bscatter_k<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)bscatter_k<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)bscatter_k<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    g_region_attr = true;
    return hipSuccess;
}

static ThetaUnitArgs unit_args(const RegionPlan& pl, char* ws)
{
    ThetaUnitArgs a{};
    a.Ra = reinterpret_cast<const int32_t*>(ws + pl.off_Ra);
    a.Rc = reinterpret_cast<const int32_t*>(ws + pl.off_Rc);
    a.Rrid = reinterpret_cast<const int32_t*>(ws + pl.off_Rr);
    a.Sa = reinterpret_cast<const int32_t*>(ws + pl.off_Sa);
    a.Sc = reinterpret_cast<const int32_t*>(ws + pl.off_Sc);
    a.Srid = reinterpret_cast<const int32_t*>(ws + pl.off_Sr);
    a.units = reinterpret_cast<const uint4*>(ws + pl.off_table);
    a.Uptr = reinterpret_cast<const uint32_t*>(ws + 8);
    a.Umax = pl.Umax;
    a.stash = pl.K > 0 ? reinterpret_cast<int2*>(ws + pl.off_stash) : nullptr;
    a.K = pl.K;
    a.nOff = pl.nOff;
    a.stamp_at = reinterpret_cast<uint64_t*>(ws + kStampOffset);
    a.stamp = pl.stamp;
    a.dbg = JL_DEBUG ? reinterpret_cast<uint64_t*>(ws + pl.off_dbg) : nullptr;
    return a;
}

static hipError_t part_side(const RegionPlan& pl, const join_rel_t& X, bool has_c, int64_t ch,
                            int64_t nCh, size_t off_h, size_t off_a, size_t off_c, size_t off_r,
                            char* ws, hipStream_t st, const char* name)
{
    const Hdr* h = reinterpret_cast<const Hdr*>(ws);
    const uint16_t* lut = reinterpret_cast<const uint16_t*>(ws + pl.off_lut);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + off_h);
    {
        prof::Scope ps(st, name);
        bhist_k<<<(unsigned)nCh, kBlk, (size_t)pl.B * 4, st>>>(X.key, X.n, ch, h, lut, pl.B, hist, nCh);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan<uint32_t>(hist, hist, (int64_t)pl.B * nCh, nullptr,
                                 reinterpret_cast<uint32_t*>(ws + pl.off_temp), st);
    if (e != hipSuccess) return e;
    int32_t* oa = reinterpret_cast<int32_t*>(ws + off_a);
    int32_t* oc = reinterpret_cast<int32_t*>(ws + off_c);
    int32_t* orr = reinterpret_cast<int32_t*>(ws + off_r);
    const size_t lds = bscatter_lds(pl.B);
    prof::Scope ps(st, name);
    if (has_c) {
        if (X.rid) bscatter_k<true, true><<<(unsigned)nCh, kBlk, lds, st>>>(X.key, X.key2, X.rid, X.n, ch, h, lut, pl.B, hist, nCh, oa, oc, orr);
        else bscatter_k<true, false><<<(unsigned)nCh, kBlk, lds, st>>>(X.key, X.key2, X.rid, X.n, ch, h, lut, pl.B, hist, nCh, oa, oc, orr);
    } else {
        if (X.rid) bscatter_k<false, true><<<(unsigned)nCh, kBlk, lds, st>>>(X.key, X.key2, X.rid, X.n, ch, h, lut, pl.B, hist, nCh, oa, oc, orr);
        else bscatter_k<false, false><<<(unsigned)nCh, kBlk, lds, st>>>(X.key, X.key2, X.rid, X.n, ch, h, lut, pl.B, hist, nCh, oa, oc, orr);
    }
    return hipGetLastError();
}

hipError_t region_count(const RegionPlan& pl, const join_rel_t& R, const join_rel_t& S,
                        const join_pred_t& p, char* ws, hipStream_t st, uint64_t* pub)
{
    hipError_t e = region_attrs();
    if (e != hipSuccess) return e;
    Hdr* h = reinterpret_cast<Hdr*>(ws);
    uint32_t* hist2 = reinterpret_cast<uint32_t*>(ws + pl.off_hist2);
    const bool has_c = p.op_c != JOIN_OP_NONE;
    {
        prof::Scope ps(st, "region.bucket");
        init_k<<<(unsigned)ceil_div(2 * kBins, 256), 256, 0, st>>>(h, hist2);
        range_k<<<512, kBlk, 0, st>>>(R.key, R.n, S.key, S.n, h);
        shift_k<<<1, 1, 0, st>>>(h);
        finehist_k<<<256, kBlk, 0, st>>>(R.key, R.n, h, hist2);
        finehist_k<<<256, kBlk, 0, st>>>(S.key, S.n, h, hist2 + kBins);
        buckets_k<<<1, 1024, 0, st>>>(hist2, hist2 + kBins, h, pl.B, (uint64_t)(R.n + S.n),
                                      reinterpret_cast<uint16_t*>(ws + pl.off_lut),
                                      reinterpret_cast<int64_t*>(ws + pl.off_vlo),
                                      reinterpret_cast<int64_t*>(ws + pl.off_vhi));
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = part_side(pl, R, has_c, pl.chR, pl.nChR, pl.off_hR, pl.off_Ra, pl.off_Rc, pl.off_Rr, ws, st, "region.partition.R");
    if (e != hipSuccess) return e;
    e = part_side(pl, S, has_c, pl.chS, pl.nChS, pl.off_hS, pl.off_Sa, pl.off_Sc, pl.off_Sr, ws, st, "region.partition.S");
    if (e != hipSuccess) return e;
    uint32_t* split = p.op_a == JOIN_OP_BAND ? reinterpret_cast<uint32_t*>(ws + pl.off_split) : nullptr;
    if (split) {
        prof::Scope ps(st, "region.split");
        bsplit_k<<<(unsigned)pl.B, kSortBlk, 0, st>>>(
            reinterpret_cast<const uint32_t*>(ws + pl.off_hS), pl.nChS, (uint32_t)S.n, pl.B,
            reinterpret_cast<const int64_t*>(ws + pl.off_vlo), reinterpret_cast<const int64_t*>(ws + pl.off_vhi),
            (int64_t)p.w, reinterpret_cast<int32_t*>(ws + pl.off_Sa),
            has_c ? reinterpret_cast<int32_t*>(ws + pl.off_Sc) : nullptr,
            reinterpret_cast<int32_t*>(ws + pl.off_Sr), split);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    uint32_t* units = reinterpret_cast<uint32_t*>(ws + pl.off_units);
    uint64_t* counts = reinterpret_cast<uint64_t*>(ws + pl.off_counts);
    BucketInfo* info = reinterpret_cast<BucketInfo*>(ws + pl.off_info);
    {
        prof::Scope ps(st, "region.classify");
        fill_u64_k<<<256, 256, 0, st>>>(counts, pl.Umax, 0);
        classify_k<<<(unsigned)(pl.B + 1), kWave, 0, st>>>(
            reinterpret_cast<const uint32_t*>(ws + pl.off_hR), pl.nChR,
            reinterpret_cast<const uint32_t*>(ws + pl.off_hS), pl.nChS, (uint32_t)R.n,
            (uint32_t)S.n, reinterpret_cast<const int64_t*>(ws + pl.off_vlo),
            reinterpret_cast<const int64_t*>(ws + pl.off_vhi), pl.B, p.op_a,
            p.op_a == JOIN_OP_BAND ? (int64_t)p.w : 0, has_c ? 1 : 0, split, info, units,
            counts + pl.Umax);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan<uint32_t>(units, units, pl.B + 1, &h->U,
                                 reinterpret_cast<uint32_t*>(ws + pl.off_temp), st);
    if (e != hipSuccess) return e;
    {
        prof::Scope ps(st, "region.classify");
        expand_k<<<(unsigned)ceil_div(pl.B, 128), 128, 0, st>>>(
            info, units, pl.B, pl.Umax, reinterpret_cast<uint4*>(ws + pl.off_table));
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = theta_count_units(unit_args(pl, ws), p, counts, st);
    if (e != hipSuccess) return e;
    return exclusive_scan<uint64_t>(counts, counts, pl.nOff, &h->total,
                                    reinterpret_cast<uint64_t*>(ws + pl.off_temp), st, pub);
}

hipError_t region_write(const RegionPlan& pl, const join_rel_t& R, const join_rel_t& S,
                        const join_pred_t& p, char* ws, int32_t* pairs, uint64_t cap,
                        hipStream_t st)
{
    (void)S;
    const uint64_t* offsets = reinterpret_cast<const uint64_t*>(ws + pl.off_counts);
    const uint64_t* total = reinterpret_cast<const uint64_t*>(ws);
    hipError_t e = theta_write_units(unit_args(pl, ws), p, offsets, total, pairs, cap, st);
    if (e != hipSuccess) return e;
    if (p.op_c == JOIN_OP_NONE) {  // green spans exist only without a condition on c
        prof::Scope ps(st, "region.cross");
        cross_k<<<1024, kCrossWaves * kWave, 0, st>>>(
            reinterpret_cast<const BucketInfo*>(ws + pl.off_info), pl.B, (uint32_t)R.n,
            reinterpret_cast<const int32_t*>(ws + pl.off_Rr),
            reinterpret_cast<const int32_t*>(ws + pl.off_Sr), offsets + pl.Umax, total,
            reinterpret_cast<int2*>(pairs), cap, reinterpret_cast<const uint64_t*>(ws + kStampOffset),
            pl.stamp);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace jl
