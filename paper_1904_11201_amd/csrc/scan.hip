// scan.hip -- device exclusive prefix sums (uint32 and uint64), reduce-then-scan.
//
// This is the "scan" of count -> scan -> write: the per-work-unit match counts become exact
// output offsets on the device (the compaction the paper leaves unspecified when it says the
// per-thread results are "summed", Section 3.3.1), and radix histograms become partition
// offsets.  Three launches for n > kSingleTiles tiles: per-tile sums, a single-workgroup scan of
// the tile sums, and a per-tile scan seeded with its prefix.  Fewer tiles use one launch.
#include "scan.hpp"

#include "prof.hpp"

namespace jl {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;  // 4096 values per workgroup
// Up to this many tiles one workgroup scans them in turn: cheaper than three launches.
constexpr int64_t kSingleTiles = 4;

template <typename T>
__device__ __forceinline__ T wave_scan_t(T x);
template <>
__device__ __forceinline__ uint32_t wave_scan_t<uint32_t>(uint32_t x) { return wave_incl_scan(x); }
template <>
__device__ __forceinline__ uint64_t wave_scan_t<uint64_t>(uint64_t x) { return wave_incl_scan64(x); }

// Block exclusive scan of one T per thread (kScanBlock threads); returns prefix, sets *sum.
template <typename T>
__device__ __forceinline__ T block_scan_t(T x, T* lds, T* sum)
{
    constexpr int W = kScanBlock / kWave;
    const int wv = threadIdx.x / kWave;
    const T inc = wave_scan_t<T>(x);
    if (lane_id() == kWave - 1) lds[wv] = inc;
    __syncthreads();
    T before = 0, s = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        T t = lds[i];
        before += (i < wv) ? t : (T)0;
        s += t;
    }
    __syncthreads();
    *sum = s;
    return before + inc - x;
}

// Per-tile sums.
template <typename T>
__global__ __launch_bounds__(kScanBlock) void tile_sum_k(const T* __restrict__ in, int64_t n,
                                                         T* __restrict__ sums)
{
    __shared__ T lds[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
        s += (i < n) ? in[i] : (T)0;
    }
    T tot;
    block_scan_t<T>(s, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scan one tile (kScanTile values) starting at `base` with carry-in `carry`; items are kept in
// registers in blocked order so that each thread owns kScanItems consecutive values.
template <typename T>
__device__ __forceinline__ T scan_tile(const T* __restrict__ in, T* __restrict__ out, int64_t n,
                                       int64_t base, T carry, T* lds)
{
    T v[kScanItems];
    const int64_t my = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = (my + k < n) ? in[my + k] : (T)0;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    T tot;
    T run = carry + block_scan_t<T>(s, lds, &tot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        T x = v[k];
        if (my + k < n) out[my + k] = run;
        run += x;
    }
    return carry + tot;
}

// Single workgroup: exclusive scan of all n values in tiles, carrying the running sum.
// pub: NULL, or a pinned host slot that also receives the total.
template <typename T>
__global__ __launch_bounds__(kScanBlock) void scan_single_k(const T* __restrict__ in,
                                                            T* __restrict__ out, int64_t n,
                                                            T* __restrict__ total, uint64_t* pub)
{
    __shared__ T lds[kScanBlock / kWave];
    T carry = 0;
    for (int64_t base = 0; base < n; base += kScanTile) carry = scan_tile<T>(in, out, n, base, carry, lds);
    if (threadIdx.x == 0 && total) *total = carry;
    if (threadIdx.x == 0 && pub) publish_total(pub, (uint64_t)carry);
}

// Per-tile scan seeded with the scanned tile sums.
template <typename T>
__global__ __launch_bounds__(kScanBlock) void scan_apply_k(const T* __restrict__ in,
                                                           T* __restrict__ out, int64_t n,
                                                           const T* __restrict__ prefix)
{
    __shared__ T lds[kScanBlock / kWave];
    scan_tile<T>(in, out, n, (int64_t)blockIdx.x * kScanTile, prefix[blockIdx.x], lds);
}

}  // namespace

template <typename T>
size_t scan_temp_elems(int64_t n)
{
    int64_t tiles = ceil_div(n, kScanTile);
    return tiles <= kSingleTiles ? 0 : (size_t)tiles;
}

template <typename T>
hipError_t exclusive_scan(const T* in, T* out, int64_t n, T* total, T* temp, hipStream_t st,
                         uint64_t* pub)
{
    if (n < 0) n = 0;
    prof::Scope ps(st, sizeof(T) == 8 ? "scan.u64" : "scan.u32");
    int64_t tiles = ceil_div(n, kScanTile);
    if (tiles <= kSingleTiles) {  // also n == 0: writes *total = 0 without a memset node
        scan_single_k<T><<<1, kScanBlock, 0, st>>>(in, out, n, total, pub);
        return hipGetLastError();
    }
    // Tile sums are computed from `in` before any output is written, so in == out is safe:
    // scan_apply reads a tile only in the workgroup that writes it.
    tile_sum_k<T><<<(unsigned)tiles, kScanBlock, 0, st>>>(in, n, temp);
    scan_single_k<T><<<1, kScanBlock, 0, st>>>(temp, temp, tiles, total, pub);
    scan_apply_k<T><<<(unsigned)tiles, kScanBlock, 0, st>>>(in, out, n, temp);
    return hipGetLastError();
}

template size_t scan_temp_elems<uint32_t>(int64_t);
template size_t scan_temp_elems<uint64_t>(int64_t);
template hipError_t exclusive_scan<uint32_t>(const uint32_t*, uint32_t*, int64_t, uint32_t*,
                                             uint32_t*, hipStream_t, uint64_t*);
template hipError_t exclusive_scan<uint64_t>(const uint64_t*, uint64_t*, int64_t, uint64_t*,
                                             uint64_t*, hipStream_t, uint64_t*);

}  // namespace jl
