// theta.hip -- tiled nested-loop theta join on gfx950: count pass and write pass.
//
// The paper evaluates theta joins (and its nested-loop equi join) by giving each GPU thread a
// rectangle of the |T| x |S| pair matrix (Section 3.3.1, equations NBS/NBT/IDS/IDT; Section
// 4.2: the GPU theta join uses the same thread organisation).  Here the matrix is cut into
// work units of (R block of 64*kRB rows) x (S tile of TS rows), one wave per unit:
//   - each lane keeps kRB R rows in VGPRs (precomputed predicate constants),
//   - S values are wave-uniform: loaded with scalar loads and used as SGPR operands,
//   - one v_cmp per (S row, R row) produces a 64-lane mask in SGPRs.
// Selective predicates (BAND, EQ) first OR the masks of the first condition over a group of 8
// S rows; only a group with a hit is evaluated exactly (short-circuit AND).  Predicates that
// hold for a large share of pairs are counted directly with per-lane counters.
//
// Both passes walk the same units in the same order, so the write pass fills exactly
// [offset[u], offset[u] + count[u]) for each unit: the exact result size of Section 3.3.3
// with no over-allocation.
#include "theta.hpp"
#include "debug.hpp"

#include "prof.hpp"
#include "scan.hpp"

namespace jl {

namespace {

constexpr int kThetaBlock = 256;                    // 4 waves, one unit each
constexpr int kWavesPerBlock = kThetaBlock / kWave;
constexpr int kRB = 8;                              // R rows per lane
constexpr int64_t kRowsPerWave = (int64_t)kWave * kRB;
constexpr int kSGroup = 8;                          // S rows per scalar-load group

struct ThetaGeom {
    const int32_t* Ra;
    const int32_t* Rc;
    const int32_t* Rrid;
    int64_t nR;
    const int32_t* Sa;
    const int32_t* Sc;
    const int32_t* Srid;
    int64_t nS;
    int64_t w;
    int64_t TS;   // S rows per tile
    int64_t nSt;  // S tiles
    int64_t U;    // units = R blocks * S tiles
    int2* stash;  // [U][K] matches kept by the count pass (selective predicates), or NULL
    int64_t K;
    // Explicit unit table (region-pruned theta join): unit u covers R rows [x, y) and S rows
    // [z, w) of the arrays above; NULL means the dense grid of R blocks x S tiles.
    const uint4* units;
    const uint32_t* Uptr;  // device unit count when units != NULL (clamped to U)
    int64_t nOff;          // entries of the offsets array the write pass reads
    uint64_t* stamp_at;    // plan stamp in the workspace header: recorded by the count pass,
    uint64_t stamp;        // checked by the write pass
    uint64_t* dbg;         // checking build: pairs written per unit (NULL: not counted)
};

// Per-R-row constants of op_a.  BAND keeps [lo, lo + wid] with lo = max(a - w, INT32_MIN),
// hi = min(a + w, INT32_MAX), wid = hi - lo (< 2^32): s is in the band iff
// (uint32)(s - lo) <= wid, exact for every int32 s (no wrap-around can land inside).
template <int OP>
__device__ __forceinline__ void prep_a(int32_t a, int64_t w, int32_t& x0, uint32_t& x1)
{
    if constexpr (OP == JOIN_OP_BAND) {
        int64_t lo = (int64_t)a - w, hi = (int64_t)a + w;
        lo = lo < INT32_MIN ? INT32_MIN : lo;
        hi = hi > INT32_MAX ? INT32_MAX : hi;
        x0 = (int32_t)lo;
        x1 = (uint32_t)(hi - lo);
    } else {
        x0 = a;
        x1 = 0;
    }
}

// op(r, s) with r from R (per lane) and s from S (wave-uniform).
template <int OP>
__device__ __forceinline__ bool holds(int32_t x0, uint32_t x1, int32_t s)
{
    if constexpr (OP == JOIN_OP_NONE) return true;
    if constexpr (OP == JOIN_OP_EQ) return x0 == s;
    if constexpr (OP == JOIN_OP_NE) return x0 != s;
    if constexpr (OP == JOIN_OP_LT) return x0 < s;
    if constexpr (OP == JOIN_OP_LE) return x0 <= s;
    if constexpr (OP == JOIN_OP_GT) return x0 > s;
    if constexpr (OP == JOIN_OP_GE) return x0 >= s;
    if constexpr (OP == JOIN_OP_BAND) return (uint32_t)(s - x0) <= x1;
    return false;
}

template <int OPA>
constexpr bool selective() { return OPA == JOIN_OP_BAND || OPA == JOIN_OP_EQ; }

struct RRows {
    int32_t x0[kRB];
    uint32_t x1[kRB];
    int32_t xc[kRB];
};

// A copy of the R constants the compiler cannot prove equal to the originals.  The rare exact
// path of a selective group evaluates on this copy, so the filter's 64 differences die right
// after the minimum instead of being kept alive (and spilled) for reuse.
__device__ __forceinline__ RRows opaque_copy(const RRows& a)
{
    RRows b = a;
#pragma unroll
    for (int r = 0; r < kRB; ++r) asm volatile("" : "+v"(b.x0[r]), "+v"(b.x1[r]), "+v"(b.xc[r]));
    return b;
}

template <int OPA, int OPC>
__device__ __forceinline__ void load_r(const ThetaGeom& g, int64_t r0, int64_t rEnd, int lane,
                                       RRows& rr)
{
#pragma unroll
    for (int r = 0; r < kRB; ++r) {
        const int64_t row = r0 + r * kWave + lane;
        const bool valid = row < rEnd;
        const int32_t a = valid ? g.Ra[row] : 0;
        prep_a<OPA>(a, g.w, rr.x0[r], rr.x1[r]);
        if constexpr (OPC != JOIN_OP_NONE) rr.xc[r] = valid ? g.Rc[row] : 0;
        else rr.xc[r] = 0;
    }
}

// Unit u: R rows [r0, rEnd) (at most 64 * kRB of them) and S rows [s0, s1).
__device__ __forceinline__ void unit_of(const ThetaGeom& g, int64_t u, int64_t& r0, int64_t& rEnd,
                                        int64_t& s0, int64_t& s1)
{
    if (g.units) {  // u is uniform: scalar loads, so the unit's bounds live in SGPRs
        const cptr<uint32_t> q = as_const(reinterpret_cast<const uint32_t*>(g.units)) + 4 * u;
        r0 = q[0];
        rEnd = q[1];
        s0 = q[2];
        s1 = q[3];
        return;
    }
    const int64_t rb = u / g.nSt;
    const int64_t st = u - rb * g.nSt;
    r0 = rb * kRowsPerWave;
    rEnd = r0 + kRowsPerWave < g.nR ? r0 + kRowsPerWave : g.nR;
    s0 = st * g.TS;
    s1 = s0 + g.TS < g.nS ? s0 + g.TS : g.nS;
}

__device__ __forceinline__ int64_t unit_count(const ThetaGeom& g)
{
    if (!g.units) return g.U;
    const int64_t U = *g.Uptr;
    return U < g.U ? U : g.U;
}

// Evaluate one S row against the wave's kRB R rows exactly and emit the matches in (r, lane)
// order at base, base+1, ...: slots below `cap` are written to `out`, and base advances by the
// number of matches either way (so a capacity-limited destination still counts exactly).
template <int OPA, int OPC>
__device__ __forceinline__ void emit_row(const RRows& rr, const int32_t (&rid)[kRB],
                                         const uint64_t (&vm)[kRB], int32_t sa, int32_t sc,
                                         int32_t srid, uint64_t& base, int2* __restrict__ out,
                                         uint64_t cap, int lane)
{
#pragma unroll
    for (int r = 0; r < kRB; ++r) {
        // one ballot per condition: each compare lands in a lane mask and the masks are ANDed
        // on the scalar unit (a ballot of the combined bool would first widen it to a VGPR)
        uint64_t m = ballot(holds<OPA>(rr.x0[r], rr.x1[r], sa)) & vm[r];
        if constexpr (OPC != JOIN_OP_NONE) m &= ballot(holds<OPC>(rr.xc[r], 0u, sc));
        if (m) {
            if ((m >> lane) & 1ull) {
                const uint64_t slot = base + mask_rank(m);
                if (slot < cap) out[slot] = make_int2(rid[r], srid);
            }
            base += (uint64_t)__popcll(m);
        }
    }
}

__device__ __forceinline__ void load_rids(const ThetaGeom& g, int64_t r0, int64_t rEnd, int lane,
                                          int32_t (&rid)[kRB], uint64_t (&vm)[kRB])
{
#pragma unroll
    for (int r = 0; r < kRB; ++r) {
        const int64_t row = r0 + r * kWave + lane;
        const bool valid = row < rEnd;
        rid[r] = valid ? (g.Rrid ? g.Rrid[row] : (int32_t)row) : 0;
        vm[r] = ballot(valid);
    }
}

// Selective predicates: filter 8 S rows at a time on op_a alone; a group that may hold a pair is
// evaluated exactly and its pairs go to `out` (capacity `cap`) starting at `base`.  The fast
// filter keeps only op_a's constants per R row live.  The rare exact path walks one R row
// at a time and reloads that row's c value and rid (cache-resident), so it needs only a few
// registers beyond the filter's and the filter keeps its occupancy.  Pairs of a group are
// emitted in (R row r, S row j, lane) order.
template <int OPA, int OPC>
__device__ __forceinline__ void sweep_selective(const ThetaGeom& g, const RRows& rr, int64_t r0,
                                                int64_t rEnd, int64_t s0, int64_t s1, uint64_t& base,
                                                int2* __restrict__ out, uint64_t cap, int lane)
{
    const cptr<int32_t> Sa = as_const(g.Sa);
    const cptr<int32_t> Sc = as_const(g.Sc);
    const cptr<int32_t> Srid = as_const(g.Srid);
    auto exact = [&](int64_t jb, int64_t je) {
        const RRows q = opaque_copy(rr);
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
            const int64_t row = r0 + r * kWave + lane;
            const bool valid = row < rEnd;
            const uint64_t vm = ballot(valid);
            if (!vm) continue;
            const int32_t xc = (OPC != JOIN_OP_NONE && valid) ? g.Rc[row] : 0;
            const int32_t rid = valid ? (g.Rrid ? g.Rrid[row] : (int32_t)row) : 0;
#pragma unroll 1
            for (int64_t j = jb; j < je; ++j) {
                const int32_t sc = (OPC != JOIN_OP_NONE) ? Sc[j] : 0;
                const uint64_t m =
                    ballot(holds<OPA>(q.x0[r], q.x1[r], Sa[j]) && holds<OPC>(xc, 0u, sc)) & vm;
                if (m) {
                    if ((m >> lane) & 1ull) {
                        const uint64_t slot = base + mask_rank(m);
                        if (slot < cap) out[slot] = make_int2(rid, Srid ? Srid[j] : (int32_t)j);
                    }
                    base += (uint64_t)__popcll(m);
                }
            }
        }
    };
    // A pair can hold only if s - x0 <= x1 for its R row (equality: s - x0 == 0), and x1 <= wmax
    // for every row (rows clamped at the ends of the int32 range have narrower bands), so a
    // group with min(s - x0) over its 64 pairs above wmax holds no pair.  The running minimum
    // costs one subtract per pair, one three-input min per two pairs and one move per S row, with
    // one compare per group; two minima alternate so consecutive mins do not wait on each other.
    const uint32_t wmax = OPA == JOIN_OP_BAND ? (uint32_t)(2 * (int64_t)g.w) : 0u;
    int64_t j = s0;
    for (; j + kSGroup <= s1; j += kSGroup) {
        int32_t sa[kSGroup];
#pragma unroll
        for (int k = 0; k < kSGroup; ++k) sa[k] = Sa[j + k];
        uint32_t m0 = ~0u, m1 = ~0u;
#pragma unroll
        for (int k = 0; k < kSGroup; ++k) {
            // the S value is moved into a vector register once for its 8 subtracts: a subtract
            // of two vector registers issues faster than one that reads a scalar register
            int32_t sv;
            asm volatile("v_mov_b32 %0, %1" : "=v"(sv) : "s"(sa[k]));
#pragma unroll
            for (int r = 0; r < kRB; r += 2) {
                const uint32_t d0 = (uint32_t)(sv - rr.x0[r]);
                const uint32_t d1 = (uint32_t)(sv - rr.x0[r + 1]);
                if (k & 1) m1 = min(min(m1, d0), d1);
                else m0 = min(min(m0, d0), d1);
            }
        }
        if (ballot(min(m0, m1) <= wmax)) exact(j, j + kSGroup);
    }
    if (j < s1) exact(j, s1);
}

// ------------------------------------------------------------------------------- count pass --
// Selective predicates also keep up to K matches of the unit in a per-unit stash, so the write
// pass of a unit with at most K matches is a copy instead of a second sweep.
// DENSE (region units of a selective predicate): the units were chosen because their value
// ranges are close, so most 8-row groups hold a match and the group filter would send nearly
// every group down its exact path.  Instead every S row is evaluated exactly against the wave's R rows
// (both columns and rids kept in registers), one ballot per R row.
template <int OPA, int OPC, bool DENSE = false>
__global__ __launch_bounds__(kThetaBlock) void theta_count_k(ThetaGeom g,
                                                             uint64_t* __restrict__ counts)
{
    const int lane = (int)lane_id();
    if (g.stamp_at && blockIdx.x == 0 && threadIdx.x == 0) *g.stamp_at = g.stamp;  // for the write pass
    const int64_t u = (int64_t)blockIdx.x * kWavesPerBlock + uniform((int32_t)(threadIdx.x >> 6));
    if (u >= unit_count(g)) return;
    {
        int64_t r0, rEnd, s0, s1;
        unit_of(g, u, r0, rEnd, s0, s1);
        RRows rr;
        load_r<OPA, selective<OPA>() && !DENSE ? JOIN_OP_NONE : OPC>(g, r0, rEnd, lane, rr);

        if constexpr (selective<OPA>() && DENSE) {
            int32_t rid[kRB];
            uint64_t vm[kRB];
            load_rids(g, r0, rEnd, lane, rid, vm);
            const cptr<int32_t> Sa = as_const(g.Sa);
            const cptr<int32_t> Sc = as_const(g.Sc);
            const cptr<int32_t> Srid = as_const(g.Srid);
            uint64_t n = 0;
            int2* st = g.stash ? g.stash + u * g.K : nullptr;
            const uint64_t kcap = st ? (uint64_t)g.K : 0ull;
            // Region units always come with the bucketed rid column (positions when the input
            // has none), so the rids load unconditionally with the other columns.
            // 8 S rows' scalar loads in flight together, the next group's while this one is
            // evaluated
            int64_t j = s0;
            int32_t na[kSGroup], nc[kSGroup], nr[kSGroup];
            auto fetch = [&](int64_t j0) {
#pragma unroll
                for (int k = 0; k < kSGroup; ++k) {
                    na[k] = Sa[j0 + k];
                    nc[k] = (OPC != JOIN_OP_NONE) ? Sc[j0 + k] : 0;
                    nr[k] = Srid[j0 + k];
                }
            };
            if (j + kSGroup <= s1) fetch(j);
            for (; j + kSGroup <= s1; j += kSGroup) {
                int32_t sa[kSGroup], sc[kSGroup], sr[kSGroup];
#pragma unroll
                for (int k = 0; k < kSGroup; ++k) {
                    sa[k] = na[k];
                    sc[k] = nc[k];
                    sr[k] = nr[k];
                }
                if (j + 2 * kSGroup <= s1) fetch(j + kSGroup);
#pragma unroll
                for (int k = 0; k < kSGroup; ++k)
                    emit_row<OPA, OPC>(rr, rid, vm, sa[k], sc[k], sr[k], n, st, kcap, lane);
            }
            for (; j < s1; ++j) {
                const int32_t sc = (OPC != JOIN_OP_NONE) ? Sc[j] : 0;
                emit_row<OPA, OPC>(rr, rid, vm, Sa[j], sc, Srid[j], n, st, kcap, lane);
            }
            if (lane == 0) counts[u] = n;
        } else if constexpr (selective<OPA>()) {
            uint64_t n = 0;
            int2* st = g.stash ? g.stash + u * g.K : nullptr;
            sweep_selective<OPA, OPC>(g, rr, r0, rEnd, s0, s1, n, st, st ? (uint64_t)g.K : 0ull,
                                      lane);
            if (lane == 0) counts[u] = n;
        } else {
            const cptr<int32_t> Sa = as_const(g.Sa);
            const cptr<int32_t> Sc = as_const(g.Sc);
            uint32_t cnt[kRB];
#pragma unroll
            for (int r = 0; r < kRB; ++r) cnt[r] = 0;
            int64_t j = s0;
            for (; j + kSGroup <= s1; j += kSGroup) {
                int32_t sa[kSGroup], sc[kSGroup];
#pragma unroll
                for (int k = 0; k < kSGroup; ++k) {
                    sa[k] = Sa[j + k];
                    sc[k] = (OPC != JOIN_OP_NONE) ? Sc[j + k] : 0;
                }
#pragma unroll
                for (int k = 0; k < kSGroup; ++k)
#pragma unroll
                    for (int r = 0; r < kRB; ++r)
                        cnt[r] += (holds<OPA>(rr.x0[r], rr.x1[r], sa[k]) &&
                                   holds<OPC>(rr.xc[r], 0u, sc[k])) ? 1u : 0u;
            }
            for (; j < s1; ++j) {
                const int32_t sa = Sa[j];
                const int32_t sc = (OPC != JOIN_OP_NONE) ? Sc[j] : 0;
#pragma unroll
                for (int r = 0; r < kRB; ++r)
                    cnt[r] += (holds<OPA>(rr.x0[r], rr.x1[r], sa) && holds<OPC>(rr.xc[r], 0u, sc)) ? 1u : 0u;
            }
            // Lanes past the end of the R block carry garbage counts: only valid rows are summed.
            uint64_t mine = 0;
#pragma unroll
            for (int r = 0; r < kRB; ++r) mine += (r0 + r * kWave + lane < rEnd) ? (uint64_t)cnt[r] : 0ull;
            const uint64_t tot = wave_sum64(mine);
            if (lane == 0) counts[u] = tot;
        }
    }
}

// ------------------------------------------------------------------------------- write pass --
template <int OPA, int OPC, bool DENSE = false>
__global__ __launch_bounds__(kThetaBlock) void theta_write_k(ThetaGeom g,
                                                             const uint64_t* __restrict__ offsets,
                                                             const uint64_t* __restrict__ total,
                                                             int2* __restrict__ out, uint64_t cap)
{
    const uint64_t tot = *total;
    // an output too small for the exact count, or a plan other than the count pass's, receives
    // nothing
    if (tot > cap || (g.stamp_at && *g.stamp_at != g.stamp)) return;
    const int lane = (int)lane_id();
    const int64_t u = (int64_t)blockIdx.x * kWavesPerBlock + uniform((int32_t)(threadIdx.x >> 6));
    if (u >= unit_count(g)) return;
    {
        const uint64_t off = uniform(offsets[u]);
        const uint64_t cnt = (u + 1 < g.nOff ? uniform(offsets[u + 1]) : tot) - off;
        if (cnt == 0) return;
        if (g.stash && cnt <= (uint64_t)g.K) {  // the count pass kept every match of this unit
            const int2* st = g.stash + u * g.K;
            for (uint64_t i = lane; i < cnt; i += kWave)
                if (off + i < cap) out[off + i] = st[i];
#if JL_DEBUG
            if (g.dbg && lane == 0) g.dbg[u] = cnt;
#endif
            return;
        }
        int64_t r0, rEnd, s0, s1;
        unit_of(g, u, r0, rEnd, s0, s1);
        uint64_t base = off;
        if constexpr (selective<OPA>() && !DENSE) {
            RRows rr;
            load_r<OPA, JOIN_OP_NONE>(g, r0, rEnd, lane, rr);
            sweep_selective<OPA, OPC>(g, rr, r0, rEnd, s0, s1, base, out, cap, lane);
        } else {
            RRows rr;
            load_r<OPA, OPC>(g, r0, rEnd, lane, rr);
            int32_t rid[kRB];
            uint64_t vm[kRB];
            load_rids(g, r0, rEnd, lane, rid, vm);
            const cptr<int32_t> Sa = as_const(g.Sa);
            const cptr<int32_t> Sc = as_const(g.Sc);
            const cptr<int32_t> Srid = as_const(g.Srid);
            for (int64_t j = s0; j < s1; ++j) {
                const int32_t sc = (OPC != JOIN_OP_NONE) ? Sc[j] : 0;
                const int32_t srid = Srid ? Srid[j] : (int32_t)j;
                emit_row<OPA, OPC>(rr, rid, vm, Sa[j], sc, srid, base, out, cap, lane);
            }
        }
#if JL_DEBUG
        if (g.dbg && lane == 0) g.dbg[u] = base - off;
#endif
    }
}

// ------------------------------------------------------------------------------ dispatching --
using CountFn = void (*)(ThetaGeom, uint64_t*);
using WriteFn = void (*)(ThetaGeom, const uint64_t*, const uint64_t*, int2*, uint64_t);

template <int OPA, bool DENSE>
struct Table {
    static CountFn count(int opc)
    {
        switch (opc) {
        case JOIN_OP_NONE: return theta_count_k<OPA, JOIN_OP_NONE, DENSE>;
        case JOIN_OP_EQ: return theta_count_k<OPA, JOIN_OP_EQ, DENSE>;
        case JOIN_OP_NE: return theta_count_k<OPA, JOIN_OP_NE, DENSE>;
        case JOIN_OP_LT: return theta_count_k<OPA, JOIN_OP_LT, DENSE>;
        case JOIN_OP_LE: return theta_count_k<OPA, JOIN_OP_LE, DENSE>;
        case JOIN_OP_GT: return theta_count_k<OPA, JOIN_OP_GT, DENSE>;
        case JOIN_OP_GE: return theta_count_k<OPA, JOIN_OP_GE, DENSE>;
        default: return nullptr;
        }
    }
    static WriteFn write(int opc)
    {
        switch (opc) {
        case JOIN_OP_NONE: return theta_write_k<OPA, JOIN_OP_NONE, DENSE>;
        case JOIN_OP_EQ: return theta_write_k<OPA, JOIN_OP_EQ, DENSE>;
        case JOIN_OP_NE: return theta_write_k<OPA, JOIN_OP_NE, DENSE>;
        case JOIN_OP_LT: return theta_write_k<OPA, JOIN_OP_LT, DENSE>;
        case JOIN_OP_LE: return theta_write_k<OPA, JOIN_OP_LE, DENSE>;
        case JOIN_OP_GT: return theta_write_k<OPA, JOIN_OP_GT, DENSE>;
        case JOIN_OP_GE: return theta_write_k<OPA, JOIN_OP_GE, DENSE>;
        default: return nullptr;
        }
    }
};

// dense: region units (only the selective operators have a separate dense form)
CountFn count_fn(int opa, int opc, bool dense = false)
{
    switch (opa) {
    case JOIN_OP_EQ: return dense ? Table<JOIN_OP_EQ, true>::count(opc) : Table<JOIN_OP_EQ, false>::count(opc);
    case JOIN_OP_NE: return Table<JOIN_OP_NE, false>::count(opc);
    case JOIN_OP_LT: return Table<JOIN_OP_LT, false>::count(opc);
    case JOIN_OP_LE: return Table<JOIN_OP_LE, false>::count(opc);
    case JOIN_OP_GT: return Table<JOIN_OP_GT, false>::count(opc);
    case JOIN_OP_GE: return Table<JOIN_OP_GE, false>::count(opc);
    case JOIN_OP_BAND: return dense ? Table<JOIN_OP_BAND, true>::count(opc) : Table<JOIN_OP_BAND, false>::count(opc);
    default: return nullptr;
    }
}

WriteFn write_fn(int opa, int opc, bool dense = false)
{
    switch (opa) {
    case JOIN_OP_EQ: return dense ? Table<JOIN_OP_EQ, true>::write(opc) : Table<JOIN_OP_EQ, false>::write(opc);
    case JOIN_OP_NE: return Table<JOIN_OP_NE, false>::write(opc);
    case JOIN_OP_LT: return Table<JOIN_OP_LT, false>::write(opc);
    case JOIN_OP_LE: return Table<JOIN_OP_LE, false>::write(opc);
    case JOIN_OP_GT: return Table<JOIN_OP_GT, false>::write(opc);
    case JOIN_OP_GE: return Table<JOIN_OP_GE, false>::write(opc);
    case JOIN_OP_BAND: return dense ? Table<JOIN_OP_BAND, true>::write(opc) : Table<JOIN_OP_BAND, false>::write(opc);
    default: return nullptr;
    }
}

ThetaGeom geom(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S, const join_pred_t& p,
               char* ws)
{
    ThetaGeom g;
    g.K = pl.K;
    g.stash = pl.K > 0 ? reinterpret_cast<int2*>(ws + pl.off_stash) : nullptr;
    g.Ra = R.key;
    g.Rc = R.key2;
    g.Rrid = R.rid;
    g.nR = R.n;
    g.Sa = S.key;
    g.Sc = S.key2;
    g.Srid = S.rid;
    g.nS = S.n;
    g.w = p.op_a == JOIN_OP_BAND ? (int64_t)p.w : 0;
    g.TS = pl.TS;
    g.nSt = pl.nSt;
    g.U = pl.U;
    g.units = nullptr;
    g.Uptr = nullptr;
    g.nOff = pl.U;
    g.stamp_at = reinterpret_cast<uint64_t*>(ws + kStampOffset);
    g.stamp = pl.stamp;
    g.dbg = JL_DEBUG ? reinterpret_cast<uint64_t*>(ws + pl.off_dbg) : nullptr;
    return g;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

ThetaGeom unit_geom(const ThetaUnitArgs& a, const join_pred_t& p)
{
    ThetaGeom g{};
    g.Ra = a.Ra;
    g.Rc = a.Rc;
    g.Rrid = a.Rrid;
    g.Sa = a.Sa;
    g.Sc = a.Sc;
    g.Srid = a.Srid;
    g.w = p.op_a == JOIN_OP_BAND ? (int64_t)p.w : 0;
    g.U = a.Umax;
    g.stash = a.stash;
    g.K = a.stash ? a.K : 0;
    g.units = a.units;
    g.Uptr = a.Uptr;
    g.nOff = a.nOff;
    g.stamp_at = a.stamp_at;
    g.stamp = a.stamp;
    g.dbg = a.dbg;
    return g;
}

}  // namespace

hipError_t theta_count_units(const ThetaUnitArgs& a, const join_pred_t& p, uint64_t* counts,
                             hipStream_t st)
{
    if (a.Umax <= 0) return hipSuccess;
    CountFn f = count_fn(p.op_a, p.op_c, true);
    if (!f) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)ceil_div(a.Umax, kWavesPerBlock);
    prof::Scope ps(st, "region.count");
    hipLaunchKernelGGL(f, dim3(grid), dim3(kThetaBlock), 0, st, unit_geom(a, p), counts);
    return hipGetLastError();
}

hipError_t theta_write_units(const ThetaUnitArgs& a, const join_pred_t& p,
                             const uint64_t* offsets, const uint64_t* total, int32_t* pairs,
                             uint64_t cap, hipStream_t st)
{
    if (a.Umax <= 0) return hipSuccess;
    WriteFn f = write_fn(p.op_a, p.op_c, true);
    if (!f) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)ceil_div(a.Umax, kWavesPerBlock);
    prof::Scope ps(st, "region.write");
    hipLaunchKernelGGL(f, dim3(grid), dim3(kThetaBlock), 0, st, unit_geom(a, p), offsets, total,
                       reinterpret_cast<int2*>(pairs), cap);
    return hipGetLastError();
}

ThetaPlan theta_plan(int64_t nR, int64_t nS, int op_a, int64_t target_waves, int64_t ts_override,
                     int64_t stash_k)
{
    ThetaPlan pl{};
    const int64_t nRb = nR > 0 ? ceil_div(nR, kRowsPerWave) : 0;
    int64_t TS;
    if (ts_override > 0) {
        TS = ts_override;
    } else {
        int64_t nSt = nRb > 0 ? ceil_div(target_waves, nRb) : 1;
        int64_t max_tiles = nS > 0 ? ceil_div(nS, 256) : 1;
        if (nSt > max_tiles) nSt = max_tiles;
        if (nSt < 1) nSt = 1;
        TS = nS > 0 ? ceil_div(nS, nSt) : 1;
    }
    TS = ((TS + kSGroup - 1) / kSGroup) * kSGroup;
    if (TS > (1ll << 24)) TS = 1ll << 24;  // per-lane uint32 counters hold kRB * TS
    if (TS < kSGroup) TS = kSGroup;
    pl.TS = TS;
    pl.nSt = nS > 0 ? ceil_div(nS, TS) : 0;
    pl.U = nRb * pl.nSt;
    size_t off = 256;  // header: [0] total (uint64)
    pl.off_counts = off;
    off = align_up(off + (size_t)(pl.U > 0 ? pl.U : 1) * sizeof(uint64_t));
    pl.off_temp = off;
    off = align_up(off + scan_temp_elems<uint64_t>(pl.U) * sizeof(uint64_t) + 8);
    // Only the selective operators (or an unknown one, for sizing) get the match stash.
    const bool sel = op_a == JOIN_OP_BAND || op_a == JOIN_OP_EQ || op_a == JOIN_OP_NONE;
    pl.K = sel && stash_k > 0 ? stash_k : 0;
    pl.off_stash = off;
    off = align_up(off + (size_t)pl.U * (size_t)pl.K * sizeof(int2));
    pl.off_dbg = off;  // last: the checking build's per-unit written counts
    off = align_up(off + (JL_DEBUG ? (size_t)(pl.U > 0 ? pl.U : 1) * 8 : 0));
    pl.bytes = off;
    pl.stamp = plan_stamp({JOIN_KIND_THETA, nR, nS, op_a, pl.TS, pl.nSt, pl.U, pl.K, (int64_t)pl.bytes});
    return pl;
}

hipError_t theta_count(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S,
                       const join_pred_t& p, char* ws, hipStream_t st, uint64_t* pub)
{
    uint64_t* total = reinterpret_cast<uint64_t*>(ws);
    uint64_t* counts = reinterpret_cast<uint64_t*>(ws + pl.off_counts);
    uint64_t* temp = reinterpret_cast<uint64_t*>(ws + pl.off_temp);
    if (pl.U > 0) {
        CountFn f = count_fn(p.op_a, p.op_c);
        if (!f) return hipErrorInvalidValue;
        const unsigned grid = (unsigned)ceil_div(pl.U, kWavesPerBlock);
        prof::Scope ps(st, "theta.count");
        hipLaunchKernelGGL(f, dim3(grid), dim3(kThetaBlock), 0, st, geom(pl, R, S, p, ws), counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return exclusive_scan<uint64_t>(counts, counts, pl.U, total, temp, st, pub);
}

hipError_t theta_write(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S,
                       const join_pred_t& p, char* ws, int32_t* pairs, uint64_t cap,
                       hipStream_t st)
{
    if (pl.U <= 0) return hipSuccess;
    const uint64_t* offsets = reinterpret_cast<const uint64_t*>(ws + pl.off_counts);
    WriteFn f = write_fn(p.op_a, p.op_c);
    if (!f) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)ceil_div(pl.U, kWavesPerBlock);
    prof::Scope ps(st, "theta.write");
    hipLaunchKernelGGL(f, dim3(grid), dim3(kThetaBlock), 0, st, geom(pl, R, S, p, ws), offsets,
                       reinterpret_cast<const uint64_t*>(ws), reinterpret_cast<int2*>(pairs), cap);
    return hipGetLastError();
}

}  // namespace jl
