// theta.hpp -- tiled nested-loop theta join (count pass, scan, write pass).
#pragma once
#include "common.hpp"

namespace jl {

struct ThetaPlan {
    int64_t TS;   // S rows per tile
    int64_t nSt;  // S tiles
    int64_t U;    // work units (one wave each)
    int64_t K;    // per-unit match stash of the count pass (0: none)
    size_t off_counts, off_temp, off_stash, off_dbg, bytes;
    uint64_t stamp;  // signature of the fields above (plan_stamp)
};

// Plan for |R| = nR, |S| = nS and operator op_a (JOIN_OP_NONE: unknown, sized for the largest
// layout).  target_waves sets how many units the grid should hold; ts_override > 0 forces the
// S tile length; stash_k is the per-unit match stash of selective predicates (0 disables it).
ThetaPlan theta_plan(int64_t nR, int64_t nS, int op_a, int64_t target_waves, int64_t ts_override,
                     int64_t stash_k);

// Count pass + device scan.  Leaves offsets in ws and the total at ws[0..8).
hipError_t theta_count(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S,
                       const join_pred_t& p, char* ws, hipStream_t st, uint64_t* pub = nullptr);

// Theta kernels over an explicit unit table (the red regions of the region-pruned join).
struct ThetaUnitArgs {
    const int32_t *Ra, *Rc, *Rrid;  // bucketed R columns (rid materialised)
    const int32_t *Sa, *Sc, *Srid;  // bucketed S columns
    const uint4* units;             // [Umax] {r0, rEnd, s0, s1}
    const uint32_t* Uptr;           // device unit count
    int64_t Umax;
    int2* stash;                    // [Umax][K] or NULL
    int64_t K;
    int64_t nOff;                   // entries of the offsets array
    uint64_t* stamp_at;             // plan stamp in the workspace header (see ThetaPlan)
    uint64_t stamp;
    uint64_t* dbg;                  // checking build: pairs written per unit, or NULL
};

hipError_t theta_count_units(const ThetaUnitArgs& a, const join_pred_t& p, uint64_t* counts,
                             hipStream_t st);
hipError_t theta_write_units(const ThetaUnitArgs& a, const join_pred_t& p,
                             const uint64_t* offsets, const uint64_t* total, int32_t* pairs,
                             uint64_t cap, hipStream_t st);

// Write pass from the offsets left by theta_count.
hipError_t theta_write(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S,
                       const join_pred_t& p, char* ws, int32_t* pairs, uint64_t cap,
                       hipStream_t st);

}  // namespace jl
