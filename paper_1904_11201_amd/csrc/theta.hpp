// theta.hpp -- tiled nested-loop theta join (count pass, scan, write pass).
#pragma once
#include "common.hpp"

namespace jl {

struct ThetaPlan {
    int64_t TS;   // S rows per tile
    int64_t nSt;  // S tiles
    int64_t U;    // work units (one wave each)
    int64_t K;    // per-unit match stash of the count pass (0: none)
    size_t off_counts, off_temp, off_stash, bytes;
};

// Plan for |R| = nR, |S| = nS and operator op_a (JOIN_OP_NONE: unknown, sized for the largest
// layout).  target_waves sets how many units the grid should hold; ts_override > 0 forces the
// S tile length; stash_k is the per-unit match stash of selective predicates (0 disables it).
ThetaPlan theta_plan(int64_t nR, int64_t nS, int op_a, int64_t target_waves, int64_t ts_override,
                     int64_t stash_k);

// Count pass + device scan.  Leaves offsets in ws and the total at ws[0..8).
hipError_t theta_count(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S,
                       const join_pred_t& p, char* ws, hipStream_t st);

// Write pass from the offsets left by theta_count.
hipError_t theta_write(const ThetaPlan& pl, const join_rel_t& R, const join_rel_t& S,
                       const join_pred_t& p, char* ws, int32_t* pairs, uint64_t cap,
                       hipStream_t st);

}  // namespace jl
