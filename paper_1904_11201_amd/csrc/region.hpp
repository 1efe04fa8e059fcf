// region.hpp -- theta join with region pruning (bucketed ranges, red/green/white regions).
#pragma once
#include "common.hpp"

namespace jl {

struct RegionPlan {
    int bits, B;                 // B = 2^bits value buckets shared by both sides
    int64_t chR, chS, nChR, nChS;
    int64_t Umax;                // bound on red units
    int64_t K;                   // per-unit match stash (selective predicates)
    int64_t nOff;                // Umax red counts + 2 green counts per bucket
    size_t off_hist2, off_lut, off_vlo, off_vhi, off_hR, off_hS;
    size_t off_Ra, off_Rc, off_Rr, off_Sa, off_Sc, off_Sr;
    size_t off_info, off_split, off_units, off_table, off_counts, off_stash, off_temp, off_dbg, bytes;
    uint64_t stamp;  // signature of the fields above (plan_stamp)
};

RegionPlan region_plan(int64_t nR, int64_t nS, int op_a, int64_t stash_k);

// Range, buckets, partition, classification, red-unit count pass and the scan of all counts.
// Leaves the exact total at ws[0..8).
hipError_t region_count(const RegionPlan& pl, const join_rel_t& R, const join_rel_t& S,
                        const join_pred_t& p, char* ws, hipStream_t st, uint64_t* pub = nullptr);

// Write pass: red units (stash copy or re-sweep) and green cross products.
hipError_t region_write(const RegionPlan& pl, const join_rel_t& R, const join_rel_t& S,
                        const join_pred_t& p, char* ws, int32_t* pairs, uint64_t cap,
                        hipStream_t st);

}  // namespace jl
