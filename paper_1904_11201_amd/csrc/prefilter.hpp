// prefilter.hpp -- the pre-filter in front of the hash join: key-presence filters of both
// relations, both relations compacted to the tuples whose key may occur on the other side.
#pragma once
#include "common.hpp"
#include "hash.hpp"

namespace jl {

struct PrefilterPlan {
    int64_t nR, nS;
    int logR, logS;          // log2 of the filter sizes in bits (of R, of S); 0 = no filter
    int semi;                // 1: no filters; the inner join records its semi-join (probe side too large)
    int ordered;             // 1: compaction in input order (deterministic option), else arrival order
    int grid;                // compaction workgroups
    uint64_t off_wcnt, off_wtmp;  // ordered compaction: per-workgroup counts, scan storage
    uint64_t off_cnt;        // 2 uint32: surviving R rows, surviving S rows
    uint64_t off_fR, off_fS; // the two bit filters
    uint64_t off_kR, off_rR, off_kS, off_rS;  // compacted columns (key, rid)
    uint64_t off_inner;      // the inner hash join's workspace, sized for the unfiltered sizes
    uint64_t inner_bytes;
    uint64_t bytes;
    uint64_t stamp;          // signature of the fields above and of the full-size inner plan
};

PrefilterPlan prefilter_plan(int64_t nR, int64_t nS, int num_cus);

// Filters and compaction (launches), then the surviving sizes are read to the host (one
// 8-byte read) and the inner hash join's count pass runs on the survivors.
hipError_t prefilter_count(const PrefilterPlan& pl, const join_rel_t& R, const join_rel_t& S,
                           char* ws, hipStream_t st, int num_cus, uint64_t* pub = nullptr);

// Reads the surviving sizes (one 8-byte read, none if neither side has a filter), then the
// inner hash join's write pass.
hipError_t prefilter_write(const PrefilterPlan& pl, const join_rel_t& R, const join_rel_t& S,
                           char* ws, int32_t* pairs, uint64_t cap, hipStream_t st, int num_cus);

// The exact total of the last count pass lives at the start of the inner workspace.
inline uint64_t prefilter_total_offset(const PrefilterPlan& pl) { return pl.off_inner; }

}  // namespace jl
