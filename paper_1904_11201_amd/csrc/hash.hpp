// hash.hpp -- partitioned hash equi join (histogram, scatter, LDS-table count and write).
#pragma once
#include "common.hpp"

namespace jl {

// One radix partition after the scatter: its R and S ranges in the partitioned tuples, its
// work-unit split (nRc R chunks that fit the LDS table, nSs S slices) and its join's fan-out.
struct PartInfo {
    uint32_t rStart, nR, sStart, nS, nSs, nRc, bits, pad;
};

// One chunk of one relation side of one join, for the histogram and scatter kernels.
struct SideItem {
    const int32_t* key;
    const int32_t* rid;  // NULL: rid = row position
    int64_t beg;         // first row of the chunk
    uint32_t len;        // rows in the chunk
    int32_t bits;        // the join's fan-out
    uint32_t part0;      // the join's first partition in the partition arrays
    uint64_t cnt0;       // first per-tile count row of the chunk: tile t's row of 2^bits
                         // counts starts at element cnt0 + t * 2^bits of the side's count array
};

// Everything the count and write kernels need to walk the work units.
struct JoinGeom {
    const int32_t* rk;  // single: the input build keys
    const int32_t* rr;  // single: the input build rids; NULL means position
    const int32_t* sk;  // single: the input probe keys
    const int32_t* sr;  // single: the input probe rids; NULL means position
    const int2* rt;     // partitioned: (key, rid) build tuples, partition-major
    const int2* st;     // partitioned: (key, rid) probe tuples, partition-major
    const PartInfo* part;       // [P]
    const uint32_t* unitStart;  // [P + 1], exclusive scan of units per partition
    const uint4* urec;          // [Umax], each unit's record (unit_rec)
    const uint32_t* Uptr;       // device total of units
    PartInfo one;               // the single partition when single != 0
    uint32_t Uhost;             // units when single != 0
    uint32_t cap;               // R chunk capacity (entries)
    int64_t Umax;               // size of the counts array
    int bits;                   // partition bits; the table position uses the bits below them
    int P;
    int single;
    int contig;  // write pass: contiguous runs of units per workgroup (else round robin)
    uint64_t* stamp_at;  // plan stamp in the workspace header (NULL for batches: no re-planning)
    uint64_t stamp;      // this plan's stamp: the count pass records it, the write pass checks it
    uint64_t* dbg;       // checking build: pairs written per unit (NULL: not counted)
    uint32_t* semi;      // the probe rows with matches, per unit and wave (NULL: not recorded)
    uint32_t* sched;     // [3]: count ticket, write ticket, write arrivals (NULL: static shares)
};

struct HashPlan {
    int64_t nR, nS;
    int single;    // 1: no partitioning, units = R chunks x S slices of the inputs themselves
    int prebuilt;  // 1: R comes partitioned from a resident build (RView)
    int ordered;   // 1: the ordered scatter (output order fixed by the input), else arrival order
    int semi;      // 1: the count pass records the probe rows with matches and the write pass
                   // visits only those (partitioned plans; asked for by the pre-filter)
    int bits, P;
    int cap, slice;
    int64_t nSs;  // S slices (single)
    int64_t chR, chS, nChR, nChS;
    int64_t Umax;
    int gridCount, gridWrite;  // persistent grids of the count and write kernels
    size_t off_tot, off_grpR, off_grpS, off_done, off_baseR, off_baseS, off_tupR, off_tupS;
    size_t off_info, off_units, off_umap, off_cntR, off_cntS;
    size_t off_counts, off_wave, off_temp, off_dbg, off_semi, bytes;
    uint64_t stamp;  // signature of the fields above (plan_stamp)
};

// prebuilt_bits >= 0: R is a resident build partitioned with that fan-out (no single path, no
// R arrays in the workspace).
// semi: record the semi-join in the count pass (ignored by the unpartitioned path).
HashPlan hash_plan(int64_t nR, int64_t nS, int num_cus, int prebuilt_bits = -1, bool semi = false);

// A build relation already partitioned (resident build): its partition sizes, starts, tuples.
struct RView {
    const uint32_t* tot;
    const uint32_t* base;
    const int2* tup;
};

// Layout of a resident build buffer.
struct BuildPlan {
    int64_t nR;
    int32_t bits, P;
    int32_t ordered, pad;
    int64_t chR, nChR;
    uint64_t off_tot, off_base, off_tup, off_temp, off_cnt, bytes;
};

BuildPlan hash_build_plan(int64_t nR, int num_cus);
hipError_t hash_build(const BuildPlan& b, const join_rel_t& R, char* build, hipStream_t st);
RView build_view(const BuildPlan& b, const void* build);

// Histogram, scatter, planning, count pass and the scan of counts.  Leaves the exact total at
// ws[0..8) and the per-unit offsets in ws; pub (may be NULL): a pinned host slot (its device
// address) that the kernel producing the total also stores it into.
hipError_t hash_count(const HashPlan& pl, const join_rel_t& R, const join_rel_t& S, char* ws,
                      hipStream_t st, const RView* pre = nullptr, uint64_t* pub = nullptr);

// Write pass from the state hash_count left in ws.
hipError_t hash_write(const HashPlan& pl, const join_rel_t& R, const join_rel_t& S, char* ws,
                      int32_t* pairs, uint64_t cap, hipStream_t st, const RView* pre = nullptr);

// A batch of independent equi joins: layout of the shared workspace and launch sizes.  Kept
// by the caller as an opaque join_batch_plan_t between the prepare, count and write calls.
struct BatchPlan {
    int32_t njobs, maxBits, cap, slice;
    int32_t ordered, pad;
    int64_t nParts, nItemsR, nItemsS, sumR, sumS, Umax;
    uint64_t off_jpart0, off_jbits, off_itemsR, off_itemsS, off_tot, off_baseR, off_baseS;
    uint64_t off_tupR, off_tupS, off_info, off_units, off_umap;
    uint64_t off_item0R, off_item0S, off_cntR, off_cntS;  // per-join first items, per-tile counts
    uint64_t off_counts, off_wave, off_temp, bytes;
    int32_t gridCount, gridWrite;
};

// Plans the batch (fan-out per join, items, workspace layout).  Returns -1 when the batch
// exceeds the 32-bit row, partition or unit indices.
int hash_batch_plan(int njobs, const join_job_t* jobs, int num_cus, BatchPlan* out);

// Uploads the join and item tables into ws and waits for the copies.
hipError_t hash_batch_upload(const BatchPlan& bp, const join_job_t* jobs, char* ws, hipStream_t st);

// Histogram, scatter, planning and count pass of every join, the scan of unit counts, and the
// per-join output offsets (offsets[0..njobs], offsets[njobs] = total).  Launches only.
hipError_t hash_batch_count(const BatchPlan& bp, char* ws, uint64_t* offsets, hipStream_t st);

// Write pass of every join from the state hash_batch_count left in ws.  Launches only.
hipError_t hash_batch_write(const BatchPlan& bp, char* ws, int32_t* pairs, uint64_t cap, hipStream_t st);

}  // namespace jl
