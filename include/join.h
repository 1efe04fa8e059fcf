/*
 * join.h -- C ABI of libjoin, a single-GPU (MI355X, gfx950) relational join library.
 *
 * The operations follow "GPU-based Efficient Join Algorithms on Hadoop" (Wang, Li, Wang, Li):
 *   - the equi join and theta join problem statements (Section 2.3): two relations, a join
 *     condition on one attribute of each, and the output is the set of matching tuple pairs;
 *   - the column layout handed to the GPU (Section 3.2.2): one buffer per attribute, all in the
 *     same tuple order, and a match of record m of one table with record n of the other yields
 *     the pair of positions (m, n);
 *   - the GPU entry points of Algorithm 1 (Join_GPU(T', S', NB_T, NB_S)) and Algorithm 3
 *     (GPU_theta_join(S, T)), which receive both tables and their sizes;
 *   - the result-size problem of Section 3.3.3: the paper preallocates a bound (NB_T * NB_S,
 *     Section 3.3.1, or its estimate R_size); this library instead counts the result exactly,
 *     scans the per-work-unit counts on the device and writes each pair at its exact offset, so
 *     the caller allocates the output once at its exact size.
 *
 * Naming: the paper's table T (the smaller, hashed table, Section 2.3 and Section 3.3.2) is R
 * here; its S is S.  A predicate always reads  R.col  op  S.col.
 *
 * Conventions for every call below
 *   - Pointers inside join_rel_t, the workspace and the output are DEVICE pointers on the
 *     current HIP device.  join_rel_t / join_pred_t structs themselves and `count` are HOST
 *     pointers (except join_hash_noalloc's `count`, a device pointer).  The caller owns every
 *     buffer; the library never allocates device memory and keeps no pointer after a call
 *     returns.  The one piece of device memory the library holds is the static 64 MiB array that
 *     join_hash_noalloc works in, which exists once per GPU from the loading of the library's
 *     GPU code until the process ends.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All device work is
 *     enqueued on it in order.  The only host synchronisation is the wait for the exact count
 *     in join_count, join_hash, join_theta and join_probe_count: the kernel that produces it
 *     stores it into a pinned host word the library keeps per host thread, and the calling
 *     thread polls that word (until it changes, or the stream fails or goes idle without it).
 *   - Counts and offsets are uint64.  Output is int32 pairs, interleaved (rid_R, rid_S), i.e. a
 *     row-major [count][2] int32 array.  The order of pairs is unspecified; the multiset is
 *     exact (bag semantics: duplicate keys produce every matching pair).
 *   - Status codes are returned; nothing throws or aborts across the ABI.  After a non-zero
 *     status, join_last_error() describes it (thread-local).
 */
#ifndef JOIN_H
#define JOIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define JOIN_OK 0
#define JOIN_E_INVAL 1       /* bad argument: NULL with n > 0, n < 0, bad op, w < 0, ...       */
#define JOIN_E_CAPACITY 2    /* output capacity below the exact count; nothing was written     */
#define JOIN_E_WORKSPACE 3   /* workspace NULL or smaller than join_workspace_bytes()          */
#define JOIN_E_HIP 4         /* a HIP runtime call failed; text in join_last_error()           */
#define JOIN_E_UNSUPPORTED 5 /* a size beyond the supported range (n > 2^31 - 1)               */

/* ---- join kinds -------------------------------------------------------------------------- */
#define JOIN_KIND_HASH 1  /* equi join R.key = S.key (Section 3.3.2, hash join)                */
#define JOIN_KIND_THETA 2 /* theta join, nested-loop evaluation (Sections 3.3.1 and 4.2)       */
#define JOIN_KIND_THETA_REGION 3 /* theta join with the improved algorithm's region pruning
                                  * (Section 4.2, Algorithm 3): key ranges cut into buckets shared
                                  * by both tables; white regions skipped, green regions counted
                                  * and cross-joined without evaluation, red regions evaluated by
                                  * the nested loop.  Same predicates and results as
                                  * JOIN_KIND_THETA. */
#define JOIN_KIND_HASH_PREFILTER 4 /* equi join preceded by the pre-filter of Algorithm 1
                                    * (Section 3.1): a relation of at most 2^21 rows gets a bit
                                    * filter of its keys (16 bits per row, at most 2^24 bits) and
                                    * the other relation is reduced to the tuples whose key may
                                    * occur in it (never dropping a matching tuple); with two
                                    * small relations both are reduced.  Then joined as
                                    * JOIN_KIND_HASH: same result.  Pays off when a small
                                    * relation meets a large one with few matching keys.  Its
                                    * join_materialize reads the surviving sizes from the device
                                    * (one 8-byte host read). */

/* ---- predicate operators (Section 2.3: =, <, >, <=, >=; Figure "greenc": not-equal) -------- */
typedef enum {
    JOIN_OP_NONE = 0, /* no condition on this column (only valid for op_c)                    */
    JOIN_OP_EQ = 1,   /* R.x == S.x                                                          */
    JOIN_OP_NE = 2,   /* R.x != S.x                                                          */
    JOIN_OP_LT = 3,   /* R.x <  S.x   (signed int32)                                         */
    JOIN_OP_LE = 4,   /* R.x <= S.x                                                          */
    JOIN_OP_GT = 5,   /* R.x >  S.x                                                          */
    JOIN_OP_GE = 6,   /* R.x >= S.x                                                          */
    JOIN_OP_BAND = 7  /* |R.a - S.a| <= w, exact integer arithmetic; only valid for op_a      */
} join_op_t;

/* One relation in column layout (Section 3.2.2).  Device pointers.
 *   key  : the equi-join key, or theta column a.  Required when n > 0.
 *   key2 : theta column c; required when the predicate's op_c != JOIN_OP_NONE, else ignored.
 *   rid  : opaque int32 payload written to the output; NULL means "row position" (0..n-1).
 *   n    : number of rows, 0 <= n <= 2^31 - 1. */
typedef struct {
    const int32_t* key;
    const int32_t* key2;
    const int32_t* rid;
    int64_t n;
} join_rel_t;

/* Theta predicate: op_a(R.key, S.key) AND op_c(R.key2, S.key2).
 *   op_a : JOIN_OP_EQ .. JOIN_OP_BAND
 *   w    : band half-width for JOIN_OP_BAND, 0 <= w <= 2^31 - 1 (ignored otherwise)
 *   op_c : JOIN_OP_NONE .. JOIN_OP_GE (BAND is rejected on c) */
typedef struct {
    int32_t op_a;
    int32_t w;
    int32_t op_c;
} join_pred_t;

/* Workspace size in bytes needed by join_count / join_materialize / join_hash / join_theta for
 * this kind and these sizes.  Depends only on (kind, nR, nS, pred) and the library's tuning
 * environment (JOIN_HASH_BITS, ...), so the same value serves a count and its later
 * materialize.  Returns 0 for invalid arguments (kind unknown, n < 0). */
size_t join_workspace_bytes(int kind, int64_t nR, int64_t nS, const join_pred_t* pred);

/* Exact result size (Section 3.3.3, done exactly).  Runs the count pass and the device scan of
 * per-work-unit counts, leaves the plan, partitioned data and offsets in `ws`, and writes the
 * exact number of output pairs to *count (host).  `pred` may be NULL for JOIN_KIND_HASH.
 * Between join_count and join_materialize the caller must not change R, S or ws.
 * Errors: JOIN_E_INVAL, JOIN_E_WORKSPACE, JOIN_E_UNSUPPORTED, JOIN_E_HIP. */
int join_count(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred,
               void* ws, size_t ws_bytes, void* stream, uint64_t* count);

/* Write pass: writes every pair at the offset the preceding join_count computed in `ws`
 * (same kind, R, S, pred and ws).  `pairs` holds `capacity` pairs (2*capacity int32).  If the
 * exact count exceeds `capacity`, nothing is written and JOIN_E_CAPACITY is returned when the
 * library can tell on the host (the count of the last join_count on this thread for this ws);
 * in every case the device never writes past `capacity`.  Asynchronous: no host sync. */
int join_materialize(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred,
                     void* ws, size_t ws_bytes, int32_t* pairs, uint64_t capacity, void* stream);

/* One-shot equi join (Algorithm 1's Join_GPU, hash join of Section 3.3.2): count, scan, and
 * if capacity >= *count write.  snprintf semantics: *count is always set on success of the
 * count; if capacity < *count nothing is written, JOIN_E_CAPACITY is returned and ws stays
 * valid for a later join_materialize without recounting. */
int join_hash(const join_rel_t* R, const join_rel_t* S, void* ws, size_t ws_bytes,
              int32_t* pairs, uint64_t capacity, uint64_t* count, void* stream);

/* One-shot theta join (Algorithm 3's GPU_theta_join; nested-loop evaluation of Section 3.3.1
 * with the predicate of Section 2.3).  Same semantics as join_hash. */
int join_theta(const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred, void* ws,
               size_t ws_bytes, int32_t* pairs, uint64_t capacity, uint64_t* count,
               void* stream);

/* ---- the hash join without a workspace argument -------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): join_hash with its workspace taken from a static
 * device array of 64 MiB that the library holds on every GPU it runs on until the process ends,
 * instead of a caller buffer.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine) and does not synchronise: the exact count is written to `count`, a DEVICE
 * pointer to one uint64, and the pairs are written to `pairs` (device, `capacity` pairs) only if
 * the count fits (device-side snprintf semantics: count always set, pairs written only when
 * count <= capacity).  Same inputs and result as join_hash.
 * Every call on one GPU uses that GPU's array, which keeps the last call's contents; each call
 * clears what it accumulates into before use.  Calls that overlap in time on one GPU (other
 * streams, other host threads) race on the array and must be serialised by the caller.
 * Errors: JOIN_E_INVAL, JOIN_E_UNSUPPORTED, JOIN_E_WORKSPACE (the join's workspace, the size
 * join_workspace_bytes(JOIN_KIND_HASH, ...) reports, exceeds 64 MiB), JOIN_E_HIP. */
int join_hash_noalloc(const join_rel_t* R, const join_rel_t* S, int32_t* pairs, uint64_t capacity,
                      uint64_t* count, void* stream);

/* ---- resident builds ---------------------------------------------------------------------
 * The partitioned form of a build relation R, kept in caller-owned device memory and probed by
 * many probe relations S_k: the R side's histogram and scatter run once (join_build) instead of
 * once per join.  In the paper the smaller table T is the one hashed and S the one probed
 * (Sections 2.3 and 3.3.2); a serving loop that sees the same T again keeps it partitioned.
 * The result of join_probe_* equals join_hash(R, S) as a multiset of (rid_R, rid_S) pairs.
 * The build buffer must stay unchanged while it is probed; R itself may be freed after
 * join_build's work has completed on its stream. */
typedef struct {
    uint64_t opaque[16]; /* plain bytes: sizes, fan-out and layout of the build buffer */
} join_build_t;

/* Bytes of the build buffer for a build side of nR rows; 0 if nR < 0 or nR > 2^31 - 1. */
size_t join_build_bytes(int64_t nR);

/* Partitions R into `build` (device, join_build_bytes(R->n) bytes) and fills *desc.
 * Asynchronous on `stream` (launches only).  Errors: JOIN_E_INVAL, JOIN_E_WORKSPACE,
 * JOIN_E_UNSUPPORTED, JOIN_E_HIP. */
int join_build(const join_rel_t* R, void* build, size_t build_bytes, join_build_t* desc,
               void* stream);

/* Workspace bytes for probing the build `desc` with nS rows; 0 for invalid arguments. */
size_t join_probe_workspace_bytes(const join_build_t* desc, int64_t nS);

/* Count pass of R ⋈ S with R taken from the build: same contract as join_count (one 8-byte
 * host read, *count set). */
int join_probe_count(const join_build_t* desc, const void* build, const join_rel_t* S, void* ws,
                     size_t ws_bytes, void* stream, uint64_t* count);

/* Write pass after join_probe_count (same desc, build, S, ws): same contract as
 * join_materialize. */
int join_probe_materialize(const join_build_t* desc, const void* build, const join_rel_t* S,
                           void* ws, size_t ws_bytes, int32_t* pairs, uint64_t capacity,
                           void* stream);

/* ---- batched equi joins -----------------------------------------------------------------
 * Many independent equi joins R_j.key = S_j.key (j = 0..njobs-1) in one pass of fused
 * launches.  In the paper every MapReduce reducer runs its own GPU join and the reducer count
 * is bounded so that reducers x blocks x threads fit the GPU (Section 3.3.4, equation "hier");
 * here the reducers' joins share one set of launches instead: every join gets its own fan-out
 * and partitions, and the work units of all joins form one list, so the count pass, the scan
 * and the write pass are one launch each whatever njobs is.  Join j's pairs are written
 * contiguously, in join order, to one output array: pairs [offsets[j], offsets[j+1]).
 *
 * Flow: join_batch_workspace_bytes -> join_batch_prepare (host planning, uploads the join
 * tables, waits for the upload) -> join_batch_count (launches only: no host sync, so it can be
 * captured in a HIP graph) -> read offsets[njobs] -> join_batch_materialize (launches only). */
typedef struct {
    join_rel_t R;     /* build side of join j (key, rid; key2 ignored) */
    join_rel_t S;     /* probe side of join j */
    int32_t bits;     /* log2 of join j's partition fan-out, 0..11; < 0: the library's default
                       * for |R_j| (an autotuner may choose it) */
    int32_t reserved; /* must be 0 */
} join_job_t;

/* Opaque host-side plan filled by join_batch_prepare and passed to the later calls.  Plain
 * bytes: it may be copied, and it holds no pointers. */
typedef struct {
    uint64_t opaque[64];
} join_batch_plan_t;

/* Workspace bytes for this batch; 0 for invalid arguments or a batch whose total rows per side
 * reach 2^32. */
size_t join_batch_workspace_bytes(int njobs, const join_job_t* jobs);

/* Plans the batch and uploads its tables into ws (stream-ordered, then waits on the stream).
 * Validates every job like join_count does.  Errors: JOIN_E_INVAL, JOIN_E_WORKSPACE,
 * JOIN_E_UNSUPPORTED (batch too large for 32-bit indices), JOIN_E_HIP. */
int join_batch_prepare(int njobs, const join_job_t* jobs, void* ws, size_t ws_bytes,
                       join_batch_plan_t* plan, void* stream);

/* Count pass of every join.  Writes, on the device, offsets[j] = first output pair of join j
 * for j < njobs and offsets[njobs] = total pairs.  `offsets` is a device array of njobs + 1
 * uint64.  Asynchronous: no host sync.  Errors: JOIN_E_INVAL, JOIN_E_WORKSPACE, JOIN_E_HIP. */
int join_batch_count(const join_batch_plan_t* plan, void* ws, size_t ws_bytes, uint64_t* offsets,
                     void* stream);

/* Write pass of every join into `pairs` (capacity pairs).  If the total exceeds capacity the
 * device writes nothing (read offsets[njobs] first).  Asynchronous.  The inputs and ws must not
 * change since join_batch_count.  Errors: JOIN_E_INVAL, JOIN_E_WORKSPACE, JOIN_E_HIP. */
int join_batch_materialize(const join_batch_plan_t* plan, void* ws, size_t ws_bytes, int32_t* pairs,
                           uint64_t capacity, void* stream);

/* Message for the last non-zero status on the calling thread ("" if none). */
const char* join_last_error(void);

/* ---- primitive: device exclusive scan ----------------------------------------------------
 * The "scan" of count -> scan -> write, exported so it can be checked on its own.  The paper
 * gives each thread a private result region and "sums" the regions at the end (Section 3.3.1);
 * the exclusive prefix sum of per-unit counts is that summation made exact: out[i] = sum of
 * in[0..i), computed on the device.
 *   in, out : device arrays of n uint64 (out may equal in)
 *   total   : device pointer receiving sum(in[0..n)), or NULL
 *   ws      : device workspace of at least join_scan_workspace_bytes(n) bytes
 * Asynchronous on `stream`.  Errors: JOIN_E_INVAL (n < 0, NULL arrays with n > 0),
 * JOIN_E_WORKSPACE, JOIN_E_HIP. */
size_t join_scan_workspace_bytes(int64_t n);
int join_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total, void* ws,
                  size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* JOIN_H */
