// api.hip -- the C ABI of libjoin (include/join.h): validation, plans, launch sequencing and
// the single 8-byte host read of the exact count.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "debug.hpp"
#include "hash.hpp"
#include "prefilter.hpp"
#include "region.hpp"
#include "scan.hpp"
#include "theta.hpp"
#include "tune.hpp"

namespace jl {

static thread_local char g_err[512];

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return JOIN_E_HIP;
}

}  // namespace jl

using namespace jl;

namespace {

constexpr int64_t kMaxRows = 2147483647;  // rids and positions are int32

int num_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

int64_t theta_target_waves()
{
    const int64_t w = tune_get(TUNE_THETA_WAVES, 0);
    return w > 0 ? w : (int64_t)num_cus() * 4 * 16;  // 16 waves per SIMD, two rounds at occupancy 8
}

int64_t theta_ts_override() { return tune_get(TUNE_THETA_TS, 0); }

int64_t theta_stash_k() { return tune_get(TUNE_THETA_STASH, 128); }

ThetaPlan plan_theta(int64_t nR, int64_t nS, const join_pred_t* p)
{
    return theta_plan(nR, nS, p ? p->op_a : JOIN_OP_NONE, theta_target_waves(), theta_ts_override(),
                      theta_stash_k());
}

int check_rel(const join_rel_t* X, const char* name, bool need_key2)
{
    if (!X) {
        set_error("%s is NULL", name);
        return JOIN_E_INVAL;
    }
    if (X->n < 0) {
        set_error("%s.n = %lld is negative", name, (long long)X->n);
        return JOIN_E_INVAL;
    }
    if (X->n > kMaxRows) {
        set_error("%s.n = %lld exceeds 2^31 - 1", name, (long long)X->n);
        return JOIN_E_UNSUPPORTED;
    }
    if (X->n > 0 && !X->key) {
        set_error("%s.key is NULL with n > 0", name);
        return JOIN_E_INVAL;
    }
    if (need_key2 && X->n > 0 && !X->key2) {
        set_error("%s.key2 is NULL but the predicate has a condition on column c", name);
        return JOIN_E_INVAL;
    }
    return JOIN_OK;
}

int check_pred(const join_pred_t* p)
{
    if (!p) {
        set_error("theta join needs a predicate");
        return JOIN_E_INVAL;
    }
    if (p->op_a < JOIN_OP_EQ || p->op_a > JOIN_OP_BAND) {
        set_error("op_a = %d is not one of EQ..BAND", (int)p->op_a);
        return JOIN_E_INVAL;
    }
    if (p->op_c < JOIN_OP_NONE || p->op_c > JOIN_OP_GE) {
        set_error("op_c = %d is not one of NONE..GE (BAND is only valid on column a)", (int)p->op_c);
        return JOIN_E_INVAL;
    }
    if (p->op_a == JOIN_OP_BAND && p->w < 0) {
        set_error("band half-width w = %d is negative", (int)p->w);
        return JOIN_E_INVAL;
    }
    return JOIN_OK;
}

bool is_theta(int kind) { return kind == JOIN_KIND_THETA || kind == JOIN_KIND_THETA_REGION; }

int check_args(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* p)
{
    if (kind != JOIN_KIND_HASH && kind != JOIN_KIND_THETA && kind != JOIN_KIND_THETA_REGION &&
        kind != JOIN_KIND_HASH_PREFILTER) {
        set_error("kind = %d is not one of JOIN_KIND_HASH, _THETA, _THETA_REGION, _HASH_PREFILTER", kind);
        return JOIN_E_INVAL;
    }
    int rc;
    bool key2 = false;
    if (is_theta(kind)) {
        if ((rc = check_pred(p)) != JOIN_OK) return rc;
        key2 = p->op_c != JOIN_OP_NONE;
    }
    if ((rc = check_rel(R, "R", key2)) != JOIN_OK) return rc;
    if ((rc = check_rel(S, "S", key2)) != JOIN_OK) return rc;
    return JOIN_OK;
}

RegionPlan plan_region(int64_t nR, int64_t nS, const join_pred_t* p)
{
    return region_plan(nR, nS, p ? p->op_a : JOIN_OP_NONE, theta_stash_k());
}

// Signature of the plan a call of this kind makes for these sizes under the current knobs
// (the same value the count pass records in the workspace header).
uint64_t plan_stamp_of(int kind, int64_t nR, int64_t nS, const join_pred_t* p)
{
    if (kind == JOIN_KIND_HASH) return hash_plan(nR, nS, num_cus()).stamp;
    if (kind == JOIN_KIND_HASH_PREFILTER) return prefilter_plan(nR, nS, num_cus()).stamp;
    if (kind == JOIN_KIND_THETA_REGION) return plan_region(nR, nS, p).stamp;
    return plan_theta(nR, nS, p).stamp;
}

size_t ws_needed(int kind, int64_t nR, int64_t nS, const join_pred_t* p)
{
    if (kind == JOIN_KIND_HASH) return hash_plan(nR, nS, num_cus()).bytes;
    if (kind == JOIN_KIND_HASH_PREFILTER) return prefilter_plan(nR, nS, num_cus()).bytes;
    if (kind == JOIN_KIND_THETA_REGION) return plan_region(nR, nS, p).bytes;
    return plan_theta(nR, nS, p).bytes;
}

int check_ws(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* p, void* ws,
             size_t ws_bytes)
{
    const size_t need = ws_needed(kind, R->n, S->n, p);
    if (!ws || ws_bytes < need) {
        set_error("workspace %p of %zu bytes is smaller than the %zu bytes this join needs", ws,
                  ws_bytes, need);
        return JOIN_E_WORKSPACE;
    }
    return JOIN_OK;
}

// The last exact count on this thread, so that join_materialize can refuse a too-small output
// on the host without a device read.
struct LastCount {
    bool valid;
    int kind;
    join_rel_t R, S;
    join_pred_t p;
    void* ws;
    uint64_t count;
    uint64_t stamp;  // plan stamp of that count pass
};
thread_local LastCount g_last{};

bool same_rel(const join_rel_t& a, const join_rel_t& b)
{
    return a.key == b.key && a.key2 == b.key2 && a.rid == b.rid && a.n == b.n;
}

bool matches_last(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* p, void* ws)
{
    if (!g_last.valid || g_last.kind != kind || g_last.ws != ws) return false;
    if (!same_rel(g_last.R, *R) || !same_rel(g_last.S, *S)) return false;
    if (is_theta(kind) &&
        (g_last.p.op_a != p->op_a || g_last.p.op_c != p->op_c || g_last.p.w != p->w))
        return false;
    return true;
}

// Pinned 8-byte landing slot for the count read (one per thread, kept for the process).
uint64_t* pinned_slot()
{
    static thread_local uint64_t* slot = nullptr;
    if (!slot) {
        if (hipHostMalloc((void**)&slot, 64, hipHostMallocDefault) != hipSuccess) slot = nullptr;
    }
    return slot;
}

// The exact total, device -> pinned slot -> *count.  The host waits by polling an event instead
// of a blocking stream synchronisation: the total is on the critical path of every join (the
// output is allocated from it before the write pass), and a blocking wait adds the host thread's
// wake-up to that path.
hipError_t read_total(const void* src, hipStream_t st, uint64_t* count)
{
    uint64_t* slot = pinned_slot();
    if (!slot) return hipErrorOutOfMemory;
    static thread_local struct {
        int dev = -1;
        hipEvent_t ev = nullptr;
    } w;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (w.dev != dev) {  // an event belongs to the device current when it was made
        if (w.ev) (void)hipEventDestroy(w.ev);
        w.ev = nullptr;
        if (hipEventCreateWithFlags(&w.ev, hipEventDisableTiming) != hipSuccess) w.ev = nullptr;
        w.dev = dev;
    }
    e = hipMemcpyAsync(slot, src, sizeof(uint64_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    if (w.ev && hipEventRecord(w.ev, st) == hipSuccess) {
        while ((e = hipEventQuery(w.ev)) == hipErrorNotReady) __builtin_ia32_pause();
    } else {
        e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess) *count = *slot;
    return e;
}

// Count passes skip that copy: the kernel that produces the total also stores it into the pinned
// slot through the slot's device address (publish_total), and the host polls the slot.
// The slot holds kUnpublished until then; if the stream goes idle (or fails) with the slot
// unchanged, the wait ends with an error instead of spinning on.
constexpr uint64_t kUnpublished = ~0ull;

// Device address of this thread's pinned slot for the current device, NULL when the runtime
// gives none (then the copy above is used).  Looked up again when the thread's device changes.
uint64_t* published_slot()
{
    static thread_local struct {
        int dev = -1;
        uint64_t* addr = nullptr;
    } m;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (m.dev != dev) {
        m.dev = dev;
        m.addr = nullptr;
        uint64_t* slot = pinned_slot();
        void* d = nullptr;
        if (slot && hipHostGetDevicePointer(&d, slot, 0) == hipSuccess) m.addr = static_cast<uint64_t*>(d);
        else (void)hipGetLastError();
    }
    return m.addr;
}

hipError_t wait_published(hipStream_t st, uint64_t* count)
{
    volatile uint64_t* slot = pinned_slot();
    uint64_t v;
    uint32_t spins = 0;
    while ((v = *slot) == kUnpublished) {
        __builtin_ia32_pause();
        if ((++spins & 4095u) != 0) continue;
        const hipError_t q = hipStreamQuery(st);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return q;
        if ((v = *slot) == kUnpublished) return hipErrorLaunchFailure;  // idle, nothing stored
        break;
    }
    *count = v;
    return hipSuccess;
}

// The slot the next count pass stores its total into (NULL: read it by copy), reset first.
uint64_t* arm_published_slot()
{
    uint64_t* pub = published_slot();
    if (pub) *pinned_slot() = kUnpublished;
    return pub;
}

// The exact total of the count pass just enqueued: from the slot, or copied from `src`.
hipError_t take_total(uint64_t* pub, const void* src, hipStream_t st, uint64_t* count)
{
    return pub ? wait_published(st, count) : read_total(src, st, count);
}

#if JL_DEBUG
// The checking build's view of a workspace: where its per-unit written counts are, how many units
// to check against which offsets, and how much of it the fingerprint covers (the header and the
// written counts excluded; the pre-filter's inner workspace is not checked).
struct DebugView {
    size_t fp_end;    // fingerprint covers [256, fp_end)
    size_t off_dbg;   // per-unit written counts
    size_t off_offs;  // per-unit offsets left by the count pass
    int64_t units, nOff;
};

DebugView debug_view(int kind, int64_t nR, int64_t nS, const join_pred_t* p)
{
    DebugView v{};
    if (kind == JOIN_KIND_HASH) {
        const HashPlan pl = hash_plan(nR, nS, num_cus());
        v = DebugView{pl.off_dbg, pl.off_dbg, pl.off_counts, pl.Umax, pl.Umax};
    } else if (kind == JOIN_KIND_THETA) {
        const ThetaPlan pl = plan_theta(nR, nS, p);
        v = DebugView{pl.off_dbg, pl.off_dbg, pl.off_counts, pl.U, pl.U};
    } else if (kind == JOIN_KIND_THETA_REGION) {
        const RegionPlan pl = plan_region(nR, nS, p);
        v = DebugView{pl.off_dbg, pl.off_dbg, pl.off_counts, pl.Umax, pl.nOff};
    }
    return v;
}

// Fingerprint of the relations' columns and the workspace into the header word at `slot`.
hipError_t debug_fingerprint(int kind, const join_rel_t* R, const join_rel_t* S,
                             const join_pred_t* p, char* ws, size_t slot, hipStream_t st)
{
    uint64_t* out = reinterpret_cast<uint64_t*>(ws + slot);
    hipError_t e = dbg_zero(out, 1, st);
    const join_rel_t* X[2] = {R, S};
    for (int side = 0; side < 2 && e == hipSuccess; ++side) {
        const int32_t* cols[3] = {X[side]->key, X[side]->key2, X[side]->rid};
        for (int c = 0; c < 3 && e == hipSuccess; ++c)
            e = dbg_fingerprint(cols[c], (uint64_t)X[side]->n * 4, (uint64_t)(side * 3 + c) << 40, out, st);
    }
    const DebugView v = debug_view(kind, R->n, S->n, p);
    if (e == hipSuccess && v.fp_end > 256) e = dbg_fingerprint(ws + 256, v.fp_end - 256, 7ull << 40, out, st);
    return e;
}

hipError_t read_word(const void* src, uint64_t* v, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(v, src, 8, hipMemcpyDeviceToHost, st);
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
}
#endif

int count_impl(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* p, void* ws,
               hipStream_t st, uint64_t* count)
{
    g_last.valid = false;
    if (R->n == 0 || S->n == 0) {
        *count = 0;
    } else {
        char* w = static_cast<char*>(ws);
        hipError_t e;
        size_t total_at = 0;  // where the exact total lands in ws
        uint64_t* pub = arm_published_slot();
        if (kind == JOIN_KIND_HASH) {
            const HashPlan pl = hash_plan(R->n, S->n, num_cus());
            e = hash_count(pl, *R, *S, w, st, nullptr, pub);
        } else if (kind == JOIN_KIND_HASH_PREFILTER) {
            const PrefilterPlan pl = prefilter_plan(R->n, S->n, num_cus());
            e = prefilter_count(pl, *R, *S, w, st, num_cus(), pub);
            total_at = prefilter_total_offset(pl);
        } else if (kind == JOIN_KIND_THETA_REGION) {
            e = region_count(plan_region(R->n, S->n, p), *R, *S, *p, w, st, pub);
        } else {
            const ThetaPlan pl = plan_theta(R->n, S->n, p);
            e = theta_count(pl, *R, *S, *p, w, st, pub);
        }
        if (e != hipSuccess) return hip_fail(e, is_theta(kind) ? "theta count pass" : "hash count pass");
        e = take_total(pub, w + total_at, st, count);
        if (e != hipSuccess) return hip_fail(e, "reading the exact total");
#if JL_DEBUG
        e = debug_fingerprint(kind, R, S, p, w, kDebugFpOffset, st);
        if (e != hipSuccess) return hip_fail(e, "checking build: fingerprint");
#endif
    }
    g_last.valid = true;
    g_last.kind = kind;
    g_last.R = *R;
    g_last.S = *S;
    if (p) g_last.p = *p;
    g_last.ws = ws;
    g_last.count = *count;
    g_last.stamp = plan_stamp_of(kind, R->n, S->n, p);
    return JOIN_OK;
}

int write_impl(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* p, void* ws,
               int32_t* pairs, uint64_t capacity, hipStream_t st)
{
    if (R->n == 0 || S->n == 0) return JOIN_OK;
    if (capacity > 0 && !pairs) {
        set_error("pairs is NULL with capacity %llu", (unsigned long long)capacity);
        return JOIN_E_INVAL;
    }
    char* w = static_cast<char*>(ws);
    hipError_t e;
#if JL_DEBUG
    // the inputs and the workspace must be as join_count left them
    e = debug_fingerprint(kind, R, S, p, w, kDebugFp2Offset, st);
    uint64_t fp1 = 0, fp2 = 1;
    if (e == hipSuccess) e = read_word(w + kDebugFpOffset, &fp1, st);
    if (e == hipSuccess) e = read_word(w + kDebugFp2Offset, &fp2, st);
    if (e != hipSuccess) return hip_fail(e, "checking build: fingerprint");
    if (fp1 != fp2) {
        set_error("checking build: R, S or the workspace changed between join_count and join_materialize");
        return JOIN_E_INVAL;
    }
    const DebugView dv = debug_view(kind, R->n, S->n, p);
    if (dv.units > 0) {
        e = dbg_zero(reinterpret_cast<uint64_t*>(w + dv.off_dbg), dv.units, st);
        if (e == hipSuccess) e = dbg_zero(reinterpret_cast<uint64_t*>(w + kDebugBadOffset), 1, st);
        if (e != hipSuccess) return hip_fail(e, "checking build: clearing the written counts");
    }
#endif
    if (kind == JOIN_KIND_HASH) {
        const HashPlan pl = hash_plan(R->n, S->n, num_cus());
        e = hash_write(pl, *R, *S, w, pairs, capacity, st);
    } else if (kind == JOIN_KIND_HASH_PREFILTER) {
        e = prefilter_write(prefilter_plan(R->n, S->n, num_cus()), *R, *S, w, pairs, capacity, st, num_cus());
    } else if (kind == JOIN_KIND_THETA_REGION) {
        e = region_write(plan_region(R->n, S->n, p), *R, *S, *p, w, pairs, capacity, st);
    } else {
        const ThetaPlan pl = plan_theta(R->n, S->n, p);
        e = theta_write(pl, *R, *S, *p, w, pairs, capacity, st);
    }
    if (e != hipSuccess) return hip_fail(e, is_theta(kind) ? "theta write pass" : "hash write pass");
#if JL_DEBUG
    if (dv.units > 0) {
        uint64_t total = 0, bad = 0;
        e = read_word(w, &total, st);
        if (e == hipSuccess && total <= capacity)  // an output too small receives nothing
            e = dbg_check_units(reinterpret_cast<const uint64_t*>(w + dv.off_offs),
                                reinterpret_cast<const uint64_t*>(w),
                                reinterpret_cast<const uint64_t*>(w + dv.off_dbg), dv.units, dv.nOff,
                                reinterpret_cast<uint32_t*>(w + kDebugBadOffset), st);
        if (e == hipSuccess && total <= capacity) e = read_word(w + kDebugBadOffset, &bad, st);
        if (e != hipSuccess) return hip_fail(e, "checking build: written counts");
        if ((uint32_t)bad != 0) {
            set_error("checking build: %u work units wrote a number of pairs other than they counted",
                      (unsigned)(uint32_t)bad);
            return JOIN_E_INVAL;
        }
    }
#endif
    return JOIN_OK;
}

}  // namespace

extern "C" {

size_t join_workspace_bytes(int kind, int64_t nR, int64_t nS, const join_pred_t* pred)
{
    if ((kind != JOIN_KIND_HASH && kind != JOIN_KIND_THETA && kind != JOIN_KIND_THETA_REGION &&
         kind != JOIN_KIND_HASH_PREFILTER) ||
        nR < 0 || nS < 0)
        return 0;
    return ws_needed(kind, nR, nS, pred);
}

int join_count(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred,
               void* ws, size_t ws_bytes, void* stream, uint64_t* count)
{
    int rc = check_args(kind, R, S, pred);
    if (rc != JOIN_OK) return rc;
    if (!count) {
        set_error("count is NULL");
        return JOIN_E_INVAL;
    }
    if ((rc = check_ws(kind, R, S, pred, ws, ws_bytes)) != JOIN_OK) return rc;
    return count_impl(kind, R, S, pred, ws, static_cast<hipStream_t>(stream), count);
}

int join_materialize(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred,
                     void* ws, size_t ws_bytes, int32_t* pairs, uint64_t capacity, void* stream)
{
    int rc = check_args(kind, R, S, pred);
    if (rc != JOIN_OK) return rc;
    if ((rc = check_ws(kind, R, S, pred, ws, ws_bytes)) != JOIN_OK) return rc;
    if (matches_last(kind, R, S, pred, ws)) {
        if (g_last.stamp != plan_stamp_of(kind, R->n, S->n, pred)) {
            set_error("the plan differs from the one join_count ran on this workspace (a tuning "
                      "knob changed in between); count again");
            return JOIN_E_INVAL;
        }
        if (g_last.count > capacity) {
            set_error("capacity %llu is below the exact count %llu", (unsigned long long)capacity,
                      (unsigned long long)g_last.count);
            return JOIN_E_CAPACITY;
        }
    }
    return write_impl(kind, R, S, pred, ws, pairs, capacity, static_cast<hipStream_t>(stream));
}

static int one_shot(int kind, const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred,
                    void* ws, size_t ws_bytes, int32_t* pairs, uint64_t capacity, uint64_t* count,
                    void* stream)
{
    int rc = check_args(kind, R, S, pred);
    if (rc != JOIN_OK) return rc;
    if (!count) {
        set_error("count is NULL");
        return JOIN_E_INVAL;
    }
    if ((rc = check_ws(kind, R, S, pred, ws, ws_bytes)) != JOIN_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = count_impl(kind, R, S, pred, ws, st, count)) != JOIN_OK) return rc;
    if (*count > capacity) {
        set_error("capacity %llu is below the exact count %llu", (unsigned long long)capacity,
                  (unsigned long long)*count);
        return JOIN_E_CAPACITY;
    }
    return write_impl(kind, R, S, pred, ws, pairs, capacity, st);
}

int join_hash(const join_rel_t* R, const join_rel_t* S, void* ws, size_t ws_bytes, int32_t* pairs,
              uint64_t capacity, uint64_t* count, void* stream)
{
    return one_shot(JOIN_KIND_HASH, R, S, nullptr, ws, ws_bytes, pairs, capacity, count, stream);
}

int join_theta(const join_rel_t* R, const join_rel_t* S, const join_pred_t* pred, void* ws,
               size_t ws_bytes, int32_t* pairs, uint64_t capacity, uint64_t* count, void* stream)
{
    return one_shot(JOIN_KIND_THETA, R, S, pred, ws, ws_bytes, pairs, capacity, count, stream);
}

const char* join_last_error(void) { return g_err; }

size_t join_scan_workspace_bytes(int64_t n)
{
    if (n < 0) return 0;
    return scan_temp_elems<uint64_t>(n) * sizeof(uint64_t) + 256;
}

int join_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total, void* ws,
                  size_t ws_bytes, void* stream)
{
    if (n < 0 || (n > 0 && (!in || !out))) {
        set_error("join_scan_u64: bad arguments (n = %lld)", (long long)n);
        return JOIN_E_INVAL;
    }
    const size_t need = join_scan_workspace_bytes(n);
    if (!ws || ws_bytes < need) {
        set_error("join_scan_u64: workspace of %zu bytes is below %zu", ws_bytes, need);
        return JOIN_E_WORKSPACE;
    }
    hipError_t e = exclusive_scan<uint64_t>(in, out, n, total, static_cast<uint64_t*>(ws),
                                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "join_scan_u64");
    return JOIN_OK;
}

static_assert(sizeof(BatchPlan) <= sizeof(join_batch_plan_t), "batch plan must fit the opaque blob");

static int check_jobs(int njobs, const join_job_t* jobs)
{
    if (njobs < 0 || (njobs > 0 && !jobs)) {
        set_error("njobs < 0 or jobs == NULL");
        return JOIN_E_INVAL;
    }
    for (int j = 0; j < njobs; ++j) {
        int rc = check_rel(&jobs[j].R, "R", false);
        if (rc == JOIN_OK) rc = check_rel(&jobs[j].S, "S", false);
        if (rc != JOIN_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "job %d: %s", j, join_last_error());
            set_error("%s", msg);
            return rc;
        }
        if (jobs[j].bits > 11 || jobs[j].reserved != 0) {
            set_error("job %d: bits must be < 0 (default) or 0..11, reserved must be 0", j);
            return JOIN_E_INVAL;
        }
    }
    return JOIN_OK;
}

size_t join_batch_workspace_bytes(int njobs, const join_job_t* jobs)
{
    if (check_jobs(njobs, jobs) != JOIN_OK) return 0;
    BatchPlan bp;
    if (hash_batch_plan(njobs, jobs, num_cus(), &bp) != 0) return 0;
    return (size_t)bp.bytes;
}

int join_batch_prepare(int njobs, const join_job_t* jobs, void* ws, size_t ws_bytes,
                       join_batch_plan_t* plan, void* stream)
{
    int rc = check_jobs(njobs, jobs);
    if (rc != JOIN_OK) return rc;
    if (!plan) {
        set_error("plan == NULL");
        return JOIN_E_INVAL;
    }
    BatchPlan bp;
    if (hash_batch_plan(njobs, jobs, num_cus(), &bp) != 0) {
        set_error("batch too large: rows per side, partitions or work units exceed 32-bit indices");
        return JOIN_E_UNSUPPORTED;
    }
    if (!ws || ws_bytes < bp.bytes) {
        set_error("workspace of %zu bytes, need %llu", ws_bytes, (unsigned long long)bp.bytes);
        return JOIN_E_WORKSPACE;
    }
    memset(plan, 0, sizeof(*plan));
    memcpy(plan, &bp, sizeof(bp));
    const hipError_t e = hash_batch_upload(bp, jobs, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JOIN_OK : hip_fail(e, "join_batch_prepare");
}

static int batch_args(const join_batch_plan_t* plan, void* ws, size_t ws_bytes, BatchPlan* bp)
{
    if (!plan) {
        set_error("plan == NULL");
        return JOIN_E_INVAL;
    }
    memcpy(bp, plan, sizeof(*bp));
    if (!ws || ws_bytes < bp->bytes) {
        set_error("workspace of %zu bytes, need %llu", ws_bytes, (unsigned long long)bp->bytes);
        return JOIN_E_WORKSPACE;
    }
    return JOIN_OK;
}

int join_batch_count(const join_batch_plan_t* plan, void* ws, size_t ws_bytes, uint64_t* offsets,
                     void* stream)
{
    BatchPlan bp;
    int rc = batch_args(plan, ws, ws_bytes, &bp);
    if (rc != JOIN_OK) return rc;
    if (!offsets) {
        set_error("offsets == NULL");
        return JOIN_E_INVAL;
    }
    const hipError_t e = hash_batch_count(bp, static_cast<char*>(ws), offsets, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JOIN_OK : hip_fail(e, "join_batch_count");
}

int join_batch_materialize(const join_batch_plan_t* plan, void* ws, size_t ws_bytes, int32_t* pairs,
                           uint64_t capacity, void* stream)
{
    BatchPlan bp;
    int rc = batch_args(plan, ws, ws_bytes, &bp);
    if (rc != JOIN_OK) return rc;
    if (!pairs && capacity > 0) {
        set_error("pairs == NULL with capacity > 0");
        return JOIN_E_INVAL;
    }
    const hipError_t e = hash_batch_write(bp, static_cast<char*>(ws), pairs, capacity, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JOIN_OK : hip_fail(e, "join_batch_materialize");
}

static_assert(sizeof(BuildPlan) <= sizeof(join_build_t), "build plan must fit the opaque blob");

static thread_local struct {
    bool valid;
    const void* build;
    join_rel_t S;
    void* ws;
    uint64_t count;
    uint64_t stamp;
} g_last_probe{};

size_t join_build_bytes(int64_t nR)
{
    if (nR < 0 || nR > kMaxRows) return 0;
    return (size_t)hash_build_plan(nR, num_cus()).bytes;
}

int join_build(const join_rel_t* R, void* build, size_t build_bytes, join_build_t* desc, void* stream)
{
    int rc = check_rel(R, "R", false);
    if (rc != JOIN_OK) return rc;
    if (!desc) {
        set_error("desc == NULL");
        return JOIN_E_INVAL;
    }
    const BuildPlan b = hash_build_plan(R->n, num_cus());
    if (!build || build_bytes < b.bytes) {
        set_error("build buffer of %zu bytes, need %llu", build_bytes, (unsigned long long)b.bytes);
        return JOIN_E_WORKSPACE;
    }
    memset(desc, 0, sizeof(*desc));
    memcpy(desc, &b, sizeof(b));
    if (R->n == 0) return JOIN_OK;
    const hipError_t e = hash_build(b, *R, static_cast<char*>(build), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? JOIN_OK : hip_fail(e, "join_build");
}

static int probe_args(const join_build_t* desc, const void* build, const join_rel_t* S, BuildPlan* b)
{
    if (!desc) {
        set_error("desc == NULL");
        return JOIN_E_INVAL;
    }
    memcpy(b, desc, sizeof(*b));
    if (b->nR < 0 || b->bits < 1 || b->bits > 11) {
        set_error("desc does not describe a build");
        return JOIN_E_INVAL;
    }
    if (b->nR > 0 && !build) {
        set_error("build == NULL");
        return JOIN_E_INVAL;
    }
    return check_rel(S, "S", false);
}

size_t join_probe_workspace_bytes(const join_build_t* desc, int64_t nS)
{
    BuildPlan b;
    if (!desc || nS < 0 || nS > kMaxRows) return 0;
    memcpy(&b, desc, sizeof(b));
    if (b.bits < 1 || b.bits > 11) return 0;
    return (size_t)hash_plan(b.nR, nS, num_cus(), b.bits).bytes;
}

int join_probe_count(const join_build_t* desc, const void* build, const join_rel_t* S, void* ws,
                     size_t ws_bytes, void* stream, uint64_t* count)
{
    BuildPlan b;
    int rc = probe_args(desc, build, S, &b);
    if (rc != JOIN_OK) return rc;
    if (!count) {
        set_error("count == NULL");
        return JOIN_E_INVAL;
    }
    g_last_probe.valid = false;
    const HashPlan pl = hash_plan(b.nR, S->n, num_cus(), b.bits);
    if (!ws || ws_bytes < pl.bytes) {
        set_error("workspace of %zu bytes, need %llu", ws_bytes, (unsigned long long)pl.bytes);
        return JOIN_E_WORKSPACE;
    }
    if (b.nR == 0 || S->n == 0) {
        *count = 0;
    } else {
        hipStream_t st = static_cast<hipStream_t>(stream);
        join_rel_t R{};
        R.n = b.nR;
        const RView v = build_view(b, build);
        uint64_t* pub = arm_published_slot();
        const hipError_t e = hash_count(pl, R, *S, static_cast<char*>(ws), st, &v, pub);
        if (e != hipSuccess) return hip_fail(e, "probe count pass");
        const hipError_t er = take_total(pub, ws, st, count);
        if (er != hipSuccess) return hip_fail(er, "reading the exact total");
    }
    g_last_probe.valid = true;
    g_last_probe.build = build;
    g_last_probe.S = *S;
    g_last_probe.ws = ws;
    g_last_probe.count = *count;
    g_last_probe.stamp = pl.stamp;
    return JOIN_OK;
}

int join_probe_materialize(const join_build_t* desc, const void* build, const join_rel_t* S,
                           void* ws, size_t ws_bytes, int32_t* pairs, uint64_t capacity, void* stream)
{
    BuildPlan b;
    int rc = probe_args(desc, build, S, &b);
    if (rc != JOIN_OK) return rc;
    const HashPlan pl = hash_plan(b.nR, S->n, num_cus(), b.bits);
    if (!ws || ws_bytes < pl.bytes) {
        set_error("workspace of %zu bytes, need %llu", ws_bytes, (unsigned long long)pl.bytes);
        return JOIN_E_WORKSPACE;
    }
    if (capacity > 0 && !pairs) {
        set_error("pairs is NULL with capacity %llu", (unsigned long long)capacity);
        return JOIN_E_INVAL;
    }
    if (g_last_probe.valid && g_last_probe.build == build && g_last_probe.ws == ws &&
        same_rel(g_last_probe.S, *S)) {
        if (g_last_probe.stamp != pl.stamp) {
            set_error("the plan differs from the one join_probe_count ran on this workspace (a "
                      "tuning knob changed in between); count again");
            return JOIN_E_INVAL;
        }
        if (g_last_probe.count > capacity) {
            set_error("capacity %llu < exact count %llu", (unsigned long long)capacity,
                      (unsigned long long)g_last_probe.count);
            return JOIN_E_CAPACITY;
        }
    }
    if (b.nR == 0 || S->n == 0) return JOIN_OK;
    join_rel_t R{};
    R.n = b.nR;
    const RView v = build_view(b, build);
    const hipError_t e = hash_write(pl, R, *S, static_cast<char*>(ws), pairs, capacity,
                                    static_cast<hipStream_t>(stream), &v);
    return e == hipSuccess ? JOIN_OK : hip_fail(e, "probe write pass");
}

}  // extern "C"
