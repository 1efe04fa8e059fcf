/* join_tune.h -- process-wide tuning knobs of libjoin.
 *
 * The knobs change only how the work is cut up (table capacity, fan-out, tile shapes) and, for
 * "hash.deterministic", the order of the output pairs, never the multiset of pairs.  The paper
 * tunes its own cut of the work, the reducer count alpha, by measurement (Section 3.3.4,
 * equation "hier"; Sections 5.1.4 and 5.2.4); these knobs are what the project's autotuner sets
 * from its measured cache.
 *
 * Every knob is read when a call plans its work, so a workspace sized under one setting must
 * be counted and materialized under the same setting.  The count pass records a signature of
 * its plan in the workspace; a write pass whose plan differs writes nothing (and
 * join_materialize returns JOIN_E_INVAL when the count ran on the same thread).  A value set for
 * the calling thread (join_tune_set_local) wins over a process-wide one (join_tune_set), which
 * wins over the environment variable of the same knob, which wins over the built-in default.
 * Process-wide setting is atomic per knob; concurrent calls that plan while a knob changes may
 * see either value, so a caller that tunes one call should use the thread's own setting.
 *
 * Knobs (name, environment variable, meaning):
 *   "hash.cap"               JOIN_HASH_CAP                R entries per LDS table, 64..9728
 *                                                         (batches: at most 4608, the table of
 *                                                         their 512-thread workgroups)
 *   "hash.slice"             JOIN_HASH_SLICE              S rows per work unit, >= 1024
 *   "hash.bits"              JOIN_HASH_BITS               single-join fan-out log2, -1 automatic
 *   "hash.single_max_chunks" JOIN_HASH_SINGLE_MAX_CHUNKS  R up to this many tables: no partitioning
 *   "theta.ts"               JOIN_THETA_TS                S rows per theta tile, 0 automatic
 *   "theta.waves"            JOIN_THETA_WAVES             waves a theta grid aims for, 0 automatic
 *   "theta.stash"            JOIN_THETA_STASH             matches stashed per theta work unit
 *   "hash.deterministic"     JOIN_HASH_DETERMINISTIC      1: partitioned hash joins (single and
 *                                                         batched) place tuples in an order fixed by
 *                                                         the input, so their output order is the
 *                                                         same on every run; 0 (default): arrival
 *                                                         order, faster.  Joins on the unpartitioned
 *                                                         path are deterministic either way.
 */
#ifndef JOIN_TUNE_H
#define JOIN_TUNE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JOIN_TUNE_UNKNOWN 1 /* no knob of that name (or value == NULL) */

/* Sets knob `name` to `value`, or back to its environment/default value if clear != 0.
 * Returns 0 or JOIN_TUNE_UNKNOWN. */
int join_tune_set(const char* name, int64_t value, int clear);

/* Sets knob `name` for the calling thread only (or clears that setting if clear != 0): calls
 * made by other threads do not see it.  Returns 0 or JOIN_TUNE_UNKNOWN. */
int join_tune_set_local(const char* name, int64_t value, int clear);

/* Current value of knob `name` as the calling thread sees it (its own setting, else the
 * process-wide one, else environment, else `dflt`) into *value.
 * Returns 0 or JOIN_TUNE_UNKNOWN. */
int join_tune_get(const char* name, int64_t dflt, int64_t* value);

#ifdef __cplusplus
}
#endif

#endif /* JOIN_TUNE_H */
