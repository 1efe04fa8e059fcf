/*
 * join_prof.h -- opt-in per-kernel timing of libjoin launches with HIP events.
 *
 * Instrumentation, not part of the join method: when enabled, every kernel launch the library
 * makes is bracketed by two hipEventRecord calls on the launch's own stream, and
 * join_prof_collect() waits for the recorded events and accumulates hipEventElapsedTime per
 * kernel name.  Used to measure each kernel's average launch duration for roofline figures.
 * Events are created by the library (host-side handles); no device memory is allocated.
 * Thread-safe.  All calls return JOIN_OK (0) or JOIN_E_HIP (4) with join_last_error() set.
 */
#ifndef JOIN_PROF_H
#define JOIN_PROF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* on != 0 starts recording (and clears earlier totals); on == 0 stops recording. */
int join_prof_enable(int on);

/* Wait for every recorded launch and fold its duration into the per-name totals. */
int join_prof_collect(void);

/* Number of distinct kernel names with totals. */
int join_prof_count(void);

/* Entry i (0 <= i < join_prof_count()): kernel name (valid until the next enable), number of
 * launches and summed duration in milliseconds.  Returns JOIN_E_INVAL (1) for a bad index. */
int join_prof_entry(int i, const char** name, uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* JOIN_PROF_H */
