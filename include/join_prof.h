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

/* ---- measured ceilings ----------------------------------------------------------------------
 * Plain kernels whose rates are what the chip sustains, so that roofline fractions can be
 * given against measured ceilings beside the published ones.  Both are stream-ordered on `stream`
 * (a hipStream_t passed as void*, NULL = the null stream),
 * allocate nothing, and are timed as "ceiling.copy", "ceiling.read", "ceiling.write", "ceiling.valu" (mix 0), "ceiling.valu.band" (mix 1) and
 * "ceiling.valu.min" (mix 2) while profiling is on. */

/* Copy `bytes` from device buffer src to device buffer dst (both 16-byte aligned, bytes a
 * multiple of 16, not overlapping) with a grid-stride kernel of 16-byte non-temporal loads and
 * stores, 4 in flight per lane, at most 2 workgroups of 1024 lanes per compute unit.  HBM
 * traffic is 2 * bytes.  JOIN_E_INVAL for a misaligned or null argument. */
int join_prof_copy(const void* src, void* dst, uint64_t bytes, void* stream);

/* One streaming pass over `bytes` of device memory (16-byte aligned, a multiple of 16), 16-byte
 * non-temporal accesses, at most 2 workgroups of 1024 lanes per compute unit.  mode 1 reads src
 * (8 loads in flight per lane) and stores one word per lane of the grid into dst (dst holds at
 * least 2 * 1024 * 4 * compute units bytes); mode 2 writes dst (4 stores in flight per lane; src
 * unused).  HBM traffic is `bytes`.  Timed as "ceiling.read" / "ceiling.write".  JOIN_E_INVAL
 * for another mode, a misaligned size or pointer, or a needed pointer that is null. */
int join_prof_stream(int mode, const void* src, void* dst, uint64_t bytes, void* stream);

/* Run `blocks` workgroups of 256 lanes; every lane issues 32 * iters (mix 0, 1, 3, 4) or 48 * iters
 * (mix 2) int32 VALU instructions, so the launch performs blocks * 256 * that many
 * lane-operations.  mix 0: 16 independent chains of v_add_u32 + v_xor_b32 per lane,
 * a[j] = 16 * lane + j, a[j] <- (a[j] + b) ^ b with b = 0x9E3779B9 ^ workgroup, and
 * sink[lane] = the xor of the 16 chains.  mix 1: a band test, v_sub_u32 t = b - a[j],
 * v_cmp_le_u32 t <= 2^20 into VCC and s_or_b64 of VCC into a 64-bit wave mask, and
 * sink[lane] = the mask's two halves xored.  mix 2: the nested-loop join's group filter, for
 * every pair (a[j], a[j+1]) two v_sub_u32 from b and a v_min3_u32 into one of two running
 * minima, twice per iteration, and sink[lane] = the smaller minimum (all ones when iters == 0).
 * mix 3: two v_sub_u32 a[j] = b - a[j] per chain (b from a scalar register); mix 4: two
 * v_min3_u32 per chain, a[j] = min(a[j], b, 2^20); for both, sink[lane] = the xor of the 16
 * chains.  Timed as "ceiling.valu.sub" and "ceiling.valu.min3".  sink: device
 * array of blocks * 256 uint32; clk: device array of 2 uint64 that receives the shader clock
 * cycles and the real-time counter ticks workgroup 0 spent in its loop (the real-time counter's
 * rate comes from join_prof_wall_clock_khz).  JOIN_E_INVAL for blocks outside [1, 2^22], a mix
 * outside 0..4, or a null pointer. */
int join_prof_valu(uint32_t blocks, uint32_t iters, int mix, uint32_t* sink, uint64_t* clk,
                   void* stream);

/* Rate of the device's constant real-time counter in kHz (current device). */
int join_prof_wall_clock_khz(int* khz);

#ifdef __cplusplus
}
#endif

#endif /* JOIN_PROF_H */
