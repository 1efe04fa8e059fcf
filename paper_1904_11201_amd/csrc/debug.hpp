// debug.hpp -- checks of the checking build (compiled with JL_DEBUG=1).
//
// * Fingerprints: join_count stores a fingerprint of R, S and the workspace (past its header) in
//   the workspace header; join_materialize computes it again and refuses to write when it
//   differs (the caller must not change R, S or ws in between).
// * Written vs counted: the write passes add up, per work unit, the pairs they write into a
//   debug array of the workspace; a check kernel compares each with the unit's share of the
//   offsets the count pass left, and join_materialize reports a mismatch.
#pragma once
#include "common.hpp"

#ifndef JL_DEBUG
#define JL_DEBUG 0
#endif

namespace jl {

constexpr size_t kDebugFpOffset = 72;   // uint64: fingerprint left by join_count
constexpr size_t kDebugFp2Offset = 80;  // uint64: fingerprint at join_materialize
constexpr size_t kDebugBadOffset = 88;  // uint32: work units whose written count differs

hipError_t dbg_zero(uint64_t* p, int64_t n, hipStream_t st);
// Adds the fingerprint of bytes [p, p + bytes) (whole 32-bit words; salt tells buffers apart)
// to *out.
hipError_t dbg_fingerprint(const void* p, uint64_t bytes, uint64_t salt, uint64_t* out, hipStream_t st);
// Counts into *bad the units u < units whose written[u] differs from offsets[u + 1] - offsets[u]
// (offsets has nOff entries; the last unit's end is *total).
hipError_t dbg_check_units(const uint64_t* offsets, const uint64_t* total, const uint64_t* written,
                           int64_t units, int64_t nOff, uint32_t* bad, hipStream_t st);

}  // namespace jl
