// tune.hpp -- tuning knobs read at plan time: a value set through join_tune_set wins over the
// environment variable, which wins over the built-in default.
#pragma once
#include <stdint.h>

namespace jl {

enum TuneKnob {
    TUNE_HASH_CAP = 0,     // R entries per LDS table ("hash.cap", JOIN_HASH_CAP)
    TUNE_HASH_SLICE,       // S rows per work unit ("hash.slice", JOIN_HASH_SLICE)
    TUNE_HASH_BITS,        // fan-out of single joins, -1 = automatic ("hash.bits", JOIN_HASH_BITS)
    TUNE_HASH_SINGLE_MAX,  // largest R, in LDS chunks, joined without partitioning ("hash.single_max_chunks")
    TUNE_THETA_TS,         // S rows per theta tile, 0 = automatic ("theta.ts", JOIN_THETA_TS)
    TUNE_THETA_WAVES,      // waves the theta grid aims for, 0 = automatic ("theta.waves")
    TUNE_THETA_STASH,      // matches stashed per theta unit ("theta.stash", JOIN_THETA_STASH)
    TUNE_HASH_DETERMINISTIC,  // 1: ordered scatter, output order fixed ("hash.deterministic")
    TUNE_COUNT
};

int64_t tune_get(TuneKnob k, int64_t dflt);

}  // namespace jl
