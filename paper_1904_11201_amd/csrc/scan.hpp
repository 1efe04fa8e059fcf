// scan.hpp -- device exclusive prefix sums.
#pragma once
#include "common.hpp"

namespace jl {

// Elements of temporary storage exclusive_scan<T> needs for n values.
template <typename T>
size_t scan_temp_elems(int64_t n);

// out[i] = sum(in[0..i)); *total (device, may be NULL) = sum(in[0..n)).  in may equal out.
// pub (may be NULL): a pinned host slot that also receives the sum.  Enqueued on `st`; no host
// synchronisation.
template <typename T>
hipError_t exclusive_scan(const T* in, T* out, int64_t n, T* total, T* temp, hipStream_t st,
                         uint64_t* pub = nullptr);

}  // namespace jl
