// kernels_io.hpp -- conversions between the storage type S and FP32 device
// arrays at the library boundary (fields set from, or read into, FP32).
// Values are formed in FP64 as for the FP64 entry points and rounded once to
// FP32 (reads) or to S (sets).
#pragma once
#include "kernels.hpp"

namespace tcp {

template <typename S>
void launch_from_f32(const float *src, void *dst, int64_t n, hipStream_t s);
template <typename S>
void launch_read_f32(const ReadArgs &a, float *out, hipStream_t s);

} // namespace tcp
