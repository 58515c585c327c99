// The angular-spectrum step with the exact (non-paraxial) transfer function (Sec. 1.1, the
// angular-spectrum method without the paraxial approximation): the transfer function
// H = exp(2 pi i z (sqrt(1/lambda^2 - f^2) - 1/lambda)) is not separable, so a plane takes three
// sweeps: row FFT (with the optic), column FFT * H * inverse column FFT, inverse row FFT.
#pragma once
#include "fr_internal.h"

namespace fr {

// count planes of power-of-two edge n (count <= kMaxBatch), forward or (FR_ADJOINT) adjoint,
// in place; `planes[i].h` points at float64 words z / lambda, (lambda / (n dx))^2, a split flag
// and padding, then (split flag 1) the n float2 of the paraxial factor along one axis (H is
// then formed as h[kx] h[ky] times a small float32 rest); `lens` at the thin lens or null
// split: bit i set when plane i's table carries the split form (its column sweep then forms H in
// registers)
hipError_t launch_exact_batch(const PlaneArgs *planes, int count, int n, const float2 *tw, hipStream_t s,
                              const LaunchHook &hook, uint64_t split);

}  // namespace fr
