// The angular-spectrum step with the exact (non-paraxial) transfer function (Sec. 1.1, the
// angular-spectrum method without the paraxial approximation): the transfer function
// H = exp(2 pi i z (sqrt(1/lambda^2 - f^2) - 1/lambda)) is not separable, so a plane takes three
// sweeps: row FFT (with the optic), column FFT * H * inverse column FFT, inverse row FFT.
#pragma once
#include "fr_internal.h"

namespace fr {

// count planes of power-of-two edge n (count <= kMaxBatch), forward or (FR_ADJOINT) adjoint,
// in place; `planes[i].h` points at two float64 parameters, z / lambda and (lambda / (n dx))^2,
// `lens` at the thin lens or null
hipError_t launch_exact_batch(const PlaneArgs *planes, int count, int n, const float2 *tw, hipStream_t s,
                              const LaunchHook &hook);

}  // namespace fr
