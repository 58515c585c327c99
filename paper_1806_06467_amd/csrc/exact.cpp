// fresnel_step_exact: the angular-spectrum step with the exact (non-paraxial) transfer function
// (Sec. 1.1, the angular-spectrum method without the paraxial approximation), three sweeps per
// plane (fr_exact.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/fresnel.h"
#include "fr_exact.h"
#include "fr_runtime.h"

namespace {

uint64_t dbits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof u);
  return u;
}

}  // namespace

extern "C" int fresnel_step_exact(fr_ctx *ctx_, fr_c64 *field, int32_t n, double dx_m, double wavelength_m,
                                  double z_m, const float *amp, const float *opd_m, double lens_focal_m,
                                  int32_t flags, void *stream) {
  if (!field || n <= 0 || (flags & ~FR_ADJOINT)) return FR_EINVAL;
  if (!(dx_m > 0) || !(wavelength_m > 0) || !std::isfinite(dx_m) || !std::isfinite(wavelength_m) ||
      !std::isfinite(z_m) || !std::isfinite(lens_focal_m))
    return FR_EINVAL;
  if (!fr::fresnel_size_supported(n)) return FR_EUNSUPPORTED;
  fr::Ctx *ctx = reinterpret_cast<fr::Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  fr::PlaneArgs a;
  std::memset(&a, 0, sizeof a);
  a.field = reinterpret_cast<float2 *>(field);
  a.amp = amp;
  a.opd = opd_m;
  a.n = n;
  a.win = n;
  a.inv_lambda = float(1.0 / wavelength_m);
  a.flags = flags;
  // z / lambda and (lambda / (n dx))^2, in float64 on the device
  const fr::TableKey key{fr::kExactPrm, n, dbits(dx_m), dbits(wavelength_m), dbits(z_m), 0};
  void *d = nullptr;
  if (auto it = ctx->tables.find(key); it != ctx->tables.end()) {
    d = it->second;
  } else {
    const double q = wavelength_m / (double(n) * dx_m);
    const double prm[2] = {z_m / wavelength_m, q * q};
    const int st = ctx->upload(key, prm, sizeof prm, s, &d);
    if (st != FR_OK) return st;
  }
  a.h = static_cast<const float2 *>(d);
  if (lens_focal_m != 0.0) {
    const int st = ctx->lens(n, dx_m, wavelength_m, lens_focal_m, s, &a.lens);
    if (st != FR_OK) return st;
  }
  const float2 *root;
  int st = ctx->twiddles(n, s, &root);
  if (st != FR_OK) return st;
  e = fr::launch_exact_batch(&a, 1, n, root, s, ctx->hook());
  if (e != hipSuccess) return fr::record_hip(e);
  return std::fabs(z_m) > double(n) * dx_m * dx_m / wavelength_m ? FR_W_AS_UNDERSAMPLED : FR_OK;
}
