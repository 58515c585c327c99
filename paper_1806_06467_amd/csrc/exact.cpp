// fresnel_step_exact: the angular-spectrum step with the exact (non-paraxial) transfer function
// (Sec. 1.1, the angular-spectrum method without the paraxial approximation), three sweeps per
// plane (fr_exact.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/fresnel.h"
#include "fr_exact.h"
#include "fr_runtime.h"

namespace {

uint64_t dbits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof u);
  return u;
}

// one checked plane's arguments with its tables fetched (z / lambda and (lambda / (n dx))^2 in
// float64, the lens chirp, the twiddles); returns the plane's warning bits or an error
int exact_plane(fr::Ctx *ctx, const fr_plane &p, hipStream_t s, fr::PlaneArgs *a, const float2 **root,
                bool *split_out) {
  const int n = p.n;
  std::memset(a, 0, sizeof *a);
  a->field = reinterpret_cast<float2 *>(p.field);
  a->amp = p.amp;
  a->opd = p.opd_m;
  a->n = n;
  a->win = n;
  a->inv_lambda = float(1.0 / p.wavelength_m);
  a->flags = p.flags;
  // float64 words: z / lambda, (lambda / (n dx))^2, the split flag, padding; with the split flag
  // set, then n float2: the paraxial factor along one axis, exp(-i pi lambda z k~^2 / (n dx)^2) / n
  // over the signed index k~ (so that H = h[kx] h[ky] exp(2 pi i c), with the non-separable rest
  // c = -(z / lambda) u^2 / (2 (1 + sqrt(1 - u))^2) turns, u = (lambda f)^2, small enough to form
  // in float32: no evanescent frequency on the grid and |c| <= 1/4 turn)
  const double q = p.wavelength_m / (double(n) * p.dx_m);
  const double zl = p.z_m / p.wavelength_m, a2 = q * q;
  const double umax = a2 * 2.0 * double(n / 2) * double(n / 2);
  const double rmax = 1.0 + std::sqrt(std::max(0.0, 1.0 - umax));
  const bool split = umax < 1.0 && std::fabs(zl) * umax * umax / (2.0 * rmax * rmax) <= 0.25;
  *split_out = split;
  const fr::TableKey key{fr::kExactPrm, n, dbits(p.dx_m), dbits(p.wavelength_m), dbits(p.z_m), 0};
  void *d = nullptr;
  if (auto it = ctx->tables.find(key); it != ctx->tables.end()) {
    d = it->second;
  } else {
    std::vector<double> prm(4 + (split ? n : 0), 0.0);
    prm[0] = zl;
    prm[1] = a2;
    prm[2] = split ? 1.0 : 0.0;
    if (split) {
      float2 *h = reinterpret_cast<float2 *>(prm.data() + 4);
      for (int k = 0; k < n; ++k) {
        const double kk = double(k < n / 2 ? k : k - n);
        double t = -0.5 * zl * a2 * kk * kk;
        t -= std::rint(t);
        h[k] = make_float2(float(std::cos(2.0 * M_PI * t) / n), float(std::sin(2.0 * M_PI * t) / n));
      }
    }
    const int st = ctx->upload(key, prm.data(), prm.size() * sizeof(double), s, &d);
    if (st != FR_OK) return st;
  }
  a->h = static_cast<const float2 *>(d);
  if (p.lens_focal_m != 0.0) {
    const int st = ctx->lens(n, p.dx_m, p.wavelength_m, p.lens_focal_m, s, &a->lens);
    if (st != FR_OK) return st;
  }
  if (const int st = ctx->twiddles(n, s, root); st != FR_OK) return st;
  return std::fabs(p.z_m) > double(n) * p.dx_m * p.dx_m / p.wavelength_m ? FR_W_AS_UNDERSAMPLED : FR_OK;
}

}  // namespace

extern "C" int fresnel_step_exact(fr_ctx *ctx_, fr_c64 *field, int32_t n, double dx_m, double wavelength_m,
                                  double z_m, const float *amp, const float *opd_m, double lens_focal_m,
                                  int32_t flags, void *stream) {
  fr_plane p;
  p.field = field;
  p.amp = amp;
  p.opd_m = opd_m;
  p.dx_m = dx_m;
  p.wavelength_m = wavelength_m;
  p.z_m = z_m;
  p.lens_focal_m = lens_focal_m;
  p.n = n;
  p.flags = flags;
  return fresnel_step_exact_batched(ctx_, &p, 1, stream);
}

extern "C" int fresnel_step_exact_batched(fr_ctx *ctx_, const fr_plane *planes, int32_t count, void *stream) {
  if (!planes || count <= 0) return FR_EINVAL;
  const int n = planes[0].n;
  for (int i = 0; i < count; ++i) {
    const fr_plane &p = planes[i];
    if (!p.field || p.n != n || n <= 0 || (p.flags & ~FR_ADJOINT)) return FR_EINVAL;
    if (!(p.dx_m > 0) || !(p.wavelength_m > 0) || !std::isfinite(p.dx_m) || !std::isfinite(p.wavelength_m) ||
        !std::isfinite(p.z_m) || !std::isfinite(p.lens_focal_m))
      return FR_EINVAL;
  }
  if (!fr::fresnel_size_supported(n)) return FR_EUNSUPPORTED;
  fr::Ctx *ctx = reinterpret_cast<fr::Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  // planes per launch: as many as the last-level cache holds between a plane's three sweeps
  const size_t plane_bytes = size_t(n) * size_t(n) * 8u;
  const int group = int(std::max<size_t>(1, std::min<size_t>(fr::kMaxBatch, fr::kCacheGroupBytes / plane_bytes)));
  int warn = 0;
  std::vector<fr::PlaneArgs> args(group);
  for (int i0 = 0; i0 < count; i0 += group) {
    const int g = std::min(group, count - i0);
    const float2 *root = nullptr;
    // the planes whose H takes the split form (as in a call of their own)
    uint64_t split_mask = 0;
    for (int j = 0; j < g; ++j) {
      bool split = false;
      const int st = exact_plane(ctx, planes[i0 + j], s, &args[j], &root, &split);
      if (st < 0) return st;
      warn |= st;
      if (split) split_mask |= uint64_t(1) << j;
    }
    e = fr::launch_exact_batch(args.data(), g, n, root, s, ctx->hook(), split_mask);
    if (e != hipSuccess) return fr::record_hip(e);
  }
  return warn;
}
