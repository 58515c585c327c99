// A multi-optic system propagated plane by plane (App. B: the paper's benchmark is a relay of
// optics -- a telescope aperture and primary, relay mirrors as thin lenses, a shaped pupil, a
// focal-plane mask, a final focus -- with Fresnel propagation between them; Sec. 1.2: about 19
// FFTs per wavelength). The field meets each optic's plane, is multiplied by the optic
// (transmission, OPD phasor of Eq. 3, thin lens), and travels to the next plane by the steps of
// the Gaussian pilot-beam planner (fr_plan_route): the angular spectrum between planes near the
// beam's waist, the direct step and its inverse to and from far planes. A thin lens changes the
// pilot beam by the q-law, 1/q' = 1/q - 1/f (q = z - z_waist - i z_R in the sign convention of
// the transfer function here, exp(-i pi lambda z f^2)), so every plane has the pitch of its own
// near or far representation; fr_plan_system reports those pitches (where masks are sampled)
// and the number of 2-D transforms (two per angular-spectrum step, one per direct step).
//
// The optic of a plane rides in the prologue of the plane's first step when that step is an
// angular-spectrum or direct step; before an inverse direct step, and at the last plane, an
// elementwise kernel applies it (the same float32 arithmetic as the sweeps' prologue).
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "../../include/fresnel.h"
#include "dft_small.hpp"
#include "fr_internal.h"
#include "fr_runtime.h"

namespace fr {
namespace {

// field[y][x] *= amp exp(2 pi i opd / lambda) lens[x] lens[y] (amp, opd, lens each optional)
__global__ void __launch_bounds__(256) optic_kernel(float2 *field, int n, const float *amp, const float *opd,
                                                    float inv_lambda, const float2 *lens) {
  const size_t tot = size_t(n) * n;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
    const int y = int(e / n), x = int(e % n);
    const float a = amp ? amp[e] : 1.0f;
    c32 ph{a, 0.0f};
    if (opd) {
      float sn, cs;
      sincos_turns(opd[e] * inv_lambda, &sn, &cs);
      ph = {a * cs, a * sn};
    }
    if (lens) {
      const float2 lx = lens[x], ly = lens[y];
      ph = cmul(ph, cmul(c32{lx.x, lx.y}, c32{ly.x, ly.y}));
    }
    const float2 v = field[e];
    const c32 r = cmul(c32{v.x, v.y}, ph);
    field[e] = make_float2(r.x, r.y);
  }
}

struct Pilot {
  double w0, z_w;  // waist radius and position of the Gaussian pilot beam
};

// the pilot beam after a thin lens of focal f at z_lens (q-law)
Pilot through_lens(const Pilot &p, double lam, double z_lens, double f) {
  const double z_r = M_PI * p.w0 * p.w0 / lam;
  const std::complex<double> q(z_lens - p.z_w, -z_r);
  const std::complex<double> q2 = 1.0 / (1.0 / q - 1.0 / f);
  // q2 = (z_lens - z_w') - i z_R'
  const double z_r2 = -q2.imag();
  return {std::sqrt(lam * z_r2 / M_PI), z_lens - q2.real()};
}

int check_system(int32_t n, double dx, double lam, double beam_radius, const fr_optic *optics, int32_t count) {
  if (n <= 0 || !optics || count <= 0 || !(dx > 0) || !(lam > 0) || !(beam_radius > 0)) return FR_EINVAL;
  if (!std::isfinite(dx) || !std::isfinite(lam) || !std::isfinite(beam_radius)) return FR_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!std::isfinite(optics[i].z_m) || !std::isfinite(optics[i].lens_focal_m)) return FR_EINVAL;
    if (i > 0 && !(optics[i].z_m >= 0)) return FR_EINVAL;
  }
  if (!fresnel_size_supported(n)) return FR_EUNSUPPORTED;
  return FR_OK;
}

// the plan: per plane its pitch, then the steps to the next plane
struct SystemPlan {
  std::vector<double> dx;                        // pitch at each plane (before its optic)
  std::vector<std::vector<fr_route_step>> steps; // steps from plane i to plane i + 1
  int transforms = 0;
};

int plan(int32_t n, double dx, double lam, double beam_radius, const fr_optic *optics, int32_t count, SystemPlan *P) {
  Pilot pb{beam_radius, 0.0};  // collimated input: the waist on the first plane
  double z = 0.0, pitch = dx;
  P->dx.assign(count, 0.0);
  P->steps.assign(count, {});
  for (int i = 0; i < count; ++i) {
    P->dx[i] = pitch;
    if (optics[i].lens_focal_m != 0.0) pb = through_lens(pb, lam, z, optics[i].lens_focal_m);
    if (!(pb.w0 > 0) || !std::isfinite(pb.w0) || !std::isfinite(pb.z_w)) return FR_EINVAL;
    if (i + 1 == count) break;
    const double z_next = z + optics[i + 1].z_m;
    fr_route_step st[2];
    const int k = fr_plan_route(pb.w0, pb.z_w, lam, n, pitch, z, z_next, st, 2);
    if (k < 0) return k;
    for (int j = 0; j < k; ++j) {
      P->steps[i].push_back(st[j]);
      P->transforms += st[j].kind == FR_ROUTE_AS ? 2 : 1;
      pitch = st[j].dx_out_m;
    }
    z = z_next;
  }
  return FR_OK;
}

}  // namespace
}  // namespace fr

extern "C" {

int fr_plan_system(int32_t n, double dx_m, double wavelength_m, double beam_radius_m, const fr_optic *optics,
                   int32_t count, double *plane_dx_m, int32_t *transforms) {
  int st = fr::check_system(n, dx_m, wavelength_m, beam_radius_m, optics, count);
  if (st != FR_OK) return st;
  fr::SystemPlan P;
  if ((st = fr::plan(n, dx_m, wavelength_m, beam_radius_m, optics, count, &P)) != FR_OK) return st;
  if (plane_dx_m)
    for (int i = 0; i < count; ++i) plane_dx_m[i] = P.dx[i];
  if (transforms) *transforms = P.transforms;
  return FR_OK;
}

int propagate_system(fr_ctx *ctx_, fr_c64 *field, int32_t n, double dx_m, double wavelength_m, double beam_radius_m,
                     const fr_optic *optics, int32_t count, double *dx_out_m, void *stream) {
  if (!field || !dx_out_m) return FR_EINVAL;
  int st = fr::check_system(n, dx_m, wavelength_m, beam_radius_m, optics, count);
  if (st != FR_OK) return st;
  fr::Ctx *ctx = reinterpret_cast<fr::Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  fr::SystemPlan P;
  if ((st = fr::plan(n, dx_m, wavelength_m, beam_radius_m, optics, count, &P)) != FR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  // the optic of plane i alone (before an inverse direct step, or at the last plane)
  auto apply_optic = [&](int i) -> int {
    const fr_optic &o = optics[i];
    if (!o.amp && !o.opd_m && o.lens_focal_m == 0.0) return FR_OK;
    if (int c = ctx->begin_call(); c != FR_OK) return c;
    const float2 *lens = nullptr;
    if (o.lens_focal_m != 0.0) {
      const int c = ctx->lens(n, P.dx[i], wavelength_m, o.lens_focal_m, s, &lens);
      if (c != FR_OK) return c;
    }
    const fr::LaunchHook hook = ctx->hook();
    hook(s, "relay_optic", n, 0);
    const size_t tot = size_t(n) * n;
    const int blocks = int(std::min<size_t>((tot + 255) / 256, 8192));
    hipLaunchKernelGGL(fr::optic_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<float2 *>(field), int(n),
                       o.amp, o.opd_m, float(1.0 / wavelength_m), lens);
    hipError_t err = hipGetLastError();
    hook(s, "relay_optic", n, 1);
    return err == hipSuccess ? FR_OK : fr::record_hip(err);
  };
  int warn = 0;
  for (int i = 0; i < count; ++i) {
    const fr_optic &o = optics[i];
    const auto &steps = P.steps[i];
    bool fused = false;
    if (steps.empty() || steps[0].kind == FR_ROUTE_DIRECT_INVERSE) {
      if ((st = apply_optic(i)) != FR_OK) return st;
      fused = true;
    }
    for (size_t j = 0; j < steps.size(); ++j) {
      const fr_route_step &r = steps[j];
      const bool carry = !fused && j == 0;  // the optic in this step's prologue
      const float *amp = carry ? o.amp : nullptr;
      const float *opd = carry ? o.opd_m : nullptr;
      const double f = carry ? o.lens_focal_m : 0.0;
      double dx_out = 0.0;
      if (r.kind == FR_ROUTE_AS) {
        st = fresnel_step(ctx_, field, n, r.dx_in_m, wavelength_m, r.z_m, amp, opd, f, 0, stream);
      } else if (r.kind == FR_ROUTE_DIRECT) {
        st = fresnel_direct(ctx_, field, n, r.dx_in_m, wavelength_m, r.z_m, amp, opd, f, 0, &dx_out, stream);
      } else {
        st = fresnel_direct(ctx_, field, n, r.dx_out_m, wavelength_m, r.z_m, nullptr, nullptr, 0.0, FR_INVERSE,
                            &dx_out, stream);
      }
      if (st < 0) return st;
      warn |= st;
    }
  }
  *dx_out_m = P.dx[count - 1];
  return warn;
}

}  // extern "C"
