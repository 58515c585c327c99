/* Host-side C-ABI paths of libfresnel under AddressSanitizer (no GPU needed): every entry point
 * with arguments its checks reject, the status strings, the workspace queries and the pilot-beam
 * planner. Exits nonzero on an unexpected status; ASan aborts on a memory error. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../include/fresnel.h"

static int fails = 0;
#define EXPECT(cond)                                               \
  do {                                                             \
    if (!(cond)) {                                                 \
      fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

int main(void) {
  fr_c64 *fake = (fr_c64 *)0x1000; /* never dereferenced: every call fails validation first */
  double dx_out = -7.0;
  for (int s = -6; s <= 5; ++s) EXPECT(fr_status_string(s) != NULL && strlen(fr_status_string(s)) > 0);
  EXPECT(fr_fft_size_supported(4096) == 1 && fr_fft_size_supported(4099) == 0);
  EXPECT(fresnel_step(NULL, NULL, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EINVAL);
  EXPECT(fresnel_step(NULL, fake, 4099, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EUNSUPPORTED);
  EXPECT(fresnel_step(NULL, fake, 256, 1e-4, 5e-7, NAN, NULL, NULL, 0.0, 0, NULL) == FR_EINVAL);
  EXPECT(fresnel_step(NULL, fake, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 8, NULL) == FR_EINVAL);
  EXPECT(fresnel_step_batched(NULL, NULL, 0, NULL) == FR_EINVAL);
  EXPECT(fresnel_step_exact(NULL, NULL, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EINVAL);
  EXPECT(fresnel_step_exact(NULL, fake, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 2, NULL) == FR_EINVAL);
  EXPECT(fresnel_step_exact(NULL, fake, 4099, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EUNSUPPORTED);
  EXPECT(fresnel_step_exact(NULL, fake, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EINVAL);
  {
    fr_plane ex[2];
    memset(ex, 0, sizeof ex);
    for (int i = 0; i < 2; ++i) {
      ex[i].field = fake;
      ex[i].dx_m = 1e-4;
      ex[i].wavelength_m = 5e-7;
      ex[i].z_m = 1.0;
      ex[i].n = 256;
    }
    EXPECT(fresnel_step_exact_batched(NULL, ex, 2, NULL) == FR_EINVAL); /* no context */
    EXPECT(fresnel_step_exact_batched(NULL, ex, 0, NULL) == FR_EINVAL);
    ex[1].n = 512;
    EXPECT(fresnel_step_exact_batched(NULL, ex, 2, NULL) == FR_EINVAL); /* mixed edges */
    ex[0].n = ex[1].n = 3584;
    EXPECT(fresnel_step_exact_batched(NULL, ex, 2, NULL) == FR_EUNSUPPORTED);
  }
  fr_c128 *fake64 = (fr_c128 *)0x1000;
  EXPECT(mft_f64(NULL, NULL, fake64, 64, 16, 32.0, 0.5, 0, fake64, 1u << 30, NULL) == FR_EINVAL);
  EXPECT(mft_f64(NULL, fake64, fake64, 64, 16, 32.0, NAN, 0, fake64, 1u << 30, NULL) == FR_EINVAL);
  EXPECT(mft_f64(NULL, fake64, fake64, 64, 16, 32.0, 0.5, 4, fake64, 1u << 30, NULL) == FR_EINVAL);
  EXPECT(mft_f64(NULL, fake64, fake64, 64, 16, 32.0, 0.5, FR_ADJOINT, fake64, 1u << 30, NULL) == FR_EINVAL);
  EXPECT(mft_f64(NULL, fake64, fake64, 64, 16, 32.0, 0.5, 0, fake64, 100, NULL) == FR_EWORKSPACE);
  EXPECT(mft_f64_workspace_bytes(4096, 256) == 4u * 16u * 4096u * 256u + 32u * 16u * 256u * 256u);
  EXPECT(fresnel_direct(NULL, fake, 256, 1e-4, 5e-7, 0.0, NULL, NULL, 0.0, 0, &dx_out, NULL) == FR_EINVAL);
  EXPECT(fresnel_direct(NULL, fake, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 3, &dx_out, NULL) == FR_EINVAL);
  EXPECT(fresnel_direct(NULL, fake, 3584, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, &dx_out, NULL) == FR_EUNSUPPORTED);
  EXPECT(fresnel_direct(NULL, fake, 256, 1e-4, 5e-7, 1.0, NULL, NULL, 0.0, 0, &dx_out, NULL) == FR_EINVAL);
  EXPECT(dx_out == -7.0);
  EXPECT(mft_workspace_bytes(4096, 256) > 0);
  EXPECT(mft_forward(NULL, NULL, 256, 256, NULL, 64, 64, 128.0, 0.5, NULL, NULL, 0, NULL) == FR_EINVAL);
  EXPECT(mft_forward_noalloc(NULL, NULL, 256, 256, NULL, 64, 64, 128.0, 0.5, NULL, NULL) == FR_EINVAL);
  EXPECT(fresnel_step_f64(NULL, NULL, 256, 1e-5, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EINVAL);
  {
    fr_optic ops[3] = {{0.0, 2.0, NULL, NULL}, {3.0, 1.0, NULL, NULL}, {1.0, 0.0, NULL, NULL}};
    double pitches[3];
    int32_t tr = 0;
    EXPECT(fr_plan_system(256, 1e-4, 5e-7, 2e-3, ops, 3, pitches, &tr) == FR_OK && tr > 0);
    EXPECT(fr_plan_system(256, 1e-4, 5e-7, 2e-3, ops, 0, pitches, &tr) == FR_EINVAL);
    double dx_out = 0.0;
    EXPECT(propagate_system(NULL, (fr_c64 *)16, 256, 1e-4, 5e-7, 2e-3, ops, 3, &dx_out, NULL) == FR_EINVAL);
  }
  EXPECT(fresnel_step_f64(NULL, (fr_c128 *)16, 96, 1e-5, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EUNSUPPORTED);
  EXPECT(fresnel_step_f64(NULL, (fr_c128 *)16, 256, 1e-5, 5e-7, 1.0, NULL, NULL, 0.0, 0, NULL) == FR_EINVAL);
  EXPECT(mft_forward_noalloc(NULL, (const fr_c64 *)16, 256, 255, (fr_c64 *)16, 64, 64, 128.0, 0.5, NULL, NULL) ==
         FR_EINVAL);
  EXPECT(mft_forward_noalloc(NULL, (const fr_c64 *)16, 8192, 8192, (fr_c64 *)16, 1025, 1025, 128.0, 0.5, NULL, NULL) ==
         FR_EWORKSPACE);
  EXPECT(mft_forward_noalloc(NULL, (const fr_c64 *)16, 256, 256, (fr_c64 *)16, 64, 64, 128.0, 0.5, NULL, NULL) ==
         FR_EINVAL);
  EXPECT(mft_adjoint(NULL, NULL, 64, 64, NULL, 256, 256, 128.0, 0.5, 1.0f, 0.0f, NULL, NULL, 0, NULL) == FR_EINVAL);
  EXPECT(fr_autotune(NULL, 1, 4096, 0, NULL) == FR_EINVAL);
  EXPECT(fr_profile_enable(NULL, 1) == FR_EINVAL);
  EXPECT(fr_set_cache_limit(NULL, 8) == FR_EINVAL);
  EXPECT(fr_set_cache_limit((fr_ctx *)0x1000, 0) == FR_EINVAL);
  fr_route_step steps[2];
  memset(steps, 0, sizeof steps);
  const double lam = 6e-7, w0 = 2e-3, zr = M_PI * w0 * w0 / lam;
  EXPECT(fr_plan_route(w0, 0.0, lam, 1024, 2e-5, 0.0, 3.0 * zr, steps, 2) == 1);
  EXPECT(steps[0].kind == FR_ROUTE_DIRECT && steps[0].z_m == 3.0 * zr);
  EXPECT(fr_plan_route(w0, 0.0, lam, 1024, 1e-4, -4.0 * zr, 5.0 * zr, steps, 2) == 2);
  EXPECT(steps[0].kind == FR_ROUTE_DIRECT_INVERSE && steps[1].kind == FR_ROUTE_DIRECT);
  EXPECT(fr_plan_route(w0, 0.0, lam, 1024, 2e-5, 0.0, 1.0, steps, 1) == FR_EINVAL);
  EXPECT(fr_plan_route(w0, 0.0, lam, 1024, 2e-5, 0.0, 1.0, NULL, 2) == FR_EINVAL);
  if (fails) fprintf(stderr, "%d unexpected results\n", fails);
  else printf("host ABI checks under AddressSanitizer: ok\n");
  return fails ? 1 : 0;
}
