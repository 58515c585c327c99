// Lyot coronagraph train over wavelengths, forward and adjoint (Sec. 1.1: Fresnel steps between
// optics and the semi-analytic coronagraph of Soummer et al.; Sec. 1.2: the sequence repeats for
// every wavelength).
//
// Per wavelength, with every plane resident in HBM:
//   forward:  row+column sweeps (pupil optic synthesised in the row prologue, DM phasor in the
//             column epilogue)                                               -> E_dm   (n^2)
//             occulter MFT (mask in the epilogue)                            -> E_occ  (occ^2)
//             Babinet MFT^H into the Lyot window (alpha -1, beta 1 on E_dm,
//             Lyot mask in the epilogue)                                     -> E_L    (n_d^2)
//             detector MFT, w |E|^2 accumulated into the PSF in the epilogue -> E_det  (det^2)
//   backward: the adjoint of each linear piece in reverse order, then the phase-to-height chain
//             g_s = -2 (4 pi / lambda) Im(E_dm conj(B)) and dL/dA = G^T g_s G.
// Wavelengths run in a fixed order, so the PSF and gradient sums are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fresnel.h"
#include "dft_small.hpp"
#include "fr_internal.h"
#include "fr_runtime.h"

namespace fr {

namespace {

// ---- small kernels --------------------------------------------------------------------------

// C (M x N, ldc) = alpha op(A) op(B) + beta C, real float, 16 x 16 tiles through LDS.
struct RGemm {
  int M, N, K;
  const float *A;
  int lda, transA;
  const float *B;
  int ldb, transB;
  float *C;
  int ldc;
  float alpha, beta;
};

__global__ void __launch_bounds__(256) rgemm_kernel(RGemm g) {
  __shared__ float As[16][17];
  __shared__ float Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  float acc = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    {  // A tile rows blockIdx.y*16.., cols k0..
      const int r = blockIdx.y * 16 + ty, c = k0 + tx;
      float v = 0.f;
      if (r < g.M && c < g.K) v = g.transA ? g.A[size_t(c) * g.lda + r] : g.A[size_t(r) * g.lda + c];
      As[ty][tx] = v;
    }
    {  // B tile rows k0.., cols blockIdx.x*16..
      const int r = k0 + ty, c = blockIdx.x * 16 + tx;
      float v = 0.f;
      if (r < g.K && c < g.N) v = g.transB ? g.B[size_t(c) * g.ldb + r] : g.B[size_t(r) * g.ldb + c];
      Bs[ty][tx] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = fmaf(As[ty][k], Bs[k][tx], acc);
    __syncthreads();
  }
  if (i < g.M && j < g.N) {
    float *cp = g.C + size_t(i) * g.ldc + j;
    *cp = g.alpha * acc + (g.beta != 0.f ? g.beta * *cp : 0.f);
  }
}

hipError_t rgemm(const RGemm &g, hipStream_t s, const LaunchHook &hook) {
  hook(s, "rgemm", g.K, 0);
  hipLaunchKernelGGL(rgemm_kernel, dim3((g.N + 15) / 16, (g.M + 15) / 16), dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  hook(s, "rgemm", g.K, 1);
  return e;
}

__global__ void fill_f32(float *p, size_t n, float v) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void fill_c64(float2 *p, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = make_float2(0.f, 0.f);
}

// out (nd x nd) = mask * window_{nd}(plane n x n)
__global__ void window_mask(const float2 *plane, int n, int nd, const float *mask, float2 *out) {
  const int off = (n - nd) / 2;
  const size_t tot = size_t(nd) * nd;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
    const int y = int(e / nd), x = int(e % nd);
    float2 v = plane[size_t(y + off) * n + x + off];
    const float m = mask ? mask[e] : 1.f;
    out[e] = make_float2(v.x * m, v.y * m);
  }
}

// plane window (nd x nd, centred) += src
__global__ void window_add(float2 *plane, int n, int nd, const float2 *src) {
  const int off = (n - nd) / 2;
  const size_t tot = size_t(nd) * nd;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
    const int y = int(e / nd), x = int(e % nd);
    float2 *p = plane + size_t(y + off) * n + x + off;
    const float2 a = *p, b = src[e];
    *p = make_float2(a.x + b.x, a.y + b.y);
  }
}

// y = w * g * e  (dL/dE_det up to the factor 2 carried by the phase chain)
__global__ void scale_by_grad(const float *g, float w, const float2 *e, float2 *y, size_t tot) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < tot; i += size_t(gridDim.x) * blockDim.x) {
    const float s = w * g[i];
    y[i] = make_float2(s * e[i].x, s * e[i].y);
  }
}

// g_s = -2 kappa Im(E conj(B)); E is the stored plane, or (pre != null) the pupil optic
// amp exp(2 pi i (opd + 2 pre) / lambda) synthesised here (amp/opd nd x nd centred).
__global__ void phase_grad(const float2 *e, const float2 *b, float *gs, int n, float kappa,
                           const float *amp, const float *opd, int nd, const float *pre,
                           float inv_lambda) {
  const size_t tot = size_t(n) * n;
  const int off = (n - nd) / 2;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < tot; i += size_t(gridDim.x) * blockDim.x) {
    float2 ev;
    if (e) {
      ev = e[i];
    } else {
      const int y = int(i / n), x = int(i % n);
      const int wy = y - off, wx = x - off;
      const bool in = unsigned(wy) < unsigned(nd) && unsigned(wx) < unsigned(nd);
      const size_t o = size_t(wy) * nd + wx;
      const float a = in ? amp[o] : 0.f;
      float turns = (in && opd) ? opd[o] * inv_lambda : 0.f;
      turns += 2.f * pre[i] * inv_lambda;
      float s, c;
      sincos_turns(turns, &s, &c);
      ev = make_float2(a * c, a * s);
    }
    const float2 bv = b[i];
    // Im(E conj(B)) = e.y b.x - e.x b.y
    gs[i] = -2.f * kappa * (ev.y * bv.x - ev.x * bv.y);
  }
}

template <typename K, typename... Args>
hipError_t launch1d(K kern, size_t work, hipStream_t s, const LaunchHook &hook, const char *name,
                    Args... args) {
  const int blocks = int(std::min<size_t>((work + 255) / 256, 8192));
  hook(s, name, 0, 0);
  hipLaunchKernelGGL(kern, dim3(std::max(blocks, 1)), dim3(256), 0, s, args...);
  hipError_t e = hipGetLastError();
  hook(s, name, 0, 1);
  return e;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
  size_t e, b, gs, surf, tdm, el, y1, eocc, edet, ydet, mft, total;
};

Layout layout(const fr_train_desc *d, int nmax, bool grad) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t n2 = size_t(nmax) * nmax;
  const size_t nd2 = size_t(d->n_d) * d->n_d;
  L.e = take(n2 * 8);
  L.b = grad ? take(n2 * 8) : 0;
  L.gs = grad ? take(n2 * 4) : 0;
  L.surf = take(size_t(std::max(d->n_dm, 1)) * n2 * 4);
  L.tdm = take(size_t(std::max(d->n_act, 1)) * nmax * 4);
  L.el = take(nd2 * 8);
  L.y1 = grad ? take(nd2 * 8) : 0;
  L.eocc = take(size_t(d->occ_m) * d->occ_m * 8);
  L.edet = take(size_t(d->det_m) * d->det_m * 8);
  L.ydet = grad ? take(size_t(d->det_m) * d->det_m * 8) : 0;
  const size_t m1 = mft_ws_bytes(nmax, d->occ_m);
  const size_t m2 = mft_ws_bytes(d->n_d, d->det_m);
  const size_t m3 = mft_ws_bytes(d->n_d, d->occ_m);
  L.mft = take(std::max(m1, std::max(m2, m3)));
  L.total = off;
  return L;
}

int check_desc(const fr_train_desc *d, int32_t n_lambda, const double *lam, const int32_t *n_pad,
               const float *w, int32_t mode) {
  if (!d || n_lambda <= 0 || !lam || !n_pad || !w) return FR_EINVAL;
  if (mode & ~(FR_TRAIN_NO_OCCULTER | FR_TRAIN_GRAD)) return FR_EINVAL;
  if (d->n_d <= 0 || !(d->d_m > 0) || !d->pupil_amp) return FR_EINVAL;
  if (d->n_dm < 0 || d->n_dm > 2) return FR_EINVAL;
  if (d->n_dm > 0 && (d->n_act <= 0 || !d->dm_heights_m)) return FR_EINVAL;
  if (!std::isfinite(d->z_m)) return FR_EINVAL;
  if (d->occ_m <= 0 || !(d->occ_du_c > 0) || d->det_m <= 0 || !(d->det_du_c > 0)) return FR_EINVAL;
  if (!(mode & FR_TRAIN_NO_OCCULTER) && !d->occ_mask) return FR_EINVAL;
  if (!d->lyot || !(d->lambda_c_m > 0)) return FR_EINVAL;
  if ((mode & FR_TRAIN_GRAD) && d->n_dm == 0) return FR_EINVAL;
  for (int j = 0; j < n_lambda; ++j) {
    if (!(lam[j] > 0) || !std::isfinite(w[j])) return FR_EINVAL;
    if (n_pad[j] < d->n_d || ((n_pad[j] - d->n_d) & 1)) return FR_EINVAL;
    if (!fresnel_size_supported(n_pad[j])) return FR_EUNSUPPORTED;
  }
  return FR_OK;
}

}  // namespace

size_t train_workspace_bytes(const fr_train_desc *d, int32_t n_lambda, const int32_t *n_pad, int32_t mode) {
  if (!d || n_lambda <= 0 || !n_pad) return 0;
  int nmax = 0;
  for (int j = 0; j < n_lambda; ++j) nmax = std::max(nmax, int(n_pad[j]));
  if (nmax <= 0 || d->n_d <= 0 || d->occ_m <= 0 || d->det_m <= 0) return 0;
  return layout(d, nmax, (mode & FR_TRAIN_GRAD) != 0).total;
}

int train_run(Ctx *ctx, const fr_train_desc *d, int32_t n_lambda, const double *lam,
              const int32_t *n_pad, const float *weight, int32_t mode, float *psf,
              const float *grad_psf, float *grad_heights, void *ws, size_t ws_bytes, hipStream_t s) {
  int st = check_desc(d, n_lambda, lam, n_pad, weight, mode);
  if (st != FR_OK) return st;
  const bool grad = (mode & FR_TRAIN_GRAD) != 0;
  const bool occ = !(mode & FR_TRAIN_NO_OCCULTER);
  if (!psf || (grad && (!grad_psf || !grad_heights))) return FR_EINVAL;
  if (!ws || ws_bytes < train_workspace_bytes(d, n_lambda, n_pad, mode)) return FR_EWORKSPACE;
  if (!ctx) return FR_EINVAL;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return record_hip(e);

  int nmax = 0;
  for (int j = 0; j < n_lambda; ++j) nmax = std::max(nmax, int(n_pad[j]));
  const Layout L = layout(d, nmax, grad);
  char *base = static_cast<char *>(ws);
  float2 *E = reinterpret_cast<float2 *>(base + L.e);
  float2 *B = grad ? reinterpret_cast<float2 *>(base + L.b) : nullptr;
  float *GS = grad ? reinterpret_cast<float *>(base + L.gs) : nullptr;
  float *SURF = reinterpret_cast<float *>(base + L.surf);
  float *TDM = reinterpret_cast<float *>(base + L.tdm);
  float2 *EL = reinterpret_cast<float2 *>(base + L.el);
  float2 *Y1 = grad ? reinterpret_cast<float2 *>(base + L.y1) : nullptr;
  float2 *EOCC = reinterpret_cast<float2 *>(base + L.eocc);
  float2 *EDET = reinterpret_cast<float2 *>(base + L.edet);
  float2 *YDET = grad ? reinterpret_cast<float2 *>(base + L.ydet) : nullptr;
  void *MWS = base + L.mft;
  const LaunchHook hook = ctx->hook();
  const int nd = d->n_d, na = d->n_act, ndm = d->n_dm;
  const size_t det2 = size_t(d->det_m) * d->det_m;
  const double dx = d->d_m / double(nd);

#define FR_TRY_HIP(x)                      \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) return record_hip(_e); \
  } while (0)
#define FR_TRY(x)           \
  do {                      \
    int _s = (x);           \
    if (_s != FR_OK) return _s; \
  } while (0)

  FR_TRY_HIP(launch1d(fill_f32, det2, s, hook, "fill", psf, det2, 0.f));
  if (grad) {
    const size_t ng = size_t(ndm) * na * na;
    FR_TRY_HIP(launch1d(fill_f32, ng, s, hook, "fill", grad_heights, ng, 0.f));
  }

  int surf_n = -1;
  for (int j = 0; j < n_lambda; ++j) {
    const int n = n_pad[j];
    const double lamj = lam[j];
    const size_t n2 = size_t(n) * n;
    const double du_occ = d->occ_du_c * d->lambda_c_m / lamj;
    const double du_det = d->det_du_c * d->lambda_c_m / lamj;
    const float inv_l = float(1.0 / lamj);

    // DM surfaces s = G A G^T on this grid (a8), rebuilt when the grid edge changes
    const float *G = nullptr;
    if (ndm > 0) {
      FR_TRY(ctx->dm_influence(n, nd, na, s, &G));
      if (surf_n != n) {
        for (int k = 0; k < ndm; ++k) {
          // TDM (na x n) = A G^T ; SURF_k (n x n) = G TDM
          RGemm g1{na, n, na, d->dm_heights_m + size_t(k) * na * na, na, 0, G, na, 1, TDM, n, 1.f, 0.f};
          FR_TRY_HIP(rgemm(g1, s, hook));
          RGemm g2{n, n, na, G, na, 0, TDM, n, 0, SURF + size_t(k) * n2, n, 1.f, 0.f};
          FR_TRY_HIP(rgemm(g2, s, hook));
        }
        surf_n = n;
      }
    }
    const float *surf_pre = ndm == 2 ? SURF : nullptr;
    const float *surf_post = ndm >= 1 ? SURF + size_t(ndm - 1) * n2 : nullptr;

    // ---- forward -------------------------------------------------------------------------
    PlaneArgs pa;
    std::memset(&pa, 0, sizeof pa);
    pa.field = E;
    pa.amp = d->pupil_amp;
    pa.opd = d->pupil_opd_m;
    pa.win = nd;
    pa.pre_surf = surf_pre;
    pa.post_surf = surf_post;
    pa.inv_lambda = inv_l;
    pa.flags = kSourceOptic;
    FR_TRY(ctx->transfer(n, dx, lamj, d->z_m, s, &pa.h));
    FR_TRY(run_planes(ctx, &pa, 1, n, s));                       // E = E_dm (a1, a2)

    const int off = (n - nd) / 2;
    const float2 *Ewin = E + size_t(off) * n + off;
    if (occ) {
      MftOut o;
      o.out = EOCC;
      o.ld_out = d->occ_m;
      o.mask = d->occ_mask;
      FR_TRY(mft_forward_impl(ctx, E, n, n, d->occ_m, double(nd), du_occ, o, MWS, s));   // a3
      FR_TRY(mft_adjoint_impl(ctx, EOCC, d->occ_m, d->occ_m, EL, nd, nd, double(nd), du_occ,
                              -1.f, 1.f, Ewin, n, d->lyot, MWS, s));                       // a4
    } else {
      FR_TRY_HIP(launch1d(window_mask, size_t(nd) * nd, s, hook, "window_mask", (const float2 *)E, n, nd,
                          d->lyot, EL));
    }
    {
      MftOut o;
      o.out = EDET;
      o.ld_out = d->det_m;
      o.intensity = psf;
      o.weight = weight[j];
      FR_TRY(mft_forward_impl(ctx, EL, nd, nd, d->det_m, double(nd), du_det, o, MWS, s));  // a3, a5
    }
    if (!grad) continue;

    // ---- backward (a7) ------------------------------------------------------------------
    FR_TRY_HIP(launch1d(scale_by_grad, det2, s, hook, "scale_by_grad", grad_psf, weight[j],
                        (const float2 *)EDET, YDET, det2));
    FR_TRY(mft_adjoint_impl(ctx, YDET, d->det_m, d->det_m, Y1, nd, nd, double(nd), du_det, 1.f, 0.f,
                            nullptr, 0, d->lyot, MWS, s));
    if (occ) {
      MftOut o;
      o.out = EOCC;
      o.ld_out = d->occ_m;
      o.mask = d->occ_mask;
      FR_TRY(mft_forward_impl(ctx, Y1, nd, nd, d->occ_m, double(nd), du_occ, o, MWS, s));
      FR_TRY(mft_adjoint_impl(ctx, EOCC, d->occ_m, d->occ_m, B, n, n, double(nd), du_occ, -1.f, 0.f,
                              nullptr, 0, nullptr, MWS, s));
    } else {
      FR_TRY_HIP(launch1d(fill_c64, n2, s, hook, "fill", B, n2));
    }
    FR_TRY_HIP(launch1d(window_add, size_t(nd) * nd, s, hook, "window_add", B, n, nd, (const float2 *)Y1));
    const float kappa = float(4.0 * M_PI / lamj);
    // last DM: g_s = -2 kappa Im(E_dm conj(B)); dL/dA += G^T (g_s G)
    FR_TRY_HIP(launch1d(phase_grad, n2, s, hook, "phase_grad", (const float2 *)E, (const float2 *)B, GS, n,
                        kappa, (const float *)nullptr, (const float *)nullptr, nd, (const float *)nullptr,
                        inv_l));
    float *gA = grad_heights + size_t(ndm - 1) * na * na;
    {
      RGemm g1{n, na, n, GS, n, 0, G, na, 0, TDM, na, 1.f, 0.f};   // TDM (n x na) = g_s G
      FR_TRY_HIP(rgemm(g1, s, hook));
      RGemm g2{na, na, n, G, na, 1, TDM, na, 0, gA, na, 1.f, 1.f};  // gA += G^T TDM
      FR_TRY_HIP(rgemm(g2, s, hook));
    }
    if (ndm == 2) {
      // B1 = AS_{-z}( conj(DM2 phasor) B ); g_s1 = -2 kappa Im(E_dm1 conj(B1))
      PlaneArgs pb;
      std::memset(&pb, 0, sizeof pb);
      pb.field = B;
      pb.post_surf = surf_post;
      pb.inv_lambda = inv_l;
      pb.win = n;
      pb.h = pa.h;
      pb.flags = FR_ADJOINT;
      FR_TRY(run_planes(ctx, &pb, 1, n, s));
      FR_TRY_HIP(launch1d(phase_grad, n2, s, hook, "phase_grad", (const float2 *)nullptr, (const float2 *)B,
                          GS, n, kappa, d->pupil_amp, d->pupil_opd_m, nd, (const float *)SURF, inv_l));
      RGemm g1{n, na, n, GS, n, 0, G, na, 0, TDM, na, 1.f, 0.f};
      FR_TRY_HIP(rgemm(g1, s, hook));
      RGemm g2{na, na, n, G, na, 1, TDM, na, 0, grad_heights, na, 1.f, 1.f};
      FR_TRY_HIP(rgemm(g2, s, hook));
    }
  }
#undef FR_TRY
#undef FR_TRY_HIP
  return FR_OK;
}

}  // namespace fr

extern "C" {

size_t propagate_train_workspace_bytes(const fr_train_desc *desc, int32_t n_lambda,
                                       const int32_t *n_pad, int32_t mode) {
  return fr::train_workspace_bytes(desc, n_lambda, n_pad, mode);
}

int propagate_train(fr_ctx *ctx, const fr_train_desc *desc, int32_t n_lambda, const double *lambda_m,
                    const int32_t *n_pad, const float *weight, int32_t mode, float *psf,
                    const float *grad_psf, float *grad_heights, void *ws, size_t ws_bytes,
                    void *stream) {
  return fr::train_run(reinterpret_cast<fr::Ctx *>(ctx), desc, n_lambda, lambda_m, n_pad, weight, mode,
                       psf, grad_psf, grad_heights, ws, ws_bytes, static_cast<hipStream_t>(stream));
}
}
