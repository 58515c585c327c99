// fresnel_step_f64: one Fresnel plane in float64, the paper's precision (Sec. 2.2: the
// benchmarks run in double precision). The same plane as fresnel_step (Sec. 1.1: the optic of
// Eq. 3 and a thin lens, then angular-spectrum propagation), the same two sweeps on the
// Stockham passes of fft_line.hpp (complex float64 elements, float64 twiddle tables):
//
//   row_sweep64 : load rows, optic prologue (forward) -- amplitude, exp(2 pi i opd / lambda) by a
//                 float64 sincospi, lens chirp --, FFT, * h (carrying 1/n), inverse FFT, conjugate
//                 optic epilogue (adjoint), store;
//   col_sweep64 : a tile of adjacent columns: FFT, * h, inverse FFT.
//
// Forward planes run rows then columns (the optic multiplies the input), adjoint planes columns
// then rows (the conjugate optic multiplies the output); the two sweeps commute. Tables: the
// transfer function h[k] = exp(-i pi lambda z k~^2 / (n dx)^2) / n, the lens chirp
// exp(-i pi c(i)^2 dx^2 / (lambda f)) and the twiddles, every phase formed from an exact integer
// times a float64 constant and reduced to a fraction of a turn before the float64 cos / sin.
// A complex float64 line of n elements takes 16 n bytes of LDS (plus the padding of
// fft_line.hpp), so the tiles hold half the lines of the float32 sweeps' (2048 and 4096: one row
// per row block, two columns per column tile, 32-byte row pieces; 8192: one of each). From 1024
// to 4096 the plans hold 8 elements per thread (radix-8 passes) where the float32 sweeps hold 16:
// twice the threads per line, under 128 VGPRs, so a compute unit runs 16 waves of the column
// sweep instead of 8 (measured at 4096: 200 us against 247 us per row sweep).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/fresnel.h"
#include "fft_line.hpp"
#include "fr_runtime.h"

namespace fr {
namespace {

constexpr int kMaxBatch64 = 8;

struct Plane64 {
  double2 *field;          // n x n, in place
  const double *amp;       // n x n or null
  const double *opd;       // n x n OPD [m] or null
  const double2 *h;        // n entries: the transfer function over the unsigned index, / n
  const double2 *lens;     // n entries or null
  double inv_lambda;       // 1 / lambda [1/m]
  int adjoint;
};
struct Batch64 {
  Plane64 p[kMaxBatch64];
};

__device__ __forceinline__ c64d ldz(const double2 *p) {
  const double2 v = *p;
  return {v.x, v.y};
}

// the optic at row y, slots x = t + T m: amp * exp(2 pi i opd / lambda) * lens[x] lens[y]
template <int E, int T>
__device__ __forceinline__ void optic_row(const Plane64 &pa, int n, int y, int t, c64d (&ph)[E]) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const size_t i = size_t(y) * n + t + T * m;
    const double a = pa.amp ? pa.amp[i] : 1.0;
    if (pa.opd) {
      double sn, cs;
      sincospi(2.0 * pa.opd[i] * pa.inv_lambda, &sn, &cs);
      ph[m] = {a * cs, a * sn};
    } else {
      ph[m] = {a, 0.0};
    }
  }
  if (pa.lens) {
    const c64d ly = ldz(pa.lens + y);
#pragma unroll
    for (int m = 0; m < E; ++m) ph[m] = cmul(ph[m], cmul(ldz(pa.lens + t + T * m), ly));
  }
}

template <class PL, int LINES>
__global__ void __launch_bounds__(PL::T *LINES) row_sweep64(Batch64 args, const double2 *tw) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  __shared__ c64d lds[LINES * LdsLine<N>::size];
  const Plane64 &pa = args.p[blockIdx.y];
  const int line = threadIdx.x / T;
  const int t = threadIdx.x - line * T;
  const int y = blockIdx.x * LINES + line;
  const bool optic = pa.amp || pa.opd || pa.lens;
  double2 *row = pa.field + size_t(y) * N;
  c64d v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = ldz(row + t + T * m);
  if (!pa.adjoint && optic) {
    c64d ph[E];
    optic_row<E, T>(pa, N, y, t, ph);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], ph[m]);
  }
  c64d *my = lds + line * LdsLine<N>::size;
  PL::forward(v, my, t, tw);
  // slot m holds frequency t + T m; the adjoint takes AS over -z: conj(h)
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = pa.adjoint ? cmulc(v[m], ldz(pa.h + t + T * m)) : cmul(v[m], ldz(pa.h + t + T * m));
  PL::inverse(v, my, t, tw);
  if (pa.adjoint && optic) {
    c64d ph[E];
    optic_row<E, T>(pa, N, y, t, ph);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], ph[m]);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) row[t + T * m] = make_double2(v[m].x, v[m].y);
}

template <class PL, int LINES>
__global__ void __launch_bounds__(PL::T *LINES) col_sweep64(Batch64 args, const double2 *tw) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  // the lines of the tile start 8 elements apart in the bank pattern
  constexpr int LINE = LdsLine<N>::size + 8;
  __shared__ c64d lds[LINES * LINE];
  const Plane64 &pa = args.p[blockIdx.y];
  const int c = threadIdx.x % LINES;
  const int t = threadIdx.x / LINES;
  // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous run of tiles, so that
  // the tiles sharing a 128-byte line of a row are read through one L2
  constexpr int G = N / LINES;
  int g = blockIdx.x;
  if constexpr (G % 8 == 0) g = (blockIdx.x & 7) * (G / 8) + (blockIdx.x >> 3);
  const int x = g * LINES + c;
  double2 *col = pa.field + x;
  c64d v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = ldz(col + size_t(t + T * m) * N);
  c64d *my = lds + c * LINE;
  PL::forward(v, my, t, tw);
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = pa.adjoint ? cmulc(v[m], ldz(pa.h + t + T * m)) : cmul(v[m], ldz(pa.h + t + T * m));
  PL::inverse(v, my, t, tw);
#pragma unroll
  for (int m = 0; m < E; ++m) col[size_t(t + T * m) * N] = make_double2(v[m].x, v[m].y);
}

template <class PL, int RL, int CL>
hipError_t launch64(const Batch64 &b, int count, bool adjoint, const double2 *tw, hipStream_t s,
                    const LaunchHook &hook) {
  constexpr int N = PL::N;
  static_assert(N % RL == 0 && N % CL == 0, "tile must divide n");
  auto rows = [&]() {
    hook(s, adjoint ? "row_sweep64_adj" : "row_sweep64", count, 0);
    hipLaunchKernelGGL((row_sweep64<PL, RL>), dim3(N / RL, count), dim3(PL::T * RL), 0, s, b, tw);
    hipError_t e = hipGetLastError();
    hook(s, adjoint ? "row_sweep64_adj" : "row_sweep64", count, 1);
    return e;
  };
  auto cols = [&]() {
    hook(s, adjoint ? "col_sweep64_adj" : "col_sweep64", count, 0);
    hipLaunchKernelGGL((col_sweep64<PL, CL>), dim3(N / CL, count), dim3(PL::T * CL), 0, s, b, tw);
    hipError_t e = hipGetLastError();
    hook(s, adjoint ? "col_sweep64_adj" : "col_sweep64", count, 1);
    return e;
  };
  hipError_t e = adjoint ? cols() : rows();
  if (e != hipSuccess) return e;
  return adjoint ? rows() : cols();
}

// the float32 sweeps' edges and tiles, halved for 16-byte elements (8 elements per thread from
// 1024 to 4096)
template <class F>
auto with_plan64(int n, F &&f) {
  switch (n) {
    case 64: return f(Plan<64, 8, 8, 8>{}, std::integral_constant<int, 8>{}, std::integral_constant<int, 16>{});
    case 128: return f(Plan<128, 16, 16, 8>{}, std::integral_constant<int, 8>{}, std::integral_constant<int, 16>{});
    case 256: return f(Plan<256, 16, 16, 16>{}, std::integral_constant<int, 8>{}, std::integral_constant<int, 16>{});
    case 512: return f(Plan<512, 8, 8, 8, 8>{}, std::integral_constant<int, 2>{}, std::integral_constant<int, 8>{});
    case 1024: return f(Plan<1024, 8, 8, 8, 8, 2>{}, std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{});
    case 2048: return f(Plan<2048, 8, 8, 8, 8, 4>{}, std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
    case 4096: return f(Plan<4096, 8, 8, 8, 8, 8>{}, std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
    default: return f(Plan<8192, 16, 16, 16, 16, 2>{}, std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{});
  }
}

bool size64_supported(int n) {
  switch (n) {
    case 64: case 128: case 256: case 512: case 1024: case 2048: case 4096: case 8192: return true;
    default: return false;
  }
}

uint64_t dbits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof u);
  return u;
}

double2 turn_to_z(double turns, double scale) {
  const double f = turns - std::nearbyint(turns);
  return make_double2(std::cos(2.0 * M_PI * f) * scale, std::sin(2.0 * M_PI * f) * scale);
}

// cached float64 tables (built on the host, uploaded once per geometry)
int table64(Ctx *ctx, const TableKey &key, const std::vector<double2> &h, hipStream_t s, const double2 **out) {
  void *d = nullptr;
  const int st = ctx->upload(key, h.data(), h.size() * sizeof(double2), s, &d);
  *out = static_cast<const double2 *>(d);
  return st;
}

int twiddles64(Ctx *ctx, int n, hipStream_t s, const double2 **out) {
  const TableKey key{kRoots64, n, 0, 0, 0, 0};
  if (auto it = ctx->tables.find(key); it != ctx->tables.end()) {
    *out = static_cast<const double2 *>(it->second);
    return FR_OK;
  }
  return with_plan64(n, [&](auto plan, auto, auto) {
    using PL = decltype(plan);
    std::vector<double2> h(std::max(PL::twiddles, 1));
    PL::build_twiddles(h.data());
    return table64(ctx, key, h, s, out);
  });
}

// h[k] = exp(-i pi lambda z k~^2 / (n dx)^2) / n over the signed index k~
int transfer64(Ctx *ctx, int n, double dx, double lam, double z, hipStream_t s, const double2 **out) {
  const TableKey key{kTransfer64, n, dbits(dx), dbits(lam), dbits(z), 0};
  if (auto it = ctx->tables.find(key); it != ctx->tables.end()) {
    *out = static_cast<const double2 *>(it->second);
    return FR_OK;
  }
  std::vector<double2> h(n);
  const double coef = -lam * z / (2.0 * (double(n) * dx) * (double(n) * dx));
  for (int k = 0; k < n; ++k) {
    const long long kt = (2 * k < n) ? k : k - n;
    h[k] = turn_to_z(double(kt * kt) * coef, 1.0 / double(n));
  }
  return table64(ctx, key, h, s, out);
}

// l[i] = exp(-i pi c(i)^2 dx^2 / (lambda f)), c(i) = i - n/2
int lens64(Ctx *ctx, int n, double dx, double lam, double f, hipStream_t s, const double2 **out) {
  const TableKey key{kLens64, n, dbits(dx), dbits(lam), dbits(f), 0};
  if (auto it = ctx->tables.find(key); it != ctx->tables.end()) {
    *out = static_cast<const double2 *>(it->second);
    return FR_OK;
  }
  std::vector<double2> h(n);
  const double coef = -dx * dx / (2.0 * lam * f);
  for (int i = 0; i < n; ++i) {
    const long long c = i - n / 2;
    h[i] = turn_to_z(double(c * c) * coef, 1.0);
  }
  return table64(ctx, key, h, s, out);
}

}  // namespace
}  // namespace fr

extern "C" int fresnel_step_f64(fr_ctx *ctx_, fr_c128 *field, int32_t n, double dx_m, double wavelength_m,
                                double z_m, const double *amp, const double *opd_m, double lens_focal_m,
                                int32_t flags, void *stream) {
  if (!field || n <= 0 || (flags & ~FR_ADJOINT)) return FR_EINVAL;
  if (!(dx_m > 0) || !(wavelength_m > 0) || !std::isfinite(dx_m) || !std::isfinite(wavelength_m) ||
      !std::isfinite(z_m) || !std::isfinite(lens_focal_m))
    return FR_EINVAL;
  if (!fr::size64_supported(n)) return FR_EUNSUPPORTED;
  fr::Ctx *ctx = reinterpret_cast<fr::Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  fr::Batch64 b;
  std::memset(&b, 0, sizeof b);
  fr::Plane64 &p = b.p[0];
  p.field = reinterpret_cast<double2 *>(field);
  p.amp = amp;
  p.opd = opd_m;
  p.inv_lambda = 1.0 / wavelength_m;
  p.adjoint = (flags & FR_ADJOINT) ? 1 : 0;
  int st = fr::transfer64(ctx, n, dx_m, wavelength_m, z_m, s, &p.h);
  if (st != FR_OK) return st;
  if (lens_focal_m != 0.0 && (st = fr::lens64(ctx, n, dx_m, wavelength_m, lens_focal_m, s, &p.lens)) != FR_OK)
    return st;
  const double2 *tw = nullptr;
  if ((st = fr::twiddles64(ctx, n, s, &tw)) != FR_OK) return st;
  const fr::LaunchHook hook = ctx->hook();
  e = fr::with_plan64(n, [&](auto plan, auto rl, auto cl) {
    return fr::launch64<decltype(plan), decltype(rl)::value, decltype(cl)::value>(b, 1, p.adjoint != 0, tw, s, hook);
  });
  if (e != hipSuccess) return fr::record_hip(e);
  return std::fabs(z_m) > double(n) * dx_m * dx_m / wavelength_m ? FR_W_AS_UNDERSAMPLED : FR_OK;
}
