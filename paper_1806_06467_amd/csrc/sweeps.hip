// Fresnel plane = two in-place sweeps over an n x n c64 field (Sec. 1.1: angular-spectrum
// propagation; Sec. 1.2: FFTs of large 2-D arrays dominate; Sec. 2.4: fftshift).
//
// The paraxial transfer function factors, H[ky][kx] = h[ky] h[kx], so
//   IDFT2( H . DFT2(U) ) = (column pass: FFT, * h, IFFT) o (row pass: FFT, * h, IFFT)
// and each pass reads and writes the plane once. No fftshift is ever materialised: the
// angular-spectrum step is shift-invariant and h is indexed by the signed frequency.
//
//   row_sweep : load a row, optic prologue (amplitude, OPD phasor of Eq. 3, thin-lens chirp),
//               FFT, * h (scaled 1/n), IFFT (as conj . FFT . conj), store.
//   col_sweep : load a tile of adjacent columns, FFT, * h, IFFT, conjugate-optic epilogue
//               for the adjoint, store.
// The column tile is LINES columns wide so that a wavefront reads LINES*8-byte contiguous
// segments; blocks are renumbered so that the blocks resident on one XCD (one L2) work on
// neighbouring columns at the same time.
#include "fft_line.hpp"
#include "fr_internal.h"
#include "../../include/fresnel.h"

namespace fr {

namespace {

__device__ __forceinline__ c32 ld2(const float2 *p) {
  float2 v = *p;
  return {v.x, v.y};
}
__device__ __forceinline__ void st2(float2 *p, c32 v) { *p = make_float2(v.x, v.y); }

// amp * exp(2 pi i opd / lambda) * lens[x] * lens[y]
__device__ __forceinline__ c32 optic_at(const PlaneArgs &pa, int n, int y, int x) {
  const size_t o = size_t(y) * n + x;
  const float a = pa.amp ? pa.amp[o] : 1.0f;
  c32 ph = {a, 0.0f};
  if (pa.opd) {
    float t = pa.opd[o] * pa.inv_lambda;
    t -= rintf(t);
    float s, c;
    sincospif(2.0f * t, &s, &c);
    ph = {a * c, a * s};
  }
  if (pa.lens) ph = cmul(ph, cmul(ld2(pa.lens + x), ld2(pa.lens + y)));
  return ph;
}

__device__ __forceinline__ bool has_optic(const PlaneArgs &pa) {
  return pa.amp || pa.opd || pa.lens;
}

// frequency product of the pass: Z = conj(Y h) (forward) or conj(Y conj(h)) (adjoint)
template <int E, int T>
__device__ __forceinline__ void freq_product(c32 (&v)[E], const float2 *h, int t, bool adj) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const c32 hk = ld2(h + t + T * m);
    v[m] = adj ? cconj(cmulc(v[m], hk)) : cconj(cmul(v[m], hk));
  }
}

template <class PL, int LINES>
__global__ void __launch_bounds__(PL::T *LINES) row_sweep(BatchArgs args, const float2 *root_) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  __shared__ c32 lds[LINES * LdsLine<N>::size];
  const PlaneArgs &pa = args.p[blockIdx.y];
  const c32 *root = reinterpret_cast<const c32 *>(root_);
  const int line = threadIdx.x / T;
  const int t = threadIdx.x - line * T;
  const int y = blockIdx.x * LINES + line;
  float2 *row = pa.field + size_t(y) * N;
  const bool adj = pa.flags & FR_ADJOINT;
  c32 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = ld2(row + t + T * m);
  if (!adj && has_optic(pa)) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], optic_at(pa, N, y, t + T * m));
  }
  c32 *my = lds + line * LdsLine<N>::size;
  PL::forward(v, my, t, root);
  freq_product<E, T>(v, pa.h, t, adj);
  PL::forward(v, my, t, root);
#pragma unroll
  for (int m = 0; m < E; ++m) st2(row + t + T * m, cconj(v[m]));
}

template <class PL, int LINES>
__global__ void __launch_bounds__(PL::T *LINES) col_sweep(BatchArgs args, const float2 *root_) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  constexpr int G = N / LINES;  // column groups per plane
  __shared__ c32 lds[LINES * (LdsLine<N>::size + 4)];
  const PlaneArgs &pa = args.p[blockIdx.y];
  const c32 *root = reinterpret_cast<const c32 *>(root_);
  const int c = threadIdx.x % LINES;
  const int t = threadIdx.x / LINES;
  // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of groups
  int g = blockIdx.x;
  if constexpr (G % 8 == 0) g = (blockIdx.x & 7) * (G / 8) + (blockIdx.x >> 3);
  const int x = g * LINES + c;
  const bool adj = pa.flags & FR_ADJOINT;
  float2 *col = pa.field + x;
  c32 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = ld2(col + size_t(t + T * m) * N);
  c32 *my = lds + c * (LdsLine<N>::size + 4);
  PL::forward(v, my, t, root);
  freq_product<E, T>(v, pa.h, t, adj);
  PL::forward(v, my, t, root);
  if (adj && has_optic(pa)) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(cconj(v[m]), cconj(optic_at(pa, N, t + T * m, x)));
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cconj(v[m]);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) st2(col + size_t(t + T * m) * N, v[m]);
}

template <class PL, int ROW_LINES, int COL_LINES>
hipError_t launch_sweeps(const BatchArgs &args, int count, const float2 *root, hipStream_t s,
                         const LaunchHook &hook) {
  constexpr int N = PL::N;
  static_assert(N % ROW_LINES == 0 && N % COL_LINES == 0, "tile must divide n");
  hook(s, "row_sweep", N, 0);
  hipLaunchKernelGGL((row_sweep<PL, ROW_LINES>), dim3(N / ROW_LINES, count),
                     dim3(PL::T * ROW_LINES), 0, s, args, root);
  hipError_t e = hipGetLastError();
  hook(s, "row_sweep", N, 1);
  if (e != hipSuccess) return e;
  hook(s, "col_sweep", N, 0);
  hipLaunchKernelGGL((col_sweep<PL, COL_LINES>), dim3(N / COL_LINES, count),
                     dim3(PL::T * COL_LINES), 0, s, args, root);
  e = hipGetLastError();
  hook(s, "col_sweep", N, 1);
  return e;
}

}  // namespace

bool fresnel_size_supported(int n) {
  switch (n) {
    case 64: case 128: case 256: case 512: case 1024: case 2048: case 4096: case 8192:
      return true;
    default:
      return false;
  }
}

hipError_t launch_fresnel_batch(const PlaneArgs *planes, int count, int n, const float2 *root,
                                hipStream_t s, const LaunchHook &hook) {
  BatchArgs args;
  for (int i = 0; i < count; ++i) args.p[i] = planes[i];
  switch (n) {
    case 64: return launch_sweeps<Plan<64, 8, 8, 8>, 8, 16>(args, count, root, s, hook);
    case 128: return launch_sweeps<Plan<128, 16, 16, 8>, 16, 32>(args, count, root, s, hook);
    case 256: return launch_sweeps<Plan<256, 16, 16, 16>, 16, 32>(args, count, root, s, hook);
    case 512: return launch_sweeps<Plan<512, 8, 8, 8, 8>, 4, 16>(args, count, root, s, hook);
    case 1024: return launch_sweeps<Plan<1024, 16, 16, 8, 8>, 4, 8>(args, count, root, s, hook);
    case 2048: return launch_sweeps<Plan<2048, 16, 16, 16, 8>, 2, 8>(args, count, root, s, hook);
    case 4096: return launch_sweeps<Plan<4096, 16, 16, 16, 16>, 1, 4>(args, count, root, s, hook);
    case 8192: return launch_sweeps<Plan<8192, 16, 16, 16, 16, 2>, 1, 2>(args, count, root, s, hook);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fr
