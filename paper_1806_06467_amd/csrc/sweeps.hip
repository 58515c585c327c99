// Fresnel plane = two in-place sweeps over an n x n c64 field (Sec. 1.1: angular-spectrum
// propagation; Sec. 1.2: FFTs of large 2-D arrays dominate; Sec. 2.4: fftshift).
//
// The paraxial transfer function factors, H[ky][kx] = h[ky] h[kx], so
//   IDFT2( H . DFT2(U) ) = (column pass: FFT, * h, IFFT) o (row pass: FFT, * h, IFFT)
// and each pass reads and writes the plane once. No fftshift is ever materialised: the
// angular-spectrum step is shift-invariant and h is indexed by the signed frequency.
//
//   row_sweep : load a row (or synthesise it from the pupil optic), optic prologue (amplitude,
//               OPD and mirror phasors of Eq. 3, thin-lens chirp), FFT, * h (scaled 1/n),
//               inverse FFT, store.
//   col_sweep : load a tile of adjacent columns, FFT, * h, inverse FFT, epilogue (the mirror
//               after the step, or the conjugate optic for the adjoint), store.
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

// Raw buffer access to one plane: a 32-bit per-lane offset plus a wave-uniform offset held in a
// scalar register, so that the sixteen strided accesses of a thread cost one address VGPR;
// accesses beyond the plane's bytes read 0 and are not written (hardware bounds check).
// (The 64-bit results are moved whole with bit casts: extracting single elements of the
// builtin's vector type was observed to address the wrong half.)
struct PlaneBuf {
  __amdgpu_buffer_rsrc_t r;
  typedef unsigned int raw64 __attribute__((__vector_size__(8)));  // the builtin's value type
  __device__ __forceinline__ PlaneBuf(const void *p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, int(bytes), 0x00020000)) {}
  __device__ __forceinline__ c32 load(unsigned vo, unsigned so) const {
    const float2 q = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    return {q.x, q.y};
  }
  __device__ __forceinline__ void store(unsigned vo, unsigned so, c32 v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw64, make_float2(v.x, v.y)), r, vo, so, 0);
  }
};

// pre optic at (y, x): amp * exp(2 pi i (opd + 2 pre_surf) / lambda) * lens[x] lens[y]
__device__ __forceinline__ c32 pre_optic(const PlaneArgs &pa, int n, int y, int x) {
  float a = 1.0f, turns = 0.0f;
  if (pa.amp || pa.opd) {
    const int off = (n - pa.win) >> 1;
    const int wy = y - off, wx = x - off;
    const bool in = unsigned(wy) < unsigned(pa.win) && unsigned(wx) < unsigned(pa.win);
    const size_t o = size_t(wy) * pa.win + wx;
    if (pa.amp) a = in ? pa.amp[o] : 0.0f;
    if (pa.opd && in) turns = pa.opd[o] * pa.inv_lambda;
  }
  if (pa.pre_surf) turns += 2.0f * pa.pre_surf[size_t(y) * n + x] * pa.inv_lambda;
  c32 ph = {a, 0.0f};
  if (pa.opd || pa.pre_surf) {
    float s, c;
    sincos_turns(turns, &s, &c);
    ph = {a * c, a * s};
  }
  if (pa.lens) ph = cmul(ph, cmul(ld2(pa.lens + x), ld2(pa.lens + y)));
  return ph;
}

// post optic at (y, x): exp(2 pi i 2 post_surf / lambda)
__device__ __forceinline__ c32 post_optic(const PlaneArgs &pa, int n, int y, int x) {
  float s, c;
  sincos_turns(2.0f * pa.post_surf[size_t(y) * n + x] * pa.inv_lambda, &s, &c);
  return {c, s};
}

__device__ __forceinline__ bool has_pre(const PlaneArgs &pa) {
  return pa.amp || pa.opd || pa.pre_surf || pa.lens;
}

// frequency product of the pass: Y h (forward) or Y conj(h) (adjoint, AS over -z); slot m
// holds frequency t + T m. h carries the 1/n of the inverse transform.
template <int E, int T>
__device__ __forceinline__ void freq_product(c32 (&v)[E], const float2 *h, int t, bool adj) {
  if (adj) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], ld2(h + t + T * m));
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], ld2(h + t + T * m));
  }
}

template <class PL, int LINES>
__global__ void __launch_bounds__(PL::T *LINES) row_sweep(BatchArgs args, const float2 *tw) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  __shared__ c32 lds[LINES * LdsLine<N>::size];
  const PlaneArgs &pa = args.p[blockIdx.y];
  const int line = threadIdx.x / T;
  const int t = threadIdx.x - line * T;
  const int y = blockIdx.x * LINES + line;
  const bool adj = pa.flags & FR_ADJOINT;
  const PlaneBuf buf(pa.field, unsigned(N) * N * 8u);
  const unsigned vo = unsigned(y * N + t) * 8u;
  c32 v[E];
  if (pa.flags & kSourceOptic) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = pre_optic(pa, N, y, t + T * m);
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = buf.load(vo, unsigned(T * m) * 8u);
    if (!adj && has_pre(pa)) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cmul(v[m], pre_optic(pa, N, y, t + T * m));
    }
    if (adj && pa.post_surf) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], post_optic(pa, N, y, t + T * m));
    }
  }
  c32 *my = lds + line * LdsLine<N>::size;
  PL::forward(v, my, t, tw);
  freq_product<E, T>(v, pa.h, t, adj);
  PL::inverse(v, my, t, tw);
#pragma unroll
  for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * 8u, v[m]);
}

template <class PL, int LINES>
__global__ void __launch_bounds__(PL::T *LINES) col_sweep(BatchArgs args, const float2 *tw) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  constexpr int G = N / LINES;  // column groups per plane
  __shared__ c32 lds[LINES * (LdsLine<N>::size + 4)];
  const PlaneArgs &pa = args.p[blockIdx.y];
  const int c = threadIdx.x % LINES;
  const int t = threadIdx.x / LINES;
  // blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of groups
  int g = blockIdx.x;
  if constexpr (G % 8 == 0) g = (blockIdx.x & 7) * (G / 8) + (blockIdx.x >> 3);
  const int x = g * LINES + c;
  const bool adj = pa.flags & FR_ADJOINT;
  const PlaneBuf buf(pa.field, unsigned(N) * N * 8u);
  const unsigned vo = unsigned(t * N + x) * 8u;
  c32 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = buf.load(vo, unsigned(T * m) * unsigned(N) * 8u);
  c32 *my = lds + c * (LdsLine<N>::size + 4);
  PL::forward(v, my, t, tw);
  freq_product<E, T>(v, pa.h, t, adj);
  PL::inverse(v, my, t, tw);
  if (adj && has_pre(pa)) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], pre_optic(pa, N, t + T * m, x));
  }
  if (!adj && pa.post_surf) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], post_optic(pa, N, t + T * m, x));
  }
#pragma unroll
  for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * unsigned(N) * 8u, v[m]);
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

// the twiddle table of the plan the sweeps use for edge n (same Plan types as the launches)
int fresnel_twiddle_count(int n) {
  switch (n) {
    case 64: return Plan<64, 8, 8, 8>::twiddles;
    case 128: return Plan<128, 16, 16, 8>::twiddles;
    case 256: return Plan<256, 16, 16, 16>::twiddles;
    case 512: return Plan<512, 8, 8, 8, 8>::twiddles;
    case 1024: return Plan<1024, 16, 16, 8, 8>::twiddles;
    case 2048: return Plan<2048, 16, 16, 16, 8>::twiddles;
    case 4096: return Plan<4096, 16, 16, 16, 16>::twiddles;
    case 8192: return Plan<8192, 16, 16, 16, 16, 2>::twiddles;
    default: return 0;
  }
}
void fresnel_twiddle_build(int n, float2 *out) {
  switch (n) {
    case 64: Plan<64, 8, 8, 8>::build_twiddles(out); break;
    case 128: Plan<128, 16, 16, 8>::build_twiddles(out); break;
    case 256: Plan<256, 16, 16, 16>::build_twiddles(out); break;
    case 512: Plan<512, 8, 8, 8, 8>::build_twiddles(out); break;
    case 1024: Plan<1024, 16, 16, 8, 8>::build_twiddles(out); break;
    case 2048: Plan<2048, 16, 16, 16, 8>::build_twiddles(out); break;
    case 4096: Plan<4096, 16, 16, 16, 16>::build_twiddles(out); break;
    case 8192: Plan<8192, 16, 16, 16, 16, 2>::build_twiddles(out); break;
    default: break;
  }
}

int fresnel_variants(int n) { return n == 4096 || n == 2048 || n == 8192 ? 3 : 1; }

hipError_t launch_fresnel_batch(const PlaneArgs *planes, int count, int n, const float2 *root,
                                hipStream_t s, const LaunchHook &hook, int variant) {
  BatchArgs args;
  for (int i = 0; i < count; ++i) args.p[i] = planes[i];
  switch (n) {
    case 64: return launch_sweeps<Plan<64, 8, 8, 8>, 8, 16>(args, count, root, s, hook);
    case 128: return launch_sweeps<Plan<128, 16, 16, 8>, 16, 32>(args, count, root, s, hook);
    case 256: return launch_sweeps<Plan<256, 16, 16, 16>, 16, 32>(args, count, root, s, hook);
    case 512: return launch_sweeps<Plan<512, 8, 8, 8, 8>, 4, 16>(args, count, root, s, hook);
    case 1024: return launch_sweeps<Plan<1024, 16, 16, 8, 8>, 4, 8>(args, count, root, s, hook);
    case 2048:
      using P2 = Plan<2048, 16, 16, 16, 8>;
      if (variant == 1) return launch_sweeps<P2, 2, 4>(args, count, root, s, hook);
      if (variant == 2) return launch_sweeps<P2, 4, 4>(args, count, root, s, hook);
      return launch_sweeps<P2, 2, 8>(args, count, root, s, hook);
    case 4096:
      using P4 = Plan<4096, 16, 16, 16, 16>;
      if (variant == 1) return launch_sweeps<P4, 1, 2>(args, count, root, s, hook);
      if (variant == 2) return launch_sweeps<P4, 2, 2>(args, count, root, s, hook);
      return launch_sweeps<P4, 1, 4>(args, count, root, s, hook);
    case 8192:
      using P8 = Plan<8192, 16, 16, 16, 16, 2>;
      if (variant == 1) return launch_sweeps<P8, 1, 1>(args, count, root, s, hook);
      if (variant == 2) return launch_sweeps<P8, 2, 1>(args, count, root, s, hook);
      return launch_sweeps<P8, 1, 2>(args, count, root, s, hook);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fr
