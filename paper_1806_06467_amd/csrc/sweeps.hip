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
#include "fr_exact.h"
#include "../../include/fresnel.h"

namespace fr {

namespace {

__device__ __forceinline__ c32 ld2(const float2 *p) {
  float2 v = *p;
  return {v.x, v.y};
}

// Raw buffer access to one plane: a 32-bit per-lane offset plus a wave-uniform offset held in a
// scalar register, so that the sixteen strided accesses of a thread cost one address VGPR.
// The hardware range check applies to the per-lane offset: lanes whose offset is past the
// buffer read 0 and do not write; every per-lane offset used here is non-negative.
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

// Same for float maps (amplitude, OPD, mirror surfaces).
struct MapBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ MapBuf(const void *p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, int(bytes), 0x00020000)) {}
  __device__ __forceinline__ float load(unsigned vo, unsigned so) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
};

// The pre optic along one row y for the thread's slots x = t + T m: amplitude, OPD (win x win
// maps centred in the plane), mirror surface (n x n) and thin lens. Returns false when the
// amplitude is zero on the whole row (a row outside the pupil window).
template <int E, int T>
__device__ __forceinline__ bool pre_optic_row(const PlaneArgs &pa, int n, int y, int t, c32 (&ph)[E]) {
  const int win = pa.win;
  const int off = (n - win) >> 1;
  const int wy = y - off;
  const bool row_in = unsigned(wy) < unsigned(win);
  if (pa.amp && !row_in) return false;
  float a[E], turns[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    a[m] = 1.0f;
    turns[m] = 0.0f;
  }
  if ((pa.amp || pa.opd) && row_in) {
    // The hardware range check of a raw buffer access looks at the per-lane (VGPR) offset
    // only, so every per-lane offset here is non-negative and inside the map: full maps use
    // lane offset + per-slot scalar offset; windowed maps clamp the column into the window
    // (lanes outside it are masked after the load).
    const unsigned bytes = unsigned(win) * unsigned(win) * 4u;
    unsigned vo[E], so[E];
    if (win == n) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        vo[m] = unsigned(wy * win + t) * 4u;
        so[m] = unsigned(T * m) * 4u;
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int wx = min(max(t + T * m - off, 0), win - 1);
        vo[m] = unsigned(wy * win + wx) * 4u;
        so[m] = 0u;
      }
    }
    if (pa.amp) {
      const MapBuf mb(pa.amp, bytes);
#pragma unroll
      for (int m = 0; m < E; ++m) a[m] = mb.load(vo[m], so[m]);
    }
    if (pa.opd) {
      const MapBuf mb(pa.opd, bytes);
#pragma unroll
      for (int m = 0; m < E; ++m) turns[m] = mb.load(vo[m], so[m]) * pa.inv_lambda;
    }
    if (win < n) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const bool in = unsigned(t + T * m - off) < unsigned(win);
        a[m] = in ? a[m] : (pa.amp ? 0.0f : 1.0f);
        turns[m] = in ? turns[m] : 0.0f;
      }
    }
  }
  if (pa.pre_surf) {
    const MapBuf sb(pa.pre_surf, unsigned(n) * unsigned(n) * 4u);
    const unsigned vo = unsigned(y * n + t) * 4u;
#pragma unroll
    for (int m = 0; m < E; ++m) turns[m] += 2.0f * sb.load(vo, unsigned(T * m) * 4u) * pa.inv_lambda;
  }
  if (pa.opd || pa.pre_surf) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      float sn, cs;
      sincos_turns(turns[m], &sn, &cs);
      ph[m] = {a[m] * cs, a[m] * sn};
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) ph[m] = {a[m], 0.0f};
  }
  if (pa.lens) {
    const c32 ly = ld2(pa.lens + y);
#pragma unroll
    for (int m = 0; m < E; ++m) ph[m] = cmul(ph[m], cmul(ld2(pa.lens + t + T * m), ly));
  }
  return true;
}

// post optic exp(2 pi i 2 post_surf / lambda) at rows y = t + T m of column x, for all slots:
// the map (4-column tiles) is read for every slot before any phasor is formed
template <int E, int T>
__device__ __forceinline__ void post_optic_col(const PlaneArgs &pa, int n, int t, int x, c32 (&ph)[E]) {
  const MapBuf map(pa.post_surf, unsigned(post_tiled_size(n)) * 4u);
  float sv[E];
#pragma unroll
  for (int m = 0; m < E; ++m) sv[m] = map.load(unsigned(post_tiled_index(n, t + T * m, x)) * 4u, 0u);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    float s, c;
    sincos_turns(2.0f * sv[m] * pa.inv_lambda, &s, &c);
    ph[m] = {c, s};
  }
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

// DIRECT: the row half of the direct (single-transform) Fresnel step: the prologue applies the
// optic times the input quadratic phase (held in the lens slot), then the forward transform only;
// for its adjoint the inverse transform, then the conjugate of both
// Up to 4096, at most 128 VGPRs (four waves per SIMD): at 4096 four 256-thread row blocks then
// share a compute unit (their LDS lines allow four) instead of three (measured 1 % faster per
// plane, bit-identical results); the 8192 row would spill under that cap.
template <class PL, int LINES, bool DIRECT = false>
__global__ void __launch_bounds__(PL::T *LINES) __attribute__((amdgpu_waves_per_eu(PL::N <= 4096 ? 4 : 1)))
row_sweep(BatchArgs args, const float2 *tw) {
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  __shared__ c32 lds[LINES * LdsLine<N>::size];
  const PlaneArgs &pa = args.p[blockIdx.y];
  const int line = threadIdx.x / T;
  const int t = threadIdx.x - line * T;
  const int y = blockIdx.x * LINES + line;
  const bool adj = pa.flags & FR_ADJOINT;
  if (adj && (pa.flags & kWindowRowsOnly)) {
    // rows of this block all outside the rows wanted from the step (block-uniform)
    const int y0 = blockIdx.x * LINES, off = (N - pa.win) >> 1;
    if (y0 + LINES <= off || y0 >= off + pa.win) return;
  }
  const PlaneBuf buf(pa.field, unsigned(N) * N * 8u);
  const unsigned vo = unsigned(y * N + t) * 8u;
  c32 v[E];
  if (!adj && has_pre(pa)) {
    c32 ph[E];
    const bool nonzero = pre_optic_row<E, T>(pa, N, y, t, ph);
    if constexpr (LINES == 1) {
      // a whole row outside the amplitude window stays zero through the row transform
      // (block-uniform); the column sweep takes it as zero without reading it, so it is not
      // stored
      if (!nonzero) return;
    }
    if (!nonzero) {
#pragma unroll
      for (int m = 0; m < E; ++m) ph[m] = {0.0f, 0.0f};
    }
    if (pa.flags & kSourceOptic) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = ph[m];
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cmul(buf.load(vo, unsigned(T * m) * 8u), ph[m]);
    }
  } else if (pa.flags & kSourceOptic) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = {1.0f, 0.0f};
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = buf.load(vo, unsigned(T * m) * 8u);
  }
  c32 *my = lds + line * LdsLine<N>::size;
  if constexpr (DIRECT) {
    // the adjoint direct step runs this sweep second: inverse transform, then the conjugate
    // optic and input phase below
    // the transform's kernel sign: + for the adjoint, flipped again over z < 0
    if (adj != bool(pa.flags & kTowardSource)) PL::inverse(v, my, t, tw);
    else PL::forward(v, my, t, tw);
  } else {
    PL::forward(v, my, t, tw);
    freq_product<E, T>(v, pa.h, t, adj);
    PL::inverse(v, my, t, tw);
  }
  if (adj && has_pre(pa)) {
    c32 ph[E];
    if (!pre_optic_row<E, T>(pa, N, y, t, ph)) {
#pragma unroll
      for (int m = 0; m < E; ++m) ph[m] = {0.0f, 0.0f};
    }
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], ph[m]);
  }
#pragma unroll
  for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * 8u, v[m]);
}

// HALF: the FFT exchanges go through half-size LDS lines in two rounds, so that two blocks fit
// on a compute unit. DIRECT: the column half of the direct Fresnel step: the forward transform,
// then the output quadratic phase of both axes (h holds it per index, with the constant's root).
// EXACT (with DIRECT): the column sweep of the exact-transfer-function step (fr_exact.h), 1 with
// H's phase formed per element in float64, 2 in its split form.
template <class PL, int LINES, bool HALF = false, bool DIRECT = false, int EXACT = 0>
__global__ void __launch_bounds__(PL::T *LINES) col_sweep(BatchArgs args, const float2 *tw) {
  static_assert(!EXACT || (DIRECT && !HALF), "the exact mode runs on full LDS lines");
  constexpr int N = PL::N, E = PL::E, T = PL::T;
  constexpr int G = N / LINES;  // column groups per plane
  // the lines of the LINES columns start 8 float2 apart in the bank pattern (measured: a
  // 3 % faster sweep than 4, 10 % than 1)
  constexpr int LINE = (HALF ? LdsLine<N / 2>::size : LdsLine<N>::size) + 8;
  __shared__ c32 lds[LINES * LINE];
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
  // the post surface's phasor, unless this tile lies where the surface is 0 (the phasor is 1)
  const int x0 = g * LINES;
  const bool post = pa.post_surf && !(pa.post_hi > pa.post_lo && (x0 + LINES <= pa.post_lo || x0 >= pa.post_hi));
  c32 v[E];
  if (!adj && pa.amp && pa.win < N) {
    // forward plane with a windowed amplitude: the rows outside the window are zero after the
    // row sweep, which did not store them (uniform over a wavefront when the window edges are
    // multiples of the wavefront's rows)
    const int off = (N - pa.win) >> 1;
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[m] = unsigned(t + T * m - off) < unsigned(pa.win) ? buf.load(vo, unsigned(T * m) * unsigned(N) * 8u)
                                                         : c32{0.0f, 0.0f};
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = buf.load(vo, unsigned(T * m) * unsigned(N) * 8u);
  }
  if (adj && post) {
    c32 ph[E];
    post_optic_col<E, T>(pa, N, t, x, ph);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], ph[m]);
  }
  c32 *my = lds + c * LINE;
  if constexpr (DIRECT) {
    if constexpr (EXACT) {
      // exact transfer function of frequency (kx, ky) = (x, t + T m) (signed), with the 1/n^2
      // of the two inverse transforms; conjugated for the adjoint. The spectrum goes through the
      // thread's own LDS slots so that the float64 phase of one element at a time is formed
      // beside no more than the loop's registers (the LDS is free between the transforms: the
      // forward one ends on a barrier after its last read).
      const double *prm = reinterpret_cast<const double *>(pa.h);
      const double zl = prm[0], a2 = prm[1];
      const int kx = x < N / 2 ? x : x - N;
      if constexpr (EXACT == 2) {
        // H = h[kx] h[ky] exp(2 pi i c): the paraxial part from its float64-built table (it
        // carries the 1/n of each inverse transform), the rest c = -(z/lambda) u^2 /
        // (2 (1 + sqrt(1 - u))^2) turns, at most a quarter turn on this grid, in float32
        const float2 *hp = reinterpret_cast<const float2 *>(prm + 4);
        const float zlf = float(zl), a2f = float(a2);
        const c32 hx = ld2(hp + x);
        PL::template forward<HALF>(v, my, t, tw);
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int k = t + T * m;
          const int ky = k < N / 2 ? k : k - N;
          const float u = a2f * float(kx * kx + ky * ky);
          const float r = 1.0f + sqrtf(1.0f - u);
          float sn, cs;
          sincos_turns(-zlf * u * u / (2.0f * r * r), &sn, &cs);
          const c32 hh = cmul(cmul(hx, ld2(hp + k)), c32{cs, sn});
          v[m] = adj ? cmulc(v[m], hh) : cmul(v[m], hh);
        }
        PL::template inverse<HALF>(v, my, t, tw);
#pragma unroll
        for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * unsigned(N) * 8u, v[m]);
        return;
      } else {
        PL::template forward<HALF>(v, my, t, tw);
#pragma unroll
        for (int m = 0; m < E; ++m) my[t + T * m] = v[m];
        constexpr float inv_n2 = 1.0f / (float(N) * float(N));
#pragma unroll 1
        for (int m = 0; m < E; ++m) {
          const int k = t + T * m;
          const int ky = k < N / 2 ? k : k - N;
          const double u = a2 * double(kx * kx + ky * ky);  // (lambda f)^2
          float amp = inv_n2, turns;
          if (u < 1.0) {
            const double tr = -zl * u / (sqrt(1.0 - u) + 1.0);
            turns = float(tr - rint(tr));
          } else {
            amp *= float(exp(-2.0 * kPi * fabs(zl) * sqrt(u - 1.0)));
            turns = float(-(zl - rint(zl)));
          }
          float sn, cs;
          sincos_turns(adj ? -turns : turns, &sn, &cs);
          my[k] = cmul(my[k], c32{amp * cs, amp * sn});
        }
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = my[t + T * m];
        __syncthreads();  // every slot read back before the inverse transform's first exchange
        PL::template inverse<HALF>(v, my, t, tw);
#pragma unroll
        for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * unsigned(N) * 8u, v[m]);
        return;
      }
    }
    // slot m holds frequency row ky = t + T m of column kx = x (after the forward transform;
    // the adjoint, which runs this sweep first, multiplies the conjugate phases before its
    // inverse transform)
    const c32 px = ld2(pa.h + x);
    const bool inv = adj != bool(pa.flags & kTowardSource);  // kernel sign, as in the row sweep
    if (adj) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], cmul(ld2(pa.h + t + T * m), px));
    }
    if (inv) PL::template inverse<HALF>(v, my, t, tw);
    else PL::template forward<HALF>(v, my, t, tw);
    if (!adj) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cmul(v[m], cmul(ld2(pa.h + t + T * m), px));
    }
#pragma unroll
    for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * unsigned(N) * 8u, v[m]);
    return;
  }
  PL::template forward<HALF>(v, my, t, tw);
  freq_product<E, T>(v, pa.h, t, adj);
  PL::template inverse<HALF>(v, my, t, tw);
  if (!adj && post) {
    c32 ph[E];
    post_optic_col<E, T>(pa, N, t, x, ph);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], ph[m]);
  }
  if (adj && (pa.flags & kWindowRowsOnly)) {
    // the row sweep that follows transforms only the rows of the window
    const int off = (N - pa.win) >> 1;
#pragma unroll
    for (int m = 0; m < E; ++m)
      if (unsigned(t + T * m - off) < unsigned(pa.win)) buf.store(vo, unsigned(T * m) * unsigned(N) * 8u, v[m]);
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) buf.store(vo, unsigned(T * m) * unsigned(N) * 8u, v[m]);
  }
}

// Forward planes run the row sweep first (optic prologue on contiguous rows) and the column
// sweep second (mirror epilogue); adjoint planes run the column sweep first (conjugate mirror
// prologue) and the row sweep second (conjugate optic epilogue). The two halves of the
// angular-spectrum step commute, so only the placement of the optics sets the order, and the
// amplitude/OPD maps are always read along rows.
template <class PL, int ROW_LINES, int COL_LINES, class PC = PL, bool CHALF = false, bool DIRECT = false>
hipError_t launch_sweeps(const BatchArgs &fwd, int nf, const BatchArgs &adj, int na,
                         const float2 *tw, hipStream_t s, const LaunchHook &hook) {
  constexpr int N = PL::N;
  static_assert(PC::N == N, "row and column plans of one edge");
  static_assert(N % ROW_LINES == 0 && N % COL_LINES == 0, "tile must divide n");
  // timing names carry the direction (the optic maps read differ), tags the planes per launch
  auto rows = [&](const BatchArgs &a, int count, const char *name) {
    hook(s, name, count, 0);
    hipLaunchKernelGGL((row_sweep<PL, ROW_LINES, DIRECT>), dim3(N / ROW_LINES, count),
                       dim3(PL::T * ROW_LINES), 0, s, a, tw);
    hipError_t e = hipGetLastError();
    hook(s, name, count, 1);
    return e;
  };
  auto cols = [&](const BatchArgs &a, int count, const char *name) {
    hook(s, name, count, 0);
    hipLaunchKernelGGL((col_sweep<PC, COL_LINES, CHALF, DIRECT>), dim3(N / COL_LINES, count),
                       dim3(PC::T * COL_LINES), 0, s, a, tw);
    hipError_t e = hipGetLastError();
    hook(s, name, count, 1);
    return e;
  };
  hipError_t e = hipSuccess;
  if (nf && (e = rows(fwd, nf, DIRECT ? "direct_rows" : "row_sweep")) != hipSuccess) return e;
  if (nf && (e = cols(fwd, nf, DIRECT ? "direct_cols" : "col_sweep")) != hipSuccess) return e;
  if (na && (e = cols(adj, na, DIRECT ? "direct_cols_adj" : "col_sweep_adj")) != hipSuccess) return e;
  if (na && (e = rows(adj, na, DIRECT ? "direct_rows_adj" : "row_sweep_adj")) != hipSuccess) return e;
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

int fresnel_variants(int n) { return n == 4096 ? 4 : n == 2048 || n == 8192 ? 3 : 1; }

hipError_t launch_fresnel_batch(const PlaneArgs *planes, int count, int n, const float2 *root,
                                hipStream_t s, const LaunchHook &hook, int variant) {
  BatchArgs fwd, adj;
  int nf = 0, na = 0;
  for (int i = 0; i < count; ++i) {
    if (planes[i].flags & FR_ADJOINT)
      adj.p[na++] = planes[i];
    else
      fwd.p[nf++] = planes[i];
  }
#define FR_SWEEPS(PL, RL, CL) return launch_sweeps<PL, RL, CL>(fwd, nf, adj, na, root, s, hook)
  switch (n) {
    case 64: {
      using P = Plan<64, 8, 8, 8>;
      FR_SWEEPS(P, 8, 16);
    }
    case 128: {
      using P = Plan<128, 16, 16, 8>;
      FR_SWEEPS(P, 16, 32);
    }
    case 256: {
      using P = Plan<256, 16, 16, 16>;
      FR_SWEEPS(P, 16, 32);
    }
    case 512: {
      using P = Plan<512, 8, 8, 8, 8>;
      FR_SWEEPS(P, 4, 16);
    }
    case 1024: {
      using P = Plan<1024, 16, 16, 8, 8>;
      FR_SWEEPS(P, 4, 8);
    }
    case 2048: {
      using P2 = Plan<2048, 16, 16, 16, 8>;
      if (variant == 1) FR_SWEEPS(P2, 2, 4);
      if (variant == 2) FR_SWEEPS(P2, 4, 4);
      FR_SWEEPS(P2, 2, 8);
    }
    case 4096: {
      using P4 = Plan<4096, 16, 16, 16, 16>;
      if (variant == 1) FR_SWEEPS(P4, 1, 2);
      if (variant == 2) FR_SWEEPS(P4, 2, 2);
      // column exchanges through half-size LDS lines
      if (variant == 3) return launch_sweeps<P4, 1, 4, P4, true>(fwd, nf, adj, na, root, s, hook);
      FR_SWEEPS(P4, 1, 4);
    }
    case 8192: {
      using P8 = Plan<8192, 16, 16, 16, 16, 2>;
      if (variant == 1) FR_SWEEPS(P8, 1, 1);
      if (variant == 2) FR_SWEEPS(P8, 2, 1);
      FR_SWEEPS(P8, 1, 2);
    }
    default: return hipErrorInvalidValue;
  }
#undef FR_SWEEPS
}

// the exact-transfer-function step: row FFT (optic prologue, or plain for the adjoint), column
// FFT * H * IFFT, row IFFT (plain, or the conjugate optic epilogue for the adjoint), each sweep
// the direct step's kernel with its own plane arguments
// (planes whose bit is set in `split` have H in its split form: their column sweep is the split
// instance's launch, the others' the float64 one's, so each plane takes the kernels it takes in
// a call of its own)
template <class PL, int RL, int CL>
hipError_t launch_exact_sweeps(const PlaneArgs *planes, int count, const float2 *tw, hipStream_t s,
                               const LaunchHook &hook, uint64_t split) {
  constexpr int N = PL::N;
  BatchArgs a, b, c, bs;
  int nb = 0, ns = 0;
  for (int i = 0; i < count; ++i) {
    const PlaneArgs &p = planes[i];
    const bool adj = p.flags & FR_ADJOINT;
    PlaneArgs plain = p;
    plain.amp = plain.opd = plain.pre_surf = plain.post_surf = nullptr;
    plain.lens = nullptr;
    a.p[i] = adj ? plain : p;
    a.p[i].flags = 0;                        // forward row transform (optic first when forward)
    PlaneArgs &col = (split >> i) & 1u ? bs.p[ns++] : b.p[nb++];
    col = p;
    col.flags = p.flags & FR_ADJOINT;
    c.p[i] = adj ? p : plain;
    c.p[i].flags = FR_ADJOINT;               // inverse row transform (conjugate optic after when adjoint)
  }
  auto rows = [&](const BatchArgs &x, const char *name) {
    hook(s, name, count, 0);
    hipLaunchKernelGGL((row_sweep<PL, RL, true>), dim3(N / RL, count), dim3(PL::T * RL), 0, s, x, tw);
    hipError_t e = hipGetLastError();
    hook(s, name, count, 1);
    return e;
  };
  hipError_t e = rows(a, "exact_rows_fwd");
  if (e != hipSuccess) return e;
  if (ns) {
    hook(s, "exact_cols", ns, 0);
    hipLaunchKernelGGL((col_sweep<PL, CL, false, true, 2>), dim3(N / CL, ns), dim3(PL::T * CL), 0, s, bs, tw);
    e = hipGetLastError();
    hook(s, "exact_cols", ns, 1);
    if (e != hipSuccess) return e;
  }
  if (nb) {
    hook(s, "exact_cols_f64", nb, 0);
    hipLaunchKernelGGL((col_sweep<PL, CL, false, true, 1>), dim3(N / CL, nb), dim3(PL::T * CL), 0, s, b, tw);
    e = hipGetLastError();
    hook(s, "exact_cols_f64", nb, 1);
  }
  if (e != hipSuccess) return e;
  return rows(c, "exact_rows_inv");
}

hipError_t launch_exact_batch(const PlaneArgs *planes, int count, int n, const float2 *root, hipStream_t s,
                              const LaunchHook &hook, uint64_t split) {
  switch (n) {
    case 64: return launch_exact_sweeps<Plan<64, 8, 8, 8>, 8, 16>(planes, count, root, s, hook, split);
    case 128: return launch_exact_sweeps<Plan<128, 16, 16, 8>, 16, 32>(planes, count, root, s, hook, split);
    case 256: return launch_exact_sweeps<Plan<256, 16, 16, 16>, 16, 32>(planes, count, root, s, hook, split);
    case 512: return launch_exact_sweeps<Plan<512, 8, 8, 8, 8>, 4, 16>(planes, count, root, s, hook, split);
    case 1024: return launch_exact_sweeps<Plan<1024, 16, 16, 8, 8>, 4, 8>(planes, count, root, s, hook, split);
    case 2048: return launch_exact_sweeps<Plan<2048, 16, 16, 16, 8>, 2, 8>(planes, count, root, s, hook, split);
    case 4096: return launch_exact_sweeps<Plan<4096, 16, 16, 16, 16>, 1, 4>(planes, count, root, s, hook, split);
    case 8192: return launch_exact_sweeps<Plan<8192, 16, 16, 16, 16, 2>, 1, 2>(planes, count, root, s, hook, split);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_direct_batch(const PlaneArgs *planes, int count, int n, const float2 *root, hipStream_t s,
                               const LaunchHook &hook) {
  BatchArgs fwd, adj;
  int nf = 0, na = 0;
  for (int i = 0; i < count; ++i) {
    if (planes[i].flags & FR_ADJOINT)
      adj.p[na++] = planes[i];
    else
      fwd.p[nf++] = planes[i];
  }
#define FR_DIRECT(PL, RL, CL) return launch_sweeps<PL, RL, CL, PL, false, true>(fwd, nf, adj, na, root, s, hook)
  switch (n) {
    case 64: { using P = Plan<64, 8, 8, 8>; FR_DIRECT(P, 8, 16); }
    case 128: { using P = Plan<128, 16, 16, 8>; FR_DIRECT(P, 16, 32); }
    case 256: { using P = Plan<256, 16, 16, 16>; FR_DIRECT(P, 16, 32); }
    case 512: { using P = Plan<512, 8, 8, 8, 8>; FR_DIRECT(P, 4, 16); }
    case 1024: { using P = Plan<1024, 16, 16, 8, 8>; FR_DIRECT(P, 4, 8); }
    case 2048: { using P = Plan<2048, 16, 16, 16, 8>; FR_DIRECT(P, 2, 8); }
    case 4096: { using P = Plan<4096, 16, 16, 16, 16>; FR_DIRECT(P, 1, 4); }
    case 8192: { using P = Plan<8192, 16, 16, 16, 16, 2>; FR_DIRECT(P, 1, 2); }
    default: return hipErrorInvalidValue;
  }
#undef FR_DIRECT
}

}  // namespace fr
