// Mixed-radix Fresnel sweeps for plane edges that factor into radices up to 16 (for example the
// per-wavelength grids 3584 ... 4096 of a broadband model, Sec. 1.2), with planes of different
// edges in one persistent launch per sweep.
//
// Same algorithm as the power-of-two sweeps (row pass and column pass, each FFT, * h, inverse
// FFT, with the optics in the prologue/epilogue), but the radix plan is a runtime list and every
// Stockham pass goes through LDS: a thread reads the R inputs of each butterfly it owns, applies
// the twiddles (per-pass float32 tables built in float64 on the host), runs DFT_R, and writes
// the outputs after a barrier. The transfer function is applied while the first inverse pass
// reads its inputs. Blocks loop over a flattened list of (plane, row) or (plane, 4-column tile)
// work items, so one launch covers a whole batch of uneven planes.
//
// All global accesses use raw buffer instructions with a per-lane offset clamped inside the
// array, so every access is range-checked by the hardware.
#include <algorithm>

#include "fft_mr.hpp"
#include "fr_internal.h"
#include "../../include/fresnel.h"

namespace fr {

namespace {

constexpr int kT = kMrThreads;    // threads per line
constexpr int kEM = kMrMaxN / kT;  // slots per thread for the global load / store

__device__ __forceinline__ c32 ld2(const float2 *p) {
  float2 v = *p;
  return {v.x, v.y};
}

struct Buf64 {
  __amdgpu_buffer_rsrc_t r;
  typedef unsigned int raw64 __attribute__((__vector_size__(8)));
  __device__ __forceinline__ Buf64(const void *p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, int(bytes), 0x00020000)) {}
  __device__ __forceinline__ c32 load(unsigned vo) const {
    const float2 q = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0u, 0));
    return {q.x, q.y};
  }
  __device__ __forceinline__ void store(unsigned vo, c32 v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw64, make_float2(v.x, v.y)), r, vo, 0u, 0);
  }
};

struct Buf32 {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Buf32(const void *p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, int(bytes), 0x00020000)) {}
  __device__ __forceinline__ float load(unsigned vo) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, 0u, 0));
  }
};

// pre optic amp exp(2 pi i (opd + 2 pre_surf) / lambda) lens[x] lens[y] at (y, x), x < n
__device__ __forceinline__ c32 mr_pre_optic(const PlaneArgs &pa, int n, int y, int x) {
  const int win = pa.win;
  const int off = (n - win) >> 1;
  const int wy = y - off, wx = x - off;
  const bool in = unsigned(wy) < unsigned(win) && unsigned(wx) < unsigned(win);
  float a = 1.0f, turns = 0.0f;
  if (pa.amp || pa.opd) {
    const unsigned o = unsigned(min(max(wy, 0), win - 1) * win + min(max(wx, 0), win - 1)) * 4u;
    const unsigned bytes = unsigned(win) * unsigned(win) * 4u;
    if (pa.amp) a = in ? Buf32(pa.amp, bytes).load(o) : 0.0f;
    if (pa.opd && in) turns = Buf32(pa.opd, bytes).load(o) * pa.inv_lambda;
  }
  if (pa.pre_surf)
    turns += 2.0f * Buf32(pa.pre_surf, unsigned(n) * unsigned(n) * 4u).load(unsigned(y * n + x) * 4u) * pa.inv_lambda;
  c32 ph = {a, 0.0f};
  if (pa.opd || pa.pre_surf) {
    float s, c;
    sincos_turns(turns, &s, &c);
    ph = {a * c, a * s};
  }
  if (pa.lens) ph = cmul(ph, cmul(ld2(pa.lens + x), ld2(pa.lens + y)));
  return ph;
}

__device__ __forceinline__ c32 mr_post_optic(const PlaneArgs &pa, int n, int y, int x) {
  float s, c;
  sincos_turns(2.0f * Buf32(pa.post_surf, unsigned(n) * unsigned(n) * 4u).load(unsigned(y * n + x) * 4u) *
                   pa.inv_lambda,
               &s, &c);
  return {c, s};
}

__device__ __forceinline__ bool mr_has_pre(const PlaneArgs &pa) {
  return pa.amp || pa.opd || pa.pre_surf || pa.lens;
}

template <bool INV>
__device__ __forceinline__ void plane_fft(c32 *lds, const MrPlane &mp, int t, const float2 *h, bool hconj) {
  mr_fft<INV, kT, kMrMaxN>(lds, mp.n, mp.npass, mp.plan, mp.tw, t, h, hconj);
}

// The batch is the kernel's only argument, so it sits at offset 0 of the kernel-argument
// segment; reading it through that pointer keeps the dynamically indexed plane table in the
// (scalar-loaded, read-only) argument segment instead of a private copy.
__device__ __forceinline__ const MrBatch &kernarg_batch() {
  return *(const MrBatch *)__builtin_amdgcn_kernarg_segment_ptr();
}

// work item -> plane (the batch is at most kMrMaxBatch planes; block-uniform scan)
__device__ __forceinline__ int mr_find(const MrBatch &a, int item) {
  int p = 0;
  while (p + 1 < a.count && item >= a.p[p + 1].first) ++p;
  return p;
}

// blocks are dealt round-robin to the 8 XCDs; inside each round of gridDim items, give every XCD
// a contiguous run of items so that concurrently running neighbours share L2 lines
__device__ __forceinline__ int mr_item(int round) {
  const int g = gridDim.x, b = blockIdx.x;
  const int local = (g % 8 == 0) ? (b & 7) * (g / 8) + (b >> 3) : b;
  return round * g + local;
}

__global__ void __launch_bounds__(kT) mr_row_sweep(MrBatch) {
  const MrBatch &args = kernarg_batch();
  __shared__ c32 lds[LdsLine<kMrMaxN>::size];
  const int t0 = threadIdx.x;
  for (int round = 0;; ++round) {
    const int item = mr_item(round);
    if (round * int(gridDim.x) >= args.total) break;
    if (item < args.total) {
      const MrPlane &mp = args.p[mr_find(args, item)];
      const PlaneArgs &pa = mp.pa;
      const int n = mp.n, y = item - mp.first;
      const int t = mr_opaque(t0);
      const bool adj = pa.flags & FR_ADJOINT;
      const Buf64 fb(pa.field, unsigned(n) * unsigned(n) * 8u);
#pragma unroll
      for (int m = 0; m < kEM; ++m) {
        const int x = t + kT * m;
        if (x < n) {
          c32 v;
          if (pa.flags & kSourceOptic) {
            v = mr_has_pre(pa) ? mr_pre_optic(pa, n, y, x) : c32{1.0f, 0.0f};
          } else {
            v = fb.load(unsigned(y * n + x) * 8u);
            if (!adj && mr_has_pre(pa)) v = cmul(v, mr_pre_optic(pa, n, y, x));
          }
          lds[lds_pad(x)] = v;
        }
      }
      __syncthreads();
      plane_fft<false>(lds, mp, t, nullptr, false);
      plane_fft<true>(lds, mp, t, pa.h, adj);
#pragma unroll
      for (int m = 0; m < kEM; ++m) {
        const int x = t + kT * m;
        if (x < n) {
          c32 v = lds[lds_pad(x)];
          if (adj && mr_has_pre(pa)) v = cmulc(v, mr_pre_optic(pa, n, y, x));
          fb.store(unsigned(y * n + x) * 8u, v);
        }
      }
      __syncthreads();
    }
  }
}

// 4 adjacent columns per item (32-byte row segments), one line of kT threads per column
__global__ void __launch_bounds__(kT * 4) mr_col_sweep(MrBatch) {
  const MrBatch &args = kernarg_batch();
  __shared__ c32 lds[4 * (LdsLine<kMrMaxN>::size + 4)];
  const int c = threadIdx.x & 3, t0 = threadIdx.x >> 2;
  c32 *my = lds + c * (LdsLine<kMrMaxN>::size + 4);
  for (int round = 0;; ++round) {
    const int item = mr_item(round);
    if (round * int(gridDim.x) >= args.total) break;
    if (item < args.total) {
      const MrPlane &mp = args.p[mr_find(args, item)];
      const PlaneArgs &pa = mp.pa;
      const int n = mp.n;
      const int t = mr_opaque(t0);
      const int x = (item - mp.first) * 4 + c;
      const bool xin = x < n;
      const int xc = min(x, n - 1);
      const bool adj = pa.flags & FR_ADJOINT;
      const Buf64 fb(pa.field, unsigned(n) * unsigned(n) * 8u);
#pragma unroll
      for (int m = 0; m < kEM; ++m) {
        const int y = t + kT * m;
        if (y < n) {
          c32 v = fb.load(unsigned(y * n + xc) * 8u);
          if (adj && pa.post_surf) v = cmulc(v, mr_post_optic(pa, n, y, xc));
          my[lds_pad(y)] = v;
        }
      }
      __syncthreads();
      plane_fft<false>(my, mp, t, nullptr, false);
      plane_fft<true>(my, mp, t, pa.h, adj);
#pragma unroll
      for (int m = 0; m < kEM; ++m) {
        const int y = t + kT * m;
        if (y < n && xin) {
          c32 v = my[lds_pad(y)];
          if (!adj && pa.post_surf) v = cmul(v, mr_post_optic(pa, n, y, x));
          fb.store(unsigned(y * n + x) * 8u, v);
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace

bool mr_plan(int n, int *npass, int *radix) { return mr_plan_build(n, kMrMaxN, kMrMaxPass, npass, radix); }
unsigned mr_pack(int npass, const int *radix) { return mr_plan_pack(npass, radix); }
int mr_twiddle_count(int npass, const int *radix) { return mr_twiddle_size(npass, radix); }
void mr_twiddle_build(int npass, const int *radix, float2 *out) { mr_twiddle_fill(npass, radix, out); }

hipError_t launch_mr_batch(const MrBatch &all, int blocks_rows, int blocks_cols, hipStream_t s,
                           const LaunchHook &hook) {
  // forward planes: rows then columns; adjoint planes: columns then rows (see the power-of-two
  // sweeps: the optic maps are always read along rows)
  MrBatch fwd, adj;
  fwd.count = adj.count = 0;
  fwd.total = adj.total = 0;
  for (int i = 0; i < all.count; ++i) {
    MrBatch &dst = (all.p[i].pa.flags & FR_ADJOINT) ? adj : fwd;
    dst.p[dst.count++] = all.p[i];
  }
  auto rows_list = [](MrBatch &b) {
    int acc = 0;
    for (int i = 0; i < b.count; ++i) {
      b.p[i].first = acc;
      acc += b.p[i].n;
    }
    b.total = acc;
  };
  auto cols_list = [](MrBatch &b) {
    int acc = 0;
    for (int i = 0; i < b.count; ++i) {
      b.p[i].first = acc;
      acc += (b.p[i].n + 3) / 4;
    }
    b.total = acc;
  };
  auto rows = [&](MrBatch b) {
    rows_list(b);
    hook(s, "mr_row_sweep", b.count, 0);
    hipLaunchKernelGGL(mr_row_sweep, dim3(std::max(1, std::min(blocks_rows, b.total))), dim3(kT), 0, s, b);
    hipError_t e = hipGetLastError();
    hook(s, "mr_row_sweep", b.count, 1);
    return e;
  };
  auto cols = [&](MrBatch b) {
    cols_list(b);
    hook(s, "mr_col_sweep", b.count, 0);
    hipLaunchKernelGGL(mr_col_sweep, dim3(std::max(1, std::min(blocks_cols, b.total))), dim3(4 * kT), 0, s, b);
    hipError_t e = hipGetLastError();
    hook(s, "mr_col_sweep", b.count, 1);
    return e;
  };
  hipError_t e = hipSuccess;
  if (fwd.count && (e = rows(fwd)) != hipSuccess) return e;
  if (fwd.count && (e = cols(fwd)) != hipSuccess) return e;
  if (adj.count && (e = cols(adj)) != hipSuccess) return e;
  if (adj.count && (e = rows(adj)) != hipSuccess) return e;
  return e;
}

}  // namespace fr
