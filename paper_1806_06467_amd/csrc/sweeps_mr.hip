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
// work items, so one launch covers a whole batch of uneven planes. For some of a broadband
// model's grid edges a register-resident form (MrReg: the line in registers between a
// transform's first and last passes, as in the power-of-two sweeps) runs instead, one row or
// 4-column tile per block, when every plane of the launch has that edge and its plan.
//
// All global accesses use raw buffer instructions with a per-lane offset clamped inside the
// array, so every access is range-checked by the hardware.
#include <algorithm>
#include <tuple>
#include <type_traits>
#include <utility>

#include "fft_mr.hpp"
#include "fr_internal.h"
#include "../../include/fresnel.h"

namespace fr {

namespace {

constexpr int kT = kMrThreads;    // threads per line
constexpr int kEM = kMrMaxN / kT;  // slots per thread for the global load / store

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

// The optic maps of a plane as buffer resources. A missing map gets zero records, so its loads
// return 0 without touching memory: every slot's loads are then issued together, with no
// branch between them, and the selects below drop the missing terms.
struct PreMaps {
  Buf32 amp, opd, pre;
  Buf64 lens;
  int n, win, off;
  float inv_lambda;
  bool has_amp, has_phase, has_lens;
  __device__ __forceinline__ PreMaps(const PlaneArgs &pa, int n_)
      : amp(pa.amp, pa.amp ? unsigned(pa.win) * unsigned(pa.win) * 4u : 0u),
        opd(pa.opd, pa.opd ? unsigned(pa.win) * unsigned(pa.win) * 4u : 0u),
        pre(pa.pre_surf, pa.pre_surf ? unsigned(n_) * unsigned(n_) * 4u : 0u),
        lens(pa.lens, pa.lens ? unsigned(n_) * 8u : 0u),
        n(n_), win(pa.win), off((n_ - pa.win) >> 1), inv_lambda(pa.inv_lambda), has_amp(pa.amp != nullptr),
        has_phase(pa.opd != nullptr || pa.pre_surf != nullptr), has_lens(pa.lens != nullptr) {}
};
struct PreVals {
  float a, o, p;
  c32 lx;
};

// loads of the pre optic at (y, x), both < n
__device__ __forceinline__ PreVals pre_fetch(const PreMaps &m, int y, int x) {
  const int wy = min(max(y - m.off, 0), m.win - 1), wx = min(max(x - m.off, 0), m.win - 1);
  const unsigned o = unsigned(wy * m.win + wx) * 4u;
  PreVals v;
  v.a = m.amp.load(o);
  v.o = m.opd.load(o);
  v.p = m.pre.load(unsigned(y * m.n + x) * 4u);
  v.lx = m.lens.load(unsigned(x) * 8u);
  return v;
}

// pre optic amp exp(2 pi i (opd + 2 pre_surf) / lambda) lens[x] lens[y] at (y, x); ly = lens[y]
__device__ __forceinline__ c32 pre_optic(const PreMaps &m, const PreVals &v, int y, int x, c32 ly) {
  const bool in = unsigned(y - m.off) < unsigned(m.win) && unsigned(x - m.off) < unsigned(m.win);
  const float a = m.has_amp ? (in ? v.a : 0.0f) : 1.0f;
  c32 ph = {a, 0.0f};
  if (m.has_phase) {
    const float turns = (in ? v.o : 0.0f) * m.inv_lambda + 2.0f * v.p * m.inv_lambda;
    float s, c;
    sincos_turns(turns, &s, &c);
    ph = {a * c, a * s};
  }
  if (m.has_lens) ph = cmul(ph, cmul(v.lx, ly));
  return ph;
}

__device__ __forceinline__ bool mr_has_pre(const PlaneArgs &pa) {
  return pa.amp || pa.opd || pa.pre_surf || pa.lens;
}

// The plan policy of a sweep instance: MrRuntime takes each plane's packed plan (any edge),
// MrCt<N, Rs...> one compile-time plan (every plane of the launch has edge N and that plan).
struct MrRuntime {
  static constexpr int N = 0;
};

template <class F, bool INV>
__device__ __forceinline__ void plane_fft(c32 *lds, const MrPlane &mp, int t, const float2 *h, bool hconj) {
  if constexpr (F::N == 0)
    mr_fft<INV, kT, kMrMaxN>(lds, mp.n, mp.npass, mp.plan, mp.tw, t, h, hconj);
  else
    F::template fft<INV, kT>(lds, mp.tw, mr_opaque(t), h, hconj);
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

// slots of the global load / store handled per batch of optic loads
constexpr int kOptBatch = 8;

// multiplies v[0..kEM) of row y by the pre optic (conjugated when CONJ), in batches of
// kOptBatch slots whose loads are issued together
template <bool CONJ>
__device__ __forceinline__ void apply_pre(c32 (&v)[kEM], const PlaneArgs &pa, int n, int y, int t, bool source) {
  const PreMaps pm(pa, n);
  const c32 ly = pm.lens.load(unsigned(y) * 8u);
#pragma unroll
  for (int m0 = 0; m0 < kEM; m0 += kOptBatch) {
    PreVals pv[kOptBatch];
#pragma unroll
    for (int q = 0; q < kOptBatch; ++q) pv[q] = pre_fetch(pm, y, min(t + kT * (m0 + q), n - 1));
#pragma unroll
    for (int q = 0; q < kOptBatch; ++q) {
      const c32 ph = pre_optic(pm, pv[q], y, min(t + kT * (m0 + q), n - 1), ly);
      v[m0 + q] = source ? ph : (CONJ ? cmulc(v[m0 + q], ph) : cmul(v[m0 + q], ph));
    }
  }
}

template <class F>
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
      const int n = F::N ? F::N : mp.n, y = item - mp.first;
      const int t = mr_opaque(t0);
      const bool adj = pa.flags & FR_ADJOINT;
      const bool source = pa.flags & kSourceOptic;
      const bool pre = mr_has_pre(pa);
      const Buf64 fb(pa.field, unsigned(n) * unsigned(n) * 8u);
      c32 v[kEM];
      if (source) {
#pragma unroll
        for (int m = 0; m < kEM; ++m) v[m] = {1.0f, 0.0f};
      } else {
#pragma unroll
        for (int m = 0; m < kEM; ++m) v[m] = fb.load(unsigned(y * n + min(t + kT * m, n - 1)) * 8u);
      }
      if (!adj && pre) apply_pre<false>(v, pa, n, y, t, source);
#pragma unroll
      for (int m = 0; m < kEM; ++m)
        if (t + kT * m < n) lds[lds_pad(t + kT * m)] = v[m];
      __syncthreads();
      plane_fft<F, false>(lds, mp, t, nullptr, false);
      plane_fft<F, true>(lds, mp, t, pa.h, adj);
#pragma unroll
      for (int m = 0; m < kEM; ++m) v[m] = lds[lds_pad(min(t + kT * m, n - 1))];
      if (adj && pre) apply_pre<true>(v, pa, n, y, t, false);
#pragma unroll
      for (int m = 0; m < kEM; ++m)
        if (t + kT * m < n) fb.store(unsigned(y * n + t + kT * m) * 8u, v[m]);
      __syncthreads();
    }
  }
}

// 4 adjacent columns per item (32-byte row segments), one line of kT threads per column
template <class F>
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
      const int n = F::N ? F::N : mp.n;
      const int t = mr_opaque(t0);
      const int x = (item - mp.first) * 4 + c;
      const bool xin = x < n;
      const int xc = min(x, n - 1);
      const bool adj = pa.flags & FR_ADJOINT;
      const Buf64 fb(pa.field, unsigned(n) * unsigned(n) * 8u);
      // a missing post map has zero records (its loads return 0)
      const Buf32 post(pa.post_surf, pa.post_surf ? unsigned(post_tiled_size(n)) * 4u : 0u);
      const bool has_post = pa.post_surf != nullptr;
      c32 v[kEM];
#pragma unroll
      for (int m = 0; m < kEM; ++m) v[m] = fb.load(unsigned(min(t + kT * m, n - 1) * n + xc) * 8u);
      if (adj && has_post) {
        float sv[kEM];
#pragma unroll
        for (int m = 0; m < kEM; ++m) sv[m] = post.load(unsigned(post_tiled_index(n, min(t + kT * m, n - 1), xc)) * 4u);
#pragma unroll
        for (int m = 0; m < kEM; ++m) {
          float sn, cs;
          sincos_turns(2.0f * sv[m] * pa.inv_lambda, &sn, &cs);
          v[m] = cmulc(v[m], c32{cs, sn});
        }
      }
#pragma unroll
      for (int m = 0; m < kEM; ++m)
        if (t + kT * m < n) my[lds_pad(t + kT * m)] = v[m];
      __syncthreads();
      plane_fft<F, false>(my, mp, t, nullptr, false);
      plane_fft<F, true>(my, mp, t, pa.h, adj);
#pragma unroll
      for (int m = 0; m < kEM; ++m) v[m] = my[lds_pad(min(t + kT * m, n - 1))];
      if (!adj && has_post) {
        float sv[kEM];
#pragma unroll
        for (int m = 0; m < kEM; ++m) sv[m] = post.load(unsigned(post_tiled_index(n, min(t + kT * m, n - 1), xc)) * 4u);
#pragma unroll
        for (int m = 0; m < kEM; ++m) {
          float sn, cs;
          sincos_turns(2.0f * sv[m] * pa.inv_lambda, &sn, &cs);
          v[m] = cmul(v[m], c32{cs, sn});
        }
      }
#pragma unroll
      for (int m = 0; m < kEM; ++m)
        if (t + kT * m < n && xin) fb.store(unsigned((t + kT * m) * n + x) * 8u, v[m]);
      __syncthreads();
    }
  }
}

// ---- register-resident sweeps of the broadband grids' plans ------------------------------
// One row (row sweep) or one 4-column tile (column sweep, 32-byte row segments) per block, the
// line held in registers E elements per thread between a transform's first and last passes and
// from one transform to the next (MrReg); grid (lines, planes) with every plane of the launch of
// the policy's edge and plan.

// the pre optic on the slots x = t + T m of row y (conjugated when CONJ; the source optic itself
// when `source`), loads issued kOptBatch slots at a time
template <int E, int T, bool CONJ>
__device__ __forceinline__ void apply_pre_reg(c32 (&v)[E], const PlaneArgs &pa, int n, int y, int t, bool source) {
  const PreMaps pm(pa, n);
  const c32 ly = pm.lens.load(unsigned(y) * 8u);
#pragma unroll
  for (int m0 = 0; m0 < E; m0 += kOptBatch) {
    constexpr int B = kOptBatch;
    PreVals pv[B];
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (m0 + q < E) pv[q] = pre_fetch(pm, y, t + T * (m0 + q));
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (m0 + q < E) {
        const c32 ph = pre_optic(pm, pv[q], y, t + T * (m0 + q), ly);
        v[m0 + q] = source ? ph : (CONJ ? cmulc(v[m0 + q], ph) : cmul(v[m0 + q], ph));
      }
  }
}

// the frequency product with h (conj(h) for the adjoint); slot m holds frequency t + T m
template <int E, int T>
__device__ __forceinline__ void freq_reg(c32 (&v)[E], const float2 *h, int t, bool adj) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const float2 q = h[t + T * m];
    v[m] = adj ? cmulc(v[m], c32{q.x, q.y}) : cmul(v[m], c32{q.x, q.y});
  }
}

template <class F>
__global__ void __launch_bounds__(F::T) mrr_row_sweep(MrBatch) {
  constexpr int N = F::N, E = F::E, T = F::T;
  const MrBatch &args = kernarg_batch();
  __shared__ c32 lds[LdsLine<N>::size];
  const MrPlane &mp = args.p[blockIdx.y];
  const PlaneArgs &pa = mp.pa;
  const int y = blockIdx.x, t = threadIdx.x;
  const bool adj = pa.flags & FR_ADJOINT;
  const bool source = pa.flags & kSourceOptic;
  const bool pre = mr_has_pre(pa);
  const Buf64 fb(pa.field, unsigned(N) * unsigned(N) * 8u);
  c32 v[E];
  if (source) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = {1.0f, 0.0f};
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = fb.load(unsigned(y * N + t + T * m) * 8u);
  }
  if (!adj && pre) apply_pre_reg<E, T, false>(v, pa, N, y, t, source);
  F::template fft<false>(v, lds, t, mp.tw);
  freq_reg<E, T>(v, pa.h, t, adj);
  F::template fft<true>(v, lds, t, mp.tw);
  if (adj && pre) apply_pre_reg<E, T, true>(v, pa, N, y, t, false);
#pragma unroll
  for (int m = 0; m < E; ++m) fb.store(unsigned(y * N + t + T * m) * 8u, v[m]);
}

// the post surface phasor exp(2 pi i 2 s / lambda) at rows t + T m of column x (conjugated when
// CONJ), from the 4-column tiled map
template <int E, int T, bool CONJ>
__device__ __forceinline__ void apply_post_reg(c32 (&v)[E], const PlaneArgs &pa, int n, int t, int x) {
  const Buf32 post(pa.post_surf, unsigned(post_tiled_size(n)) * 4u);
  float sv[E];
#pragma unroll
  for (int m = 0; m < E; ++m) sv[m] = post.load(unsigned(post_tiled_index(n, t + T * m, x)) * 4u);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    float sn, cs;
    sincos_turns(2.0f * sv[m] * pa.inv_lambda, &sn, &cs);
    v[m] = CONJ ? cmulc(v[m], c32{cs, sn}) : cmul(v[m], c32{cs, sn});
  }
}

template <class F>
__global__ void __launch_bounds__(4 * F::T) mrr_col_sweep(MrBatch) {
  constexpr int N = F::N, E = F::E, T = F::T;
  static_assert(N % 4 == 0, "4-column tiles");
  constexpr int G = N / 4;  // column tiles per plane
  constexpr int LINE = LdsLine<N>::size + 8;
  const MrBatch &args = kernarg_batch();
  __shared__ c32 lds[4 * LINE];
  const MrPlane &mp = args.p[blockIdx.y];
  const PlaneArgs &pa = mp.pa;
  const int c = threadIdx.x & 3, t = threadIdx.x >> 2;
  // blocks are dealt round-robin to the 8 XCDs: XCD i takes a contiguous run of the tiles
  const int i = blockIdx.x & 7, k = blockIdx.x >> 3;
  const int g = i * (G / 8) + min(i, G % 8) + k;
  const int x = g * 4 + c;
  const bool adj = pa.flags & FR_ADJOINT;
  const Buf64 fb(pa.field, unsigned(N) * unsigned(N) * 8u);
  c32 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = fb.load(unsigned((t + T * m) * N + x) * 8u);
  if (adj && pa.post_surf) apply_post_reg<E, T, true>(v, pa, N, t, x);
  c32 *my = lds + c * LINE;
  F::template fft<false>(v, my, t, mp.tw);
  freq_reg<E, T>(v, pa.h, t, adj);
  F::template fft<true>(v, my, t, mp.tw);
  if (!adj && pa.post_surf) apply_post_reg<E, T, false>(v, pa, N, t, x);
#pragma unroll
  for (int m = 0; m < E; ++m) fb.store(unsigned((t + T * m) * N + x) * 8u, v[m]);
}

}  // namespace

bool mr_plan(int n, int *npass, int *radix) { return mr_plan_build(n, kMrMaxN, kMrMaxPass, npass, radix); }
unsigned mr_pack(int npass, const int *radix) { return mr_plan_pack(npass, radix); }
int mr_plan_orders(int n, int max, unsigned *plans, int *npass) {
  int rad[kMrMaxPass];
  if (!mr_plan_build(n, kMrMaxN, kMrMaxPass, npass, rad)) return 0;
  std::sort(rad, rad + *npass, [](int a, int b) { return a > b; });
  int count = 0;
  do {
    plans[count++] = mr_plan_pack(*npass, rad);
  } while (count < max && std::next_permutation(rad, rad + *npass, [](int a, int b) { return a > b; }));
  return count;
}
int mr_twiddle_count(int npass, const int *radix) { return mr_twiddle_size(npass, radix); }
void mr_twiddle_build(int npass, const int *radix, float2 *out) { mr_twiddle_fill(npass, radix, out); }

// blocks of a persistent kernel that one compute unit holds at once
template <class K>
int resident_blocks(K kernel, int threads, int fallback) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    return fallback;
  }
  return nb;
}

// compile-time plans: the greedy plans of the 7-smooth grid edges of a broadband model
// (3584 ... 4032, Sec. 1.2); other edges and other pass orders take the runtime plan
using MrCtPlans = std::tuple<MrCt<3584, 16, 16, 14>, MrCt<3600, 16, 15, 15>, MrCt<3840, 16, 16, 15>,
                             MrCt<3888, 16, 9, 9, 3>, MrCt<3920, 16, 7, 7, 5>, MrCt<4000, 16, 10, 5, 5>,
                             MrCt<4032, 16, 14, 9, 2>>;
constexpr int kMrCt = std::tuple_size<MrCtPlans>::value;

// register-resident plans of the same edges: factorisations whose first and last radices divide
// the elements per thread (E), T = N / E threads per line, 4 T per column tile. With E = 14 or 15
// and every middle radix 16 a middle pass's butterflies fit the threads (one each), so 3584, 3600
// and 3840 run as the power-of-two sweeps do (measured per plane, rows / columns: 3584 81 / 109 us
// against 113 / 124 us for the greedy compile-time plan, 3600 96 / 104 against 117 / 129, 3840
// 99 / 119 against 118 / 134); for 4032 the middle passes take two rounds and the column sweep
// spills at its 128 registers (152 / 179 against 181 / 166 us: still ahead over both sweeps).
// 3888, 3920 and 4000 have no such factorisation under the 256-thread lines of a 4-column tile
// and keep the greedy compile-time plans. These orders are the edges' default plans
// (mr_default_plan); a tuning file may choose another.
using MrRegPlans = std::tuple<MrReg<3584, 14, 7, 16, 16, 2>, MrReg<3600, 15, 15, 16, 15>,
                              MrReg<3840, 15, 3, 16, 16, 5>, MrReg<4032, 18, 9, 16, 14, 2>>;
constexpr int kMrReg = std::tuple_size<MrRegPlans>::value;

// calls f(policy) and returns true when a register-resident plan runs edge n with plan `plan`
template <class Fn, int I = 0>
bool with_mr_reg(int n, unsigned plan, Fn &&f) {
  if constexpr (I == kMrReg) {
    return false;
  } else {
    using P = std::tuple_element_t<I, MrRegPlans>;
    if (n == P::N && plan == P::packed()) {
      f(P{});
      return true;
    }
    return with_mr_reg<Fn, I + 1>(n, plan, std::forward<Fn>(f));
  }
}

template <int I = 0>
unsigned mr_reg_plan(int n) {
  if constexpr (I == kMrReg) {
    return 0u;
  } else {
    using P = std::tuple_element_t<I, MrRegPlans>;
    return n == P::N ? P::packed() : mr_reg_plan<I + 1>(n);
  }
}

// calls f(policy) for the instance that runs planes of edge n with packed plan `plan` (the
// runtime policy when no compile-time plan matches)
template <class Fn, int I = 0>
auto with_mr_policy(int n, unsigned plan, Fn &&f) {
  if constexpr (I == kMrCt) {
    return f(MrRuntime{});
  } else {
    using P = std::tuple_element_t<I, MrCtPlans>;
    if (n == P::N && plan == P::packed()) return f(P{});
    return with_mr_policy<Fn, I + 1>(n, plan, std::forward<Fn>(f));
  }
}

template <int I = 0>
void resident_all(int *rows, int *cols) {
  if constexpr (I <= kMrCt) {
    using P = std::conditional_t<I == 0, MrRuntime, std::tuple_element_t<(I > 0 ? I - 1 : 0), MrCtPlans>>;
    rows[I] = resident_blocks(mr_row_sweep<P>, kT, 2);
    cols[I] = resident_blocks(mr_col_sweep<P>, 4 * kT, 1);
    resident_all<I + 1>(rows, cols);
  }
}

// 0 for the runtime plan, 1 + the index of the matching compile-time plan
template <int I = 0>
int mr_policy_index(int n, unsigned plan) {
  if constexpr (I == kMrCt) {
    return 0;
  } else {
    using P = std::tuple_element_t<I, MrCtPlans>;
    if (n == P::N && plan == P::packed()) return I + 1;
    return mr_policy_index<I + 1>(n, plan);
  }
}

unsigned mr_default_plan(int n) { return mr_reg_plan(n); }

void mr_resident(int *rows_per_cu, int *cols_per_cu) {
  static_assert(kMrCt + 1 <= kMrPolicies, "residency table size");
  resident_all(rows_per_cu, cols_per_cu);
}

hipError_t launch_mr_batch(const MrBatch &all, const int *rows_per_cu, const int *cols_per_cu, int cus,
                           hipStream_t s, const LaunchHook &hook) {
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
  // one compile-time instance when every plane of the batch has the same edge and its plan
  int pol = all.count ? mr_policy_index(all.p[0].n, all.p[0].plan) : 0;
  for (int i = 1; i < all.count && pol; ++i)
    if (all.p[i].n != all.p[0].n || all.p[i].plan != all.p[0].plan) pol = 0;
  // one register-resident instance when every plane has the same edge and its plan
  bool same = all.count > 0;
  for (int i = 1; i < all.count && same; ++i)
    if (all.p[i].n != all.p[0].n || all.p[i].plan != all.p[0].plan) same = false;
  const int nr = same ? all.p[0].n : 0;
  const unsigned planr = same ? all.p[0].plan : 0u;
  const int n0 = pol ? all.p[0].n : 0;
  const unsigned plan0 = pol ? all.p[0].plan : 0u;
  const int blocks_rows = cus * rows_per_cu[pol], blocks_cols = cus * cols_per_cu[pol];
  auto rows = [&](MrBatch b, const char *name) {
    rows_list(b);
    hook(s, name, b.count, 0);
    const bool reg = with_mr_reg(nr, planr, [&](auto p) {
      using P = decltype(p);
      hipLaunchKernelGGL((mrr_row_sweep<P>), dim3(P::N, b.count), dim3(P::T), 0, s, b);
    });
    if (!reg)
      with_mr_policy(n0, plan0, [&](auto p) {
        hipLaunchKernelGGL((mr_row_sweep<decltype(p)>), dim3(std::max(1, std::min(blocks_rows, b.total))),
                           dim3(kT), 0, s, b);
      });
    hipError_t e = hipGetLastError();
    hook(s, name, b.count, 1);
    return e;
  };
  auto cols = [&](MrBatch b, const char *name) {
    cols_list(b);
    hook(s, name, b.count, 0);
    const bool reg = with_mr_reg(nr, planr, [&](auto p) {
      using P = decltype(p);
      hipLaunchKernelGGL((mrr_col_sweep<P>), dim3(P::N / 4, b.count), dim3(4 * P::T), 0, s, b);
    });
    if (!reg)
      with_mr_policy(n0, plan0, [&](auto p) {
        hipLaunchKernelGGL((mr_col_sweep<decltype(p)>), dim3(std::max(1, std::min(blocks_cols, b.total))),
                           dim3(4 * kT), 0, s, b);
      });
    hipError_t e = hipGetLastError();
    hook(s, name, b.count, 1);
    return e;
  };
  hipError_t e = hipSuccess;
  if (fwd.count && (e = rows(fwd, "mr_row_sweep")) != hipSuccess) return e;
  if (fwd.count && (e = cols(fwd, "mr_col_sweep")) != hipSuccess) return e;
  if (adj.count && (e = cols(adj, "mr_col_sweep_adj")) != hipSuccess) return e;
  if (adj.count && (e = rows(adj, "mr_row_sweep_adj")) != hipSuccess) return e;
  return e;
}

}  // namespace fr
