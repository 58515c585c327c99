// Internal interfaces between the host runtime (api.cpp) and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fr {

struct c32;

// Optional per-launch callback (kernel timing): phase 0 just before a kernel launch on `s`,
// phase 1 just after it. `tag` distinguishes launches of one kernel (e.g. the plane edge).
struct LaunchHook {
  void (*fn)(void *user, hipStream_t s, const char *name, int tag, int phase) = nullptr;
  void *user = nullptr;
  void operator()(hipStream_t s, const char *name, int tag, int phase) const {
    if (fn) fn(user, s, name, tag, phase);
  }
};

// One plane of a Fresnel batch, as the sweep kernels see it (device pointers).
// Forward:  field <- post(x,y) * AS_z( src * pre(x,y) ),   src = field or 1 (kSourceOptic)
// Adjoint:  field <- conj(pre) * AS_{-z}( conj(post) * field )
//   pre  = amp * exp(2 pi i (opd + 2 pre_surf) / lambda) * lens[x] lens[y]
//   post = exp(2 pi i 2 post_surf / lambda)               (reflective DM after the step)
// amp and opd are win x win maps centred in the plane (offset (n - win)/2); outside the
// window amp is 0 when given. pre_surf is an n x n surface map [m], row-major; post_surf is the
// same kind of map stored in 4-column tiles (post_tiled_index) so that the column sweep, which
// applies it, reads it contiguously.
// A forward plane with a windowed amplitude (win < n) has zero rows outside the window after
// the optic; the power-of-two sweeps neither store them (row sweep) nor load them (column sweep).
constexpr int kSourceOptic = 2;  // forward only: the input field is 1 (it is not read)
constexpr int kTowardSource = 4;  // direct step over z < 0: the transforms' kernel sign flips
// adjoint planes: only the centred win rows of the output are needed (the others are left
// unspecified): the power-of-two column sweep, which runs first, stores only those rows, and
// the row sweep skips the blocks whose rows all lie outside them
constexpr int kWindowRowsOnly = 8;
struct PlaneArgs {
  float2 *field;             // n x n, in place
  const float *amp;          // win x win or null
  const float *opd;          // win x win OPD [m] or null
  const float *pre_surf;     // n x n or null
  const float *post_surf;    // n x n or null
  const float2 *h;           // n: exp(-i pi lambda z k^2/(n dx)^2) / n over signed index k
  const float2 *lens;        // n: exp(-i pi c^2 dx^2 / (lambda f)) or null
  float inv_lambda;          // 1 / lambda [1/m]
  int n;                     // plane edge
  int win;                   // window edge of amp / opd (n for full maps)
  int flags;                 // FR_ADJOINT | kSourceOptic | kTowardSource | kWindowRowsOnly
  int post_lo, post_hi;      // when post_hi > post_lo: post_surf is 0 outside columns [post_lo, post_hi)
};

// element (y, x) of an n x n map stored in 4-column tiles: tile x/4 holds rows 0..n-1 of its
// 4 columns, row-major within the tile (post_tiled_size(n) floats in all)
__host__ __device__ inline size_t post_tiled_index(int n, int y, int x) {
  return (size_t(x >> 2) * size_t(n) + size_t(y)) * 4 + size_t(x & 3);
}
__host__ __device__ inline size_t post_tiled_size(int n) { return size_t((n + 3) / 4) * 4 * size_t(n); }

constexpr int kMaxBatch = 64;
struct BatchArgs {
  PlaneArgs p[kMaxBatch];
};

// Row sweep then column sweep over `count` planes of edge n (count <= kMaxBatch).
// tw: the plan's twiddle table (fresnel_twiddle_build). Returns a hipError_t.
// `variant` selects a tile configuration (row lines per block, column tile width); every
// variant computes the same result. fresnel_variants(n) = number of variants for edge n.
hipError_t launch_fresnel_batch(const PlaneArgs *planes, int count, int n, const float2 *tw,
                                hipStream_t stream, const LaunchHook &hook, int variant);
// The direct (single-transform) Fresnel step of `count` planes of power-of-two edge n
// (count <= kMaxBatch): the row sweep applies the optic times the input quadratic phase (lens
// slot) and the forward transform, the column sweep the forward transform and the output
// quadratic phase (h slot). Same tiles as variant 0 of launch_fresnel_batch.
hipError_t launch_direct_batch(const PlaneArgs *planes, int count, int n, const float2 *tw, hipStream_t s,
                               const LaunchHook &hook);
int fresnel_variants(int n);
int fresnel_twiddle_count(int n);
void fresnel_twiddle_build(int n, float2 *out);  // host
bool fresnel_size_supported(int n);  // power-of-two edges with register-resident plans
bool plane_size_supported(int n);    // those or any mixed-radix edge

// ---- mixed-radix sweeps (any edge up to kMrMaxN that factors into radices <= 16) ----------
constexpr int kMrMaxN = 4096;
constexpr int kMrMaxPass = 6;
constexpr int kMrThreads = 256;
constexpr int kMrMaxBatch = 24;
struct MrPlane {
  PlaneArgs pa;
  int n, npass, first;  // first: index of the plane's first work item (set by the launcher)
  unsigned plan;        // radices, 5 bits per pass
  const float2 *tw;     // mr_twiddle_build table of the plan
};
struct MrBatch {
  int count, total;
  MrPlane p[kMrMaxBatch];
};
bool mr_plan(int n, int *npass, int *radix);
// distinct orders of the greedy plan's radices (the first is the greedy plan), at most `max`
int mr_plan_orders(int n, int max, unsigned *plans, int *npass);
unsigned mr_pack(int npass, const int *radix);
int mr_twiddle_count(int npass, const int *radix);
void mr_twiddle_build(int npass, const int *radix, float2 *out);  // host
// rows then columns for forward planes, columns then rows for adjoint planes; persistent grids
// of cus x the resident blocks per compute unit of the instance that runs them (a compile-time
// plan when every plane has the same edge and one of the broadband grids' plans, else the
// runtime plan)
hipError_t launch_mr_batch(const MrBatch &all, const int *rows_per_cu, const int *cols_per_cu, int cus,
                           hipStream_t s, const LaunchHook &hook);
// blocks of each instance of the two persistent sweeps that one compute unit holds at once
// (index 0 the runtime plan, then the compile-time plans); a device query, made at context
// creation
constexpr int kMrPolicies = 8;
void mr_resident(int *rows_per_cu, int *cols_per_cu);

// ---- MFT: out = alpha * c * A in B^T (+ beta * out) (* mask), complex, FP32 MFMA ------
// Generic complex GEMM pieces used by the MFT entry points.
struct CGemmArgs {
  int M, N, K;
  const float2 *A;  // M x K, row stride lda
  int lda;
  const float2 *B;  // K x N (or its transpose), row stride ldb
  int ldb;
  float2 *C;        // M x N, row stride ldc
  int ldc;
  int transA;       // 1: A is given as K x M (use A^T)
  int transB;       // 1: B is given as N x K (use B^T)
  int conjA, conjB; // conjugate the operand on load
  double alpha_re, alpha_im;  // applied in float64 in the epilogue
  float beta;       // real; the beta term reads Cin (row stride ldcin), or C when Cin is null
  const float2 *Cin;
  int ldcin;
  const float *mask;  // M x N (row stride ldm) or null: multiplies the result
  int ldm;
  double *intensity;  // M x N (row stride ldi) or null: intensity += weight |result|^2 (float64)
  int ldi;
  double weight;
  int skip_c;         // 1: do not write C (only the intensity)
};
// C = alpha op(A) op(B) (+ beta C) (* mask). split > 1 slices K; the slices' partial sums go
// to `partial` (split x M x N complex float64, 16-byte aligned) and are added in a fixed order
// by a second kernel.
constexpr int kMaxSplit = 16;
// cfg: tile configuration (0 small 64 x 64, 1 large 64 x 128, 2 extra large 128 x 128, 3 small
// with two stages of operand loads in flight, 4 small and 5 large with three real products per
// complex step, 6 small with the four real products formed from bfloat16 pieces of the
// operands on the bf16 matrix cores), or -1 for the default choice by shape
constexpr int kGemmTiles = 7;
int cgemm_split_for(int M, int N, int K, int cfg);
hipError_t launch_cgemm_split(const CGemmArgs &a, int split, int cfg, void *partial, hipStream_t stream,
                              const LaunchHook &hook);

}  // namespace fr
