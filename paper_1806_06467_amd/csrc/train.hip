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
  int tiled;  // 1: C is an n x n map stored in 4-column tiles (post_tiled_index), ldc unused
  int tn, t0; // tiled: the map's edge n and the offset of C's element (0, 0) on both axes
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
    float *cp = g.tiled ? g.C + post_tiled_index(g.tn, i + g.t0, j + g.t0) : g.C + size_t(i) * g.ldc + j;
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

__global__ void fill_f64(double *p, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

__global__ void to_f32(const double *src, float *dst, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    dst[i] = float(src[i]);
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

// DM gradient (a7) and its projection onto the actuators, dL/dA = G^T g_s G with
//   g_s[i][j] = -2 kappa Im(E[i][j] conj(B[i][j]))   (surface gradient, never stored)
// in deterministic steps:
//   dm_grad_T:   per (32-row strip, 512-column group) block, the group's share of
//                T[i][b] = sum_j g_s[i][j] G[j][b] on FP32 MFMA; one pass over E and B
//                (HBM-bound)
//   dm_grad_acc: T_sum += the sum of the group shares (group order)
//   dm_grad_G:   per 32-row block, the block's share of sum_i G[i][a] T_sum[i][b]
//   dm_grad_reduce: gA += the block shares, in a fixed order.
// G depends only on the grid edge and kappa enters g_s, so the projection is linear in the
// wavelengths' T: each DM keeps one T_sum that the wavelengths of a grid edge add into in
// wavelength order, and the last two steps run once per DM and grid edge.
// E is the stored plane, or (E == null) the pupil optic amp exp(2 pi i (opd + 2 pre) / lambda)
// synthesised here (amp/opd nd x nd centred, pre n x n).
constexpr int kRows = 32;    // rows per dm_grad_T block (one MFMA tile)
constexpr int kCJ = 64;      // columns per chunk
constexpr int kGroup = 512;  // columns per dm_grad_T block
constexpr int kGRows = 32;   // rows per dm_grad_G block
constexpr int kMaxAct = 64;  // actuators per DM edge supported

typedef float floatx16 __attribute__((ext_vector_type(16)));

// The loads of one chunk (the field values, or the optic maps when SYNTH, and the chunk's
// influence rows) with indices clamped inside the arrays; values outside the plane or the
// chunk are replaced by zero when they are used.
template <bool SYNTH>
struct GradChunk {
  static constexpr int kPer = kRows * kCJ / 256;     // field elements per thread
  static constexpr int kGPer = kCJ * kMaxAct / 256;  // influence values per thread
  float2 ev[kPer], bv[kPer];
  float ws[SYNTH ? kPer : 1], wa[SYNTH ? kPer : 1], wo[SYNTH ? kPer : 1];
  float gv[kGPer];
  // raw buffer loads: one 32-bit per-lane offset per access (planes up to 8192^2 c64 = 512 MiB)
  static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff, 0x00020000);
  }
  static __device__ __forceinline__ float2 ld64(__amdgpu_buffer_rsrc_t r, unsigned o) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
  }
  static __device__ __forceinline__ float ld32(__amdgpu_buffer_rsrc_t r, unsigned o) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
  }
  __device__ __forceinline__ void load(const float2 *E, const float2 *B, const float *G, int n, int na,
                                       const float *amp, const float *opd, int nd, const float *pre, int i0,
                                       int j0, int tid) {
    const int off = (n - nd) / 2;
    const int c = tid & (kCJ - 1);
    const __amdgpu_buffer_rsrc_t rb = rsrc(B), rg = rsrc(G);
    const int j = min(j0 + c, n - 1);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int r = (tid >> 6) + 4 * q;
      const int i = min(i0 + r, n - 1);
      const unsigned o = unsigned(i * n + j);
      bv[q] = ld64(rb, o * 8u);
      if constexpr (SYNTH) {
        const int wy = min(max(i - off, 0), nd - 1), wx = min(max(j - off, 0), nd - 1);
        const unsigned ow = unsigned(wy * nd + wx);
        ws[q] = ld32(rsrc(pre), o * 4u);
        wa[q] = ld32(rsrc(amp), ow * 4u);
        wo[q] = opd ? ld32(rsrc(opd), ow * 4u) : 0.f;
        ev[q] = make_float2(0.f, 0.f);
      } else {
        ev[q] = ld64(rsrc(E), o * 8u);
      }
    }
#pragma unroll
    for (int q = 0; q < kGPer; ++q) {
      const int e = tid + 256 * q;
      const int cc = e / kMaxAct, a = e % kMaxAct;
      gv[q] = ld32(rg, unsigned(min(j0 + cc, n - 1) * na + min(a, na - 1)) * 4u);
    }
  }
};

// Block: 4 waves over a 32-row strip and one column group. Per 64-column chunk the surface
// gradient g_s (32 x 64) and the influence rows G (64 x 64) are staged k-major in LDS; wave w
// multiplies actuator tile w & 1 over chunk columns [32 (w >> 1), 32 (w >> 1) + 32) with
// v_mfma_f32_32x32x2f32, accumulating in float32 across the group's chunks; the two column
// halves are added at the end. The next chunk's loads are issued before this chunk's products.
// Only rows [row0, row1) and columns [col0, col1) are visited (g_s is zero elsewhere: the
// pupil optic's amplitude window; or G is: the band of the Gaussian influence functions); T rows
// outside are not written.
template <bool SYNTH>
__global__ void __launch_bounds__(256) dm_grad_T(const float2 *E, const float2 *B, const float *G, int n, int na,
                                                 float kappa, const float *amp, const float *opd, int nd,
                                                 const float *pre, float inv_lambda, int row0, int row1,
                                                 int col0, int col1, float *tpart) {
  // g_s [column][row] and G [column][actuator] per chunk; after the last chunk the same memory
  // holds the column-half sums
  __shared__ union {
    struct {
      float As[kCJ][kRows + 1];
      float Bs[kCJ][kMaxAct + 1];
    } s;
    float red[2][kRows][kMaxAct / 2 + 1];
  } sm;
  using Chunk = GradChunk<SYNTH>;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int tile = w & 1, half = w >> 1;
  const int i0 = row0 + blockIdx.x * kRows;
  const int g = blockIdx.y;
  const int jbeg = col0 + g * kGroup, jend = min(col1, jbeg + kGroup);
  const int off = (n - nd) / 2;
  floatx16 acc = floatx16{0.f};
  Chunk cur;
  cur.load(E, B, G, n, na, amp, opd, nd, pre, i0, jbeg, tid);
  for (int j0 = jbeg; j0 < jend; j0 += kCJ) {
    const int cj = min(kCJ, jend - j0);
    const int c = tid & (kCJ - 1);
#pragma unroll
    for (int q = 0; q < Chunk::kPer; ++q) {
      const int r = (tid >> 6) + 4 * q;
      const int i = i0 + r, j = j0 + c;
      float2 e2 = cur.ev[q];
      bool in = i < row1 && c < cj;
      if constexpr (SYNTH) {
        const bool win = unsigned(i - off) < unsigned(nd) && unsigned(j - off) < unsigned(nd);
        float sn, cs;
        sincos_turns((2.f * cur.ws[q] + cur.wo[q]) * inv_lambda, &sn, &cs);
        e2 = make_float2(cur.wa[q] * cs, cur.wa[q] * sn);
        in = in && win;
      }
      // -2 kappa Im(E conj(B))
      sm.s.As[c][r] = in ? -2.f * kappa * (e2.y * cur.bv[q].x - e2.x * cur.bv[q].y) : 0.f;
    }
#pragma unroll
    for (int q = 0; q < Chunk::kGPer; ++q) {
      const int e = tid + 256 * q;
      const int cc = e / kMaxAct, a = e % kMaxAct;
      sm.s.Bs[cc][a] = (cc < cj && a < na) ? cur.gv[q] : 0.f;
    }
    __syncthreads();
    if (j0 + kCJ < jend) cur.load(E, B, G, n, na, amp, opd, nd, pre, i0, j0 + kCJ, tid);
    // A operand: lane supplies g_s[row lane % 32][k]; B operand: G[k][actuator lane % 32]
    const int kl = lane >> 5, rl = lane & 31;
#pragma unroll
    for (int k0 = 0; k0 < kCJ / 2; k0 += 8) {
#pragma unroll
      for (int kk = k0; kk < k0 + 8; kk += 2) {
        const int k = half * (kCJ / 2) + kk + kl;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sm.s.As[k][rl], sm.s.Bs[k][tile * 32 + rl], acc, 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }
  // accumulator r of lane l: row (r / 4) 8 + (l / 32) 4 + r % 4, actuator tile * 32 + l % 32
  if (half == 1) {
#pragma unroll
    for (int r = 0; r < 16; ++r) sm.red[tile][(r >> 2) * 8 + (lane >> 5) * 4 + (r & 3)][lane & 31] = acc[r];
  }
  __syncthreads();
  if (half == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
      const int i = i0 + row, a = tile * 32 + (lane & 31);
      if (i < row1 && a < na) tpart[(size_t(g) * n + i) * na + a] = acc[r] + sm.red[tile][row][lane & 31];
    }
  }
}

// T_sum[e] += sum over groups of tpart[group][e] (groups `stride` floats apart), in group
// order, for e < count
__global__ void __launch_bounds__(256) dm_grad_acc(const float *tpart, int groups, int count, size_t stride,
                                                   float *tsum) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < count; e += gridDim.x * 256) {
    float v = 0.f;
    for (int q = 0; q < groups; ++q) v += tpart[size_t(q) * stride + e];
    tsum[e] += v;
  }
}

// per block of kGRows rows: T rows (group shares added in group order), then the block's share
// of G^T T. All group shares of an element are loaded before they are added.
constexpr int kMaxGroups = 16;  // n <= 8192
__global__ void __launch_bounds__(256) dm_grad_G(const float *tpart, int groups, const float *G, int n, int na,
                                                 float *gpart) {
  __shared__ float Ts[kGRows][kMaxAct + 1];
  __shared__ float Gr[kGRows][kMaxAct + 1];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * kGRows;
  const int rows = min(kGRows, n - r0);
  for (int e = tid; e < kGRows * kMaxAct; e += 256) {
    const int r = e / kMaxAct, c = e % kMaxAct;
    const bool in = r < rows && c < na;
    const size_t o = size_t(r0 + min(r, rows - 1)) * na + min(c, na - 1);
    float part[kMaxGroups];
#pragma unroll
    for (int q = 0; q < kMaxGroups; ++q) part[q] = q < groups ? tpart[size_t(q) * n * na + o] : 0.f;
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < kMaxGroups; ++q) v += part[q];
    Ts[r][c] = in ? v : 0.f;
    Gr[r][c] = in ? G[o] : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < na * na; e += 256) {
    const int a = e / na, c = e % na;
    float v = 0.f;
#pragma unroll 8
    for (int r = 0; r < kGRows; ++r) v = fmaf(Gr[r][a], Ts[r][c], v);
    gpart[size_t(blockIdx.x) * na * na + e] = v;
  }
}

// gA[a][b] += sum over blocks of gpart[block][a][b]: each output's terms are split over the
// four waves of a block (wave q takes blocks q, q + 4, ...), and the four partial sums are added
// in wave order, so the result does not depend on scheduling
__global__ void __launch_bounds__(256) dm_grad_reduce(const float *part, int blocks, int nn, float *gA) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  float v = 0.f;
  if (e < nn)
    for (int s = q; s < blocks; s += 4) v += part[size_t(s) * nn + e];
  red[q][lane] = v;
  __syncthreads();
  if (q == 0 && e < nn) gA[e] += ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
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

// floats per DM surface map on an n grid (room for either layout)
size_t surf_stride(int n) { return std::max(size_t(n) * size_t(n), post_tiled_size(n)); }

// Workspace layout. Plain mode: one field plane E (and one adjoint plane B) of the largest
// grid, reused wavelength after wavelength. Batched mode: one E plane per wavelength (and one B
// plane per wavelength when the pupil DM needs the adjoint Fresnel step), so that the Fresnel
// steps of all wavelengths run in one launch per sweep. DM surface maps: one set per distinct
// grid edge in batched mode, one set (rebuilt on a change of edge) in plain mode.
struct Layout {
  std::vector<size_t> e, b;          // per wavelength (plain: all equal)
  std::vector<int> surf_n;           // distinct grid edges with a surface set
  std::vector<size_t> surf;          // offsets of those sets (n_dm maps each)
  size_t tpart, tsum, gpart, tdm, el, y1, eocc, edet, ydet, psf64, mft, total;
};

// Checkpoint layout (FR_TRAIN_FWD_SAVE writes it, FR_TRAIN_BWD reads it): per wavelength the
// field at the last DM plane (n^2 c64), then per wavelength the detector field (det^2 c64).
struct CkptLayout {
  std::vector<size_t> e, det;
  size_t total;
};

CkptLayout ckpt_layout(const fr_train_desc *d, int n_lambda, const int32_t *n_pad) {
  CkptLayout C;
  size_t off = 0;
  C.e.resize(n_lambda);
  C.det.resize(n_lambda);
  for (int j = 0; j < n_lambda; ++j) {
    C.e[j] = off;
    off += align256(size_t(n_pad[j]) * n_pad[j] * 8);
  }
  for (int j = 0; j < n_lambda; ++j) {
    C.det[j] = off;
    off += align256(size_t(d->det_m) * d->det_m * 8);
  }
  C.total = off;
  return C;
}

Layout layout(const fr_train_desc *d, int n_lambda, const int32_t *n_pad, int32_t mode) {
  Layout L;
  // the gradient is computed by FR_TRAIN_GRAD (with the forward) and FR_TRAIN_BWD (from the
  // checkpoint); with a checkpoint (FWD_SAVE or BWD) the E planes live in it, not here
  const bool grad = (mode & (FR_TRAIN_GRAD | FR_TRAIN_BWD)) != 0;
  const bool in_ckpt = (mode & (FR_TRAIN_FWD_SAVE | FR_TRAIN_BWD)) != 0;
  const bool batched = (mode & FR_TRAIN_BATCHED) != 0;
  int nmax = 0;
  for (int j = 0; j < n_lambda; ++j) nmax = std::max(nmax, int(n_pad[j]));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t n2max = size_t(nmax) * nmax;
  const size_t nd2 = size_t(d->n_d) * d->n_d;
  const bool b_per_lambda = batched && grad && d->n_dm == 2;
  L.e.assign(n_lambda, 0);
  L.b.assign(n_lambda, 0);
  if (in_ckpt) {
    // E planes and detector fields are in the checkpoint
  } else if (batched) {
    for (int j = 0; j < n_lambda; ++j) L.e[j] = take(size_t(n_pad[j]) * n_pad[j] * 8);
  } else {
    const size_t e0 = take(n2max * 8);
    for (int j = 0; j < n_lambda; ++j) L.e[j] = e0;
  }
  if (b_per_lambda) {
    for (int j = 0; j < n_lambda; ++j) L.b[j] = take(size_t(n_pad[j]) * n_pad[j] * 8);
  } else if (grad) {
    const size_t b0 = take(n2max * 8);
    for (int j = 0; j < n_lambda; ++j) L.b[j] = b0;
  }
  const size_t groups = size_t((nmax + kGroup - 1) / kGroup);
  const size_t ndm = size_t(std::max(d->n_dm, 1));
  L.tpart = grad ? take(groups * nmax * d->n_act * 4) : 0;
  L.tsum = grad ? take(ndm * nmax * d->n_act * 4) : 0;  // one T_sum per DM
  L.gpart = grad ? take(size_t((nmax + kGRows - 1) / kGRows) * d->n_act * d->n_act * 4) : 0;
  if (batched) {
    for (int j = 0; j < n_lambda; ++j)
      if (std::find(L.surf_n.begin(), L.surf_n.end(), int(n_pad[j])) == L.surf_n.end()) {
        L.surf_n.push_back(n_pad[j]);
        L.surf.push_back(take(ndm * surf_stride(n_pad[j]) * 4));
      }
  } else {
    L.surf_n.push_back(0);
    L.surf.push_back(take(ndm * surf_stride(nmax) * 4));
  }
  L.tdm = take(size_t(std::max(d->n_act, 1)) * nmax * 4);
  L.el = take(nd2 * 8);
  L.y1 = grad ? take(nd2 * 8) : 0;
  L.eocc = take(size_t(d->occ_m) * d->occ_m * 8);
  L.edet = take(size_t(d->det_m) * d->det_m * 8);
  L.ydet = grad ? take(size_t(d->det_m) * d->det_m * 8) : 0;
  L.psf64 = take(size_t(d->det_m) * d->det_m * 8);
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
  if (mode & ~(FR_TRAIN_NO_OCCULTER | FR_TRAIN_GRAD | FR_TRAIN_BATCHED | FR_TRAIN_GRAPH | FR_TRAIN_FWD_SAVE |
               FR_TRAIN_BWD))
    return FR_EINVAL;
  // one of: forward, forward + gradient, forward saving the checkpoint, gradient from it
  const int phase = mode & (FR_TRAIN_GRAD | FR_TRAIN_FWD_SAVE | FR_TRAIN_BWD);
  if (phase & (phase - 1)) return FR_EINVAL;
  if (d->n_d <= 0 || !(d->d_m > 0) || !d->pupil_amp) return FR_EINVAL;
  if (d->n_dm < 0 || d->n_dm > 2) return FR_EINVAL;
  if (d->n_dm > 0 && (d->n_act <= 0 || !d->dm_heights_m)) return FR_EINVAL;
  if (d->n_dm > 0 && d->n_act > kMaxAct) return FR_EUNSUPPORTED;
  for (int j = 0; j < n_lambda; ++j)
    if ((n_pad[j] + kGroup - 1) / kGroup > kMaxGroups) return FR_EUNSUPPORTED;
  if (!std::isfinite(d->z_m)) return FR_EINVAL;
  if (d->occ_m <= 0 || !(d->occ_du_c > 0) || d->det_m <= 0 || !(d->det_du_c > 0)) return FR_EINVAL;
  if (!(mode & FR_TRAIN_NO_OCCULTER) && !d->occ_mask) return FR_EINVAL;
  if (!d->lyot || !(d->lambda_c_m > 0)) return FR_EINVAL;
  if ((mode & (FR_TRAIN_GRAD | FR_TRAIN_FWD_SAVE | FR_TRAIN_BWD)) && d->n_dm == 0) return FR_EINVAL;
  for (int j = 0; j < n_lambda; ++j) {
    if (!(lam[j] > 0) || !std::isfinite(w[j])) return FR_EINVAL;
    if (n_pad[j] < d->n_d || ((n_pad[j] - d->n_d) & 1)) return FR_EINVAL;
    if (!plane_size_supported(n_pad[j])) return FR_EUNSUPPORTED;
  }
  return FR_OK;
}

}  // namespace

size_t train_workspace_bytes(const fr_train_desc *d, int32_t n_lambda, const int32_t *n_pad, int32_t mode) {
  if (!d || n_lambda <= 0 || !n_pad) return 0;
  for (int j = 0; j < n_lambda; ++j)
    if (n_pad[j] <= 0) return 0;
  if (d->n_d <= 0 || d->occ_m <= 0 || d->det_m <= 0) return 0;
  return layout(d, n_lambda, n_pad, mode).total;
}

// every argument check of propagate_train (nothing touched, nothing launched)
size_t train_ckpt_bytes(const fr_train_desc *d, int32_t n_lambda, const int32_t *n_pad) {
  if (!d || n_lambda <= 0 || !n_pad || d->det_m <= 0) return 0;
  for (int j = 0; j < n_lambda; ++j)
    if (n_pad[j] <= 0) return 0;
  return ckpt_layout(d, n_lambda, n_pad).total;
}

int check_call(Ctx *ctx, const fr_train_desc *d, int32_t n_lambda, const double *lam, const int32_t *n_pad,
               const float *weight, int32_t mode, const float *psf, const float *grad_psf,
               const float *grad_heights, const void *ckpt, size_t ckpt_bytes, const void *ws, size_t ws_bytes) {
  int st = check_desc(d, n_lambda, lam, n_pad, weight, mode);
  if (st != FR_OK) return st;
  const bool bwd = (mode & FR_TRAIN_BWD) != 0;
  if ((!bwd && !psf) || ((mode & (FR_TRAIN_GRAD | FR_TRAIN_BWD)) && (!grad_psf || !grad_heights)))
    return FR_EINVAL;
  if ((mode & (FR_TRAIN_FWD_SAVE | FR_TRAIN_BWD)) && (!ckpt || ckpt_bytes < train_ckpt_bytes(d, n_lambda, n_pad)))
    return FR_EWORKSPACE;
  if (!ws || ws_bytes < train_workspace_bytes(d, n_lambda, n_pad, mode)) return FR_EWORKSPACE;
  return ctx ? FR_OK : FR_EINVAL;
}

int train_run(Ctx *ctx, const fr_train_desc *d, int32_t n_lambda, const double *lam,
              const int32_t *n_pad, const float *weight, int32_t mode, float *psf,
              const float *grad_psf, float *grad_heights, void *ckpt, size_t ckpt_bytes, void *ws,
              size_t ws_bytes, hipStream_t s) {
  int st = check_call(ctx, d, n_lambda, lam, n_pad, weight, mode, psf, grad_psf, grad_heights, ckpt, ckpt_bytes,
                      ws, ws_bytes);
  if (st != FR_OK) return st;
  // fwd: this call runs the forward (every mode but FR_TRAIN_BWD); grad: it computes the gradient
  const bool fwd = !(mode & FR_TRAIN_BWD);
  const bool grad = (mode & (FR_TRAIN_GRAD | FR_TRAIN_BWD)) != 0;
  const bool in_ckpt = (mode & (FR_TRAIN_FWD_SAVE | FR_TRAIN_BWD)) != 0;
  const bool occ = !(mode & FR_TRAIN_NO_OCCULTER);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return record_hip(e);

  const bool batched = (mode & FR_TRAIN_BATCHED) != 0;
  const Layout L = layout(d, n_lambda, n_pad, mode);
  char *base = static_cast<char *>(ws);
  auto c64at = [&](size_t o) { return reinterpret_cast<float2 *>(base + o); };
  const CkptLayout CK = ckpt_layout(d, n_lambda, n_pad);
  char *cbase = static_cast<char *>(ckpt);
  // the field at the last DM plane and the detector field of wavelength j: in the checkpoint
  // (FWD_SAVE, BWD) or in the workspace (one detector field reused wavelength after wavelength)
  auto e_of = [&](int j) { return in_ckpt ? reinterpret_cast<float2 *>(cbase + CK.e[j]) : c64at(L.e[j]); };
  auto det_of = [&](int j) { return in_ckpt ? reinterpret_cast<float2 *>(cbase + CK.det[j]) : c64at(L.edet); };
  float *GPART = grad ? reinterpret_cast<float *>(base + L.gpart) : nullptr;
  float *TPART = grad ? reinterpret_cast<float *>(base + L.tpart) : nullptr;
  float *TSUM = grad ? reinterpret_cast<float *>(base + L.tsum) : nullptr;
  float *TDM = reinterpret_cast<float *>(base + L.tdm);
  float2 *EL = c64at(L.el);
  float2 *Y1 = grad ? c64at(L.y1) : nullptr;
  float2 *EOCC = c64at(L.eocc);
  float2 *YDET = grad ? c64at(L.ydet) : nullptr;
  void *MWS = base + L.mft;
  double *PSF64 = reinterpret_cast<double *>(base + L.psf64);
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

  // DM surfaces s = G A G^T on an n grid (a8): TDM (na x n) = A G^T ; SURF_k (n x n) = G TDM.
  // Rows and columns of G outside its band [lo, hi) are exactly 0, and so is the surface there:
  // the map is cleared, and the product formed on the band only (the same sums where it is).
  auto surfaces = [&](int n, float *surf) -> int {
    const float *G = nullptr;
    FR_TRY(ctx->dm_influence(n, nd, na, s, &G));
    int lo = 0, hi = n;
    ctx->dm_band(n, nd, na, &lo, &hi);
    if (hi <= lo) lo = 0, hi = n;
    const int nb = hi - lo;
    for (int k = 0; k < ndm; ++k) {
      RGemm g1{na, n, na, d->dm_heights_m + size_t(k) * na * na, na, 0, G, na, 1, TDM, n, 1.f, 0.f, 0, 0, 0};
      FR_TRY_HIP(rgemm(g1, s, hook));
      float *sk = surf + size_t(k) * surf_stride(n);
      // the DM after the step is applied by the column sweep: 4-column tiles
      const int tiled = k == ndm - 1 ? 1 : 0;
      if (nb < n) FR_TRY_HIP(launch1d(fill_f32, surf_stride(n), s, hook, "fill", sk, surf_stride(n), 0.f));
      RGemm g2{nb, nb, na, G + size_t(lo) * na, na, 0, TDM + lo, n, 0, tiled ? sk : sk + size_t(lo) * n + lo, n,
               1.f, 0.f, tiled, n, lo};
      FR_TRY_HIP(rgemm(g2, s, hook));
    }
    return FR_OK;
  };
  auto surf_of = [&](int j) -> float * {
    if (!batched) return reinterpret_cast<float *>(base + L.surf[0]);
    const size_t i = std::find(L.surf_n.begin(), L.surf_n.end(), int(n_pad[j])) - L.surf_n.begin();
    return reinterpret_cast<float *>(base + L.surf[i]);
  };

  // forward Fresnel plane of wavelength j: pupil optic (and DM1) synthesised in the row
  // prologue, step z, last-DM phasor in the column epilogue (a1, a2)
  auto fwd_plane = [&](int j, PlaneArgs *pa) -> int {
    const int n = n_pad[j];
    const float *surf = surf_of(j);
    std::memset(pa, 0, sizeof *pa);
    pa->field = e_of(j);
    pa->n = n;
    pa->amp = d->pupil_amp;
    pa->opd = d->pupil_opd_m;
    pa->win = nd;
    pa->pre_surf = ndm == 2 ? surf : nullptr;
    pa->post_surf = ndm >= 1 ? surf + size_t(ndm - 1) * surf_stride(n) : nullptr;
    // the surface G A G^T is exactly 0 outside the band where G has nonzero entries
    if (ndm >= 1) ctx->dm_band(n, nd, na, &pa->post_lo, &pa->post_hi);
    pa->inv_lambda = float(1.0 / lam[j]);
    pa->flags = kSourceOptic;
    return ctx->transfer(n, dx, lam[j], d->z_m, s, &pa->h);
  };
  // adjoint Fresnel plane of wavelength j on B_j: conj(last-DM phasor), then AS_{-z}
  auto adj_plane = [&](int j, PlaneArgs *pb) -> int {
    const int n = n_pad[j];
    std::memset(pb, 0, sizeof *pb);
    pb->field = c64at(L.b[j]);
    pb->n = n;
    pb->post_surf = surf_of(j) + size_t(ndm - 1) * surf_stride(n);
    ctx->dm_band(n, nd, na, &pb->post_lo, &pb->post_hi);
    pb->inv_lambda = float(1.0 / lam[j]);
    // B1 is read only inside the pupil window (the pupil DM's gradient)
    pb->win = nd;
    pb->flags = FR_ADJOINT | kWindowRowsOnly;
    return ctx->transfer(n, dx, lam[j], d->z_m, s, &pb->h);
  };

  // occulter, Babinet subtraction, Lyot stop, detector; psf += w_j |Ed|^2 (a3, a4, a5)
  auto focal_chain = [&](int j) -> int {
    const int n = n_pad[j];
    const float2 *E = e_of(j);
    const double du_occ = d->occ_du_c * d->lambda_c_m / lam[j];
    const double du_det = d->det_du_c * d->lambda_c_m / lam[j];
    const int off = (n - nd) / 2;
    const float2 *Ewin = E + size_t(off) * n + off;
    if (occ) {
      MftOut o;
      o.out = EOCC;
      o.ld_out = d->occ_m;
      o.mask = d->occ_mask;
      FR_TRY(mft_forward_impl(ctx, E, n, n, d->occ_m, double(nd), du_occ, o, MWS, s));
      FR_TRY(mft_adjoint_impl(ctx, EOCC, d->occ_m, d->occ_m, EL, nd, nd, double(nd), du_occ,
                              -1.f, 1.f, Ewin, n, d->lyot, MWS, s));
    } else {
      FR_TRY_HIP(launch1d(window_mask, size_t(nd) * nd, s, hook, "window_mask", E, n, nd, d->lyot, EL));
    }
    MftOut o;
    o.out = det_of(j);
    o.ld_out = d->det_m;
    o.intensity = PSF64;
    o.weight = weight[j];
    return mft_forward_impl(ctx, EL, nd, nd, d->det_m, double(nd), du_det, o, MWS, s);
  };

  // dL/dA_k += G^T g_s G with g_s = -2 kappa Im(E conj(B)) (E stored, or the pupil optic
  // synthesised from amp/opd/pre when E == null): the wavelength's T goes into DM k's T_sum; the
  // projection G^T T_sum into gA_k runs when the grid edge changes and at the end of the call
  int nmax = 0;
  for (int j = 0; j < n_lambda; ++j) nmax = std::max(nmax, int(n_pad[j]));
  int sum_n[2] = {-1, -1};  // grid edge whose T each DM's T_sum holds (-1: empty)
  auto flush = [&](int k) -> int {
    const int n = sum_n[k];
    if (n < 0) return FR_OK;
    const float *G = nullptr;
    FR_TRY(ctx->dm_influence(n, nd, na, s, &G));
    const int gblocks = (n + kGRows - 1) / kGRows;
    hook(s, "dm_grad_G", n, 0);
    hipLaunchKernelGGL(dm_grad_G, dim3(gblocks), dim3(256), 0, s, (const float *)(TSUM + size_t(k) * nmax * na), 1,
                       G, n, na, GPART);
    FR_TRY_HIP(hipGetLastError());
    hook(s, "dm_grad_G", n, 1);
    hook(s, "dm_grad_reduce", n, 0);
    hipLaunchKernelGGL(dm_grad_reduce, dim3((na * na + 63) / 64), dim3(256), 0, s, (const float *)GPART, gblocks,
                       na * na, grad_heights + size_t(k) * na * na);
    FR_TRY_HIP(hipGetLastError());
    hook(s, "dm_grad_reduce", n, 1);
    sum_n[k] = -1;
    return FR_OK;
  };
  auto dm_grad = [&](int j, int k, const float2 *E, const float2 *B, const float *pre) -> int {
    const int n = n_pad[j];
    const float *G = nullptr;
    FR_TRY(ctx->dm_influence(n, nd, na, s, &G));
    // The pupil optic (E == null) is zero outside its nd x nd window, and so is g_s there. For a
    // stored plane the rows and columns outside the band where G has a nonzero float32 entry
    // add exact zeros to T and to G^T T: they are skipped, the columns in whole kGroup groups
    // (the groups that remain are the same groups, added in the same order: the same sums).
    int r0 = (n - nd) / 2, r1 = r0 + nd, c0 = r0, c1 = r1;
    if (E) {
      int blo = 0, bhi = n;
      ctx->dm_band(n, nd, na, &blo, &bhi);
      if (bhi <= blo) blo = 0, bhi = n;
      r0 = blo, r1 = bhi;
      c0 = blo / kGroup * kGroup, c1 = std::min(n, (bhi + kGroup - 1) / kGroup * kGroup);
    }
    const int strips = (r1 - r0 + kRows - 1) / kRows, groups = (c1 - c0 + kGroup - 1) / kGroup;
    const int tn = n * na;
    float *T = TSUM + size_t(k) * nmax * na;
    if (sum_n[k] != n) {
      FR_TRY(flush(k));
      FR_TRY_HIP(launch1d(fill_f32, size_t(tn), s, hook, "fill", T, size_t(tn), 0.f));
      sum_n[k] = n;
    }
    const float kappa = float(4.0 * M_PI / lam[j]);
    const char *tname = E ? "dm_grad_T" : "dm_grad_T_pupil";
    hook(s, tname, n, 0);
    if (E)
      hipLaunchKernelGGL(dm_grad_T<false>, dim3(strips, groups), dim3(256), 0, s, E, B, G, n, na, kappa,
                         d->pupil_amp, d->pupil_opd_m, nd, pre, float(1.0 / lam[j]), r0, r1, c0, c1, TPART);
    else
      hipLaunchKernelGGL(dm_grad_T<true>, dim3(strips, groups), dim3(256), 0, s, E, B, G, n, na, kappa,
                         d->pupil_amp, d->pupil_opd_m, nd, pre, float(1.0 / lam[j]), r0, r1, c0, c1, TPART);
    FR_TRY_HIP(hipGetLastError());
    hook(s, tname, n, 1);
    // T rows outside [r0, r1) keep what they hold (zero from the fill: those rows of T are zero,
    // or meet only zero rows of G in the projection)
    FR_TRY_HIP(launch1d(dm_grad_acc, size_t(r1 - r0) * na, s, hook, "dm_grad_acc",
                        (const float *)(TPART + size_t(r0) * na), groups, (r1 - r0) * na, size_t(tn),
                        T + size_t(r0) * na));
    return FR_OK;
  };

  // backward of the focal chain to the last DM: B_j = dL/dconj(E_dm); then the last DM's
  // gradient g_s = -2 kappa Im(E_dm conj(B)) (a7)
  auto back_to_last_dm = [&](int j) -> int {
    const int n = n_pad[j];
    const size_t n2 = size_t(n) * n;
    const float2 *E = e_of(j);
    float2 *B = c64at(L.b[j]);
    const double du_occ = d->occ_du_c * d->lambda_c_m / lam[j];
    const double du_det = d->det_du_c * d->lambda_c_m / lam[j];
    FR_TRY_HIP(launch1d(scale_by_grad, det2, s, hook, "scale_by_grad", grad_psf, weight[j],
                        (const float2 *)det_of(j), YDET, det2));
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
    return dm_grad(j, ndm - 1, E, B, nullptr);
  };
  // pupil DM (n_dm == 2), after B_j went back through the adjoint step:
  // g_s1 = -2 kappa Im(E_dm1 conj(B1)), E_dm1 = pupil optic * DM1 phasor synthesised again
  auto back_to_pupil_dm = [&](int j) -> int {
    return dm_grad(j, 0, nullptr, c64at(L.b[j]), surf_of(j));
  };

  if (fwd) FR_TRY_HIP(launch1d(fill_f64, det2, s, hook, "fill", PSF64, det2));
  if (grad) {
    const size_t ng = size_t(ndm) * na * na;
    FR_TRY_HIP(launch1d(fill_f32, ng, s, hook, "fill", grad_heights, ng, 0.f));
  }

  if (!batched) {
    // plain: wavelength after wavelength, one plane at a time
    int surf_n = -1;
    for (int j = 0; j < n_lambda; ++j) {
      if (ndm > 0 && surf_n != n_pad[j]) {
        FR_TRY(surfaces(n_pad[j], surf_of(j)));
        surf_n = n_pad[j];
      }
      if (fwd) {
        PlaneArgs pa;
        FR_TRY(fwd_plane(j, &pa));
        FR_TRY(run_planes(ctx, &pa, 1, s));
        FR_TRY(focal_chain(j));
      }
      if (!grad) continue;
      FR_TRY(back_to_last_dm(j));
      if (ndm == 2) {
        PlaneArgs pb;
        FR_TRY(adj_plane(j, &pb));
        FR_TRY(run_planes(ctx, &pb, 1, s));
        FR_TRY(back_to_pupil_dm(j));
      }
    }
  } else {
    // batched: wavelengths in groups whose planes fit the last-level cache together (one 4096^2
    // plane, several smaller ones); each group's Fresnel planes in one launch per sweep, then
    // its focal chains while its planes are still cached. Sums still run in wavelength order.
    if (ndm > 0)
      for (size_t i = 0; i < L.surf_n.size(); ++i)
        FR_TRY(surfaces(L.surf_n[i], reinterpret_cast<float *>(base + L.surf[i])));
    constexpr size_t kGroupBytes = size_t(160) << 20;
    std::vector<PlaneArgs> planes(n_lambda);
    for (int g0 = 0; g0 < n_lambda;) {
      int g1 = g0;
      size_t bytes = 0;
      while (g1 < n_lambda) {
        const size_t b = size_t(n_pad[g1]) * n_pad[g1] * sizeof(float2);
        if (g1 > g0 && bytes + b > kGroupBytes) break;
        bytes += b;
        ++g1;
      }
      if (fwd) {
        for (int j = g0; j < g1; ++j) FR_TRY(fwd_plane(j, &planes[j]));
        FR_TRY(run_planes(ctx, planes.data() + g0, g1 - g0, s));
      }
      for (int j = g0; j < g1; ++j) {
        if (fwd) FR_TRY(focal_chain(j));
        if (grad) FR_TRY(back_to_last_dm(j));
      }
      if (grad && ndm == 2) {
        for (int j = g0; j < g1; ++j) FR_TRY(adj_plane(j, &planes[j]));
        FR_TRY(run_planes(ctx, planes.data() + g0, g1 - g0, s));
        for (int j = g0; j < g1; ++j) FR_TRY(back_to_pupil_dm(j));
      }
      g0 = g1;
    }
  }
  if (grad)
    for (int k = 0; k < ndm; ++k) FR_TRY(flush(k));
  if (fwd) FR_TRY_HIP(launch1d(to_f32, det2, s, hook, "psf_to_f32", (const double *)PSF64, psf, det2));
#undef FR_TRY
#undef FR_TRY_HIP
  return FR_OK;
}


// Graph mode: the whole call (every launch of every wavelength) as one instantiated graph,
// replayed when a later call bakes in the same argument bytes. The first call with new
// arguments runs eagerly (which also builds every table the graph reads), then captures the
// same launch sequence on the context's own stream.
std::string graph_key(const fr_train_desc *d, int32_t n_lambda, const double *lam, const int32_t *n_pad,
                      const float *w, int32_t mode, const void *psf, const void *gpsf, const void *gh,
                      const void *ckpt, size_t ckpt_bytes, const void *ws, size_t ws_bytes, hipStream_t s) {
  std::string k("train");
  auto put = [&](const void *p, size_t b) { k.append(static_cast<const char *>(p), b); };
  put(d, sizeof *d);
  put(&n_lambda, sizeof n_lambda);
  put(lam, sizeof(double) * n_lambda);
  put(n_pad, sizeof(int32_t) * n_lambda);
  put(w, sizeof(float) * n_lambda);
  put(&mode, sizeof mode);
  const void *ptrs[6] = {psf, gpsf, gh, ckpt, ws, s};
  put(ptrs, sizeof ptrs);
  put(&ckpt_bytes, sizeof ckpt_bytes);
  put(&ws_bytes, sizeof ws_bytes);
  return k;
}

int train_call(Ctx *ctx, const fr_train_desc *d, int32_t n_lambda, const double *lam,
               const int32_t *n_pad, const float *w, int32_t mode, float *psf, const float *gpsf,
               float *gh, void *ckpt, size_t ckpt_bytes, void *ws, size_t ws_bytes, hipStream_t s) {
  int st = check_call(ctx, d, n_lambda, lam, n_pad, w, mode, psf, gpsf, gh, ckpt, ckpt_bytes, ws, ws_bytes);
  if (st != FR_OK) return st;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return record_hip(e);
  // the cache is trimmed here, once per call (the recording run below must not trim it)
  if ((st = ctx->begin_call()) != FR_OK) return st;
  if (!(mode & FR_TRAIN_GRAPH))
    return train_run(ctx, d, n_lambda, lam, n_pad, w, mode, psf, gpsf, gh, ckpt, ckpt_bytes, ws, ws_bytes, s);
  const std::string key = graph_key(d, n_lambda, lam, n_pad, w, mode, psf, gpsf, gh, ckpt, ckpt_bytes, ws,
                                    ws_bytes, s);
  return ctx->graph_call(key, s, "train_graph", n_lambda, [&](hipStream_t cs) {
    return train_run(ctx, d, n_lambda, lam, n_pad, w, mode, psf, gpsf, gh, ckpt, ckpt_bytes, ws, ws_bytes, cs);
  });
}

}  // namespace fr

extern "C" {

size_t propagate_train_workspace_bytes(const fr_train_desc *desc, int32_t n_lambda,
                                       const int32_t *n_pad, int32_t mode) {
  return fr::train_workspace_bytes(desc, n_lambda, n_pad, mode);
}

size_t propagate_train_ckpt_bytes(const fr_train_desc *desc, int32_t n_lambda, const int32_t *n_pad) {
  return fr::train_ckpt_bytes(desc, n_lambda, n_pad);
}

int propagate_train(fr_ctx *ctx, const fr_train_desc *desc, int32_t n_lambda, const double *lambda_m,
                    const int32_t *n_pad, const float *weight, int32_t mode, float *psf,
                    const float *grad_psf, float *grad_heights, void *ckpt, size_t ckpt_bytes, void *ws,
                    size_t ws_bytes, void *stream) {
  return fr::train_call(reinterpret_cast<fr::Ctx *>(ctx), desc, n_lambda, lambda_m, n_pad, weight, mode,
                        psf, grad_psf, grad_heights, ckpt, ckpt_bytes, ws, ws_bytes,
                        static_cast<hipStream_t>(stream));
}
}
