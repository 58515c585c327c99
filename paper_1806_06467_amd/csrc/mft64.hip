// The matrix Fourier transform in float64 (Sec. 1.1, after Soummer et al.; Sec. 2.3 for the
// precision the paper benchmarks): out = (du / n_d) W in W^T and its adjoint
// (du / n_d) W^H in conj(W), as two complex GEMMs in float64 on the matrix cores (on gfx950 their
// dense float64 peak, 78.6 TFLOP/s, equals the vector units'; the matrix-core tile reads each
// operand from LDS once per 16 x 16 x 4 product instead of once per multiply-add, and leaves the
// vector units free for the loads).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fresnel.h"
#include "fr_runtime.h"

namespace fr {
namespace {

struct z64 {
  double x, y;
};

constexpr int kDepth = 16;

// C[i][j] = s sum_k A(i, k) B(k, j). A(i, k) = a[i lda + k] (or a[k lda + i] when TA), conjugated
// when CA; B(k, j) = b[k ldb + j] (or b[j ldb + k] when TB), conjugated when CB. Split K:
// blockIdx.z takes k in [z kc, (z + 1) kc) and writes its partial C at c + z c_split. A may be
// the ordered sum of sa partial matrices a_split apart (the previous product's split-K slices).
// On the float64 matrix cores: a 256-thread block forms a 64 x 64 tile of C from 16-deep slices of
// A and B staged in LDS (the next slice read into registers while the current one is
// multiplied), each wave a 32 x 32 piece as 2 x 2 blocks of 16 x 16, every complex k-step of 4 as
// four real v_mfma_f64_16x16x4 per block (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br). Fragment
// layouts (checked on gfx950 with one-hot operands): lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16] of the 16 x 4 and 4 x 16 operands, and item r of the result
// D[4 r + l / 16][l % 16].
typedef double d4 __attribute__((ext_vector_type(4)));

// At most three waves per SIMD (170 registers; left alone the compiler takes 144 + 64
// accumulation registers, which allow two): 0.61 ms against 0.66 ms for the occulter MFT's
// first product; four waves spill and run slower.
template <bool TA, bool CA, bool TB, bool CB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) zgemm_mfma_kernel(const z64 *__restrict__ a, int lda,
                                                         const z64 *__restrict__ b, int ldb, z64 *__restrict__ c,
                                                         int ldc, int M, int N, int K, double s, int kc,
                                                         size_t c_split, int sa, size_t a_split) {
  constexpr int TM = 64, TN = 64, R = TM * kDepth / 256, Q = TN * kDepth / 256;
  __shared__ z64 As[kDepth][TM + 1];
  __shared__ z64 Bs[kDepth][TN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) cr[ib][jb] = ci[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
  const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
  c += blockIdx.z * c_split;
  const int fr = lane & 15, fk = lane >> 4;  // fragment row (column) and k within a 4-deep step
  // the next slice's operands are read into registers while the current one is multiplied
  z64 va[R], vb[Q];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = tid + 256 * r;
      int i, k;
      if constexpr (TA) { i = e % TM; k = e / TM; } else { k = e % kDepth; i = e / kDepth; }
      va[r] = {0.0, 0.0};
      if (i0 + i < M && k0 + k < kend) {
        const size_t at = TA ? size_t(k0 + k) * lda + (i0 + i) : size_t(i0 + i) * lda + (k0 + k);
        va[r] = a[at];
        for (int p = 1; p < sa; ++p) {
          const z64 w = a[p * a_split + at];
          va[r].x += w.x;
          va[r].y += w.y;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q;
      int j, kb;
      if constexpr (TB) { kb = e % kDepth; j = e / kDepth; } else { j = e % TN; kb = e / TN; }
      vb[q] = {0.0, 0.0};
      if (j0 + j < N && k0 + kb < kend)
        vb[q] = TB ? b[size_t(j0 + j) * ldb + (k0 + kb)] : b[size_t(k0 + kb) * ldb + (j0 + j)];
    }
  };
  auto put = [&] {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = tid + 256 * r;
      int i, k;
      if constexpr (TA) { i = e % TM; k = e / TM; } else { k = e % kDepth; i = e / kDepth; }
      z64 v = va[r];
      if constexpr (CA) v.y = -v.y;
      As[k][i] = v;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = tid + 256 * q;
      int j, kb;
      if constexpr (TB) { kb = e % kDepth; j = e / kDepth; } else { j = e % TN; kb = e / TN; }
      z64 v = vb[q];
      if constexpr (CB) v.y = -v.y;
      Bs[kb][j] = v;
    }
  };
  if (kbeg < kend) {
    fetch(kbeg);
    put();
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kDepth) {
    const bool more = k0 + kDepth < kend;
    if (more) fetch(k0 + kDepth);
#pragma unroll
    for (int k4 = 0; k4 < kDepth; k4 += 4) {
      double ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) {
        const z64 v = As[k4 + fk][wm * 32 + ib * 16 + fr];
        ar[ib] = v.x;
        ai[ib] = v.y;
        nai[ib] = -v.y;
      }
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const z64 v = Bs[k4 + fk][wn * 32 + jb * 16 + fr];
        br[jb] = v.x;
        bi[jb] = v.y;
      }
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
          cr[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ib], br[jb], cr[ib][jb], 0, 0, 0);
          ci[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ib], bi[jb], ci[ib][jb], 0, 0, 0);
        }
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
          cr[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[ib], bi[jb], cr[ib][jb], 0, 0, 0);
          ci[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[ib], br[jb], ci[ib][jb], 0, 0, 0);
        }
    }
    __syncthreads();
    if (more) put();
    __syncthreads();
  }
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int j = j0 + wn * 32 + jb * 16 + fr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + ib * 16 + 4 * r + fk;
        if (i < M && j < N) c[size_t(i) * ldc + j] = {s * cr[ib][jb][r], s * ci[ib][jb][r]};
      }
    }
}

// most partials zsum_kernel adds
constexpr int kMaxZsum = 32;

// split-K factors of the forward transform's two products (m x n x n, then m x m x n): 4 and 32
// where their 64 x 64 tiles alone would give a launch fewer than 4 blocks per compute unit and
// the pupil is large
int f64_split(int n, int m) {
  const long tiles = long((n + 63) / 64) * long((m + 63) / 64);
  return tiles < 1024 && n >= 1024 ? 4 : 1;
}
int f64_split2(int n, int m) {
  const long tiles = long((m + 63) / 64) * long((m + 63) / 64);
  return tiles < 1024 && n >= 1024 ? kMaxZsum : 1;
}

// out[i] = s sum_p part[p stride + i], the partials added in order (np <= kMaxZsum; every
// partial's load is issued before the first addition)
__global__ void __launch_bounds__(256) zsum_kernel(const z64 *__restrict__ part, size_t stride, int np,
                                                   z64 *__restrict__ out, size_t count, double s) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= count) return;
  z64 v[kMaxZsum];
#pragma unroll
  for (int p = 0; p < kMaxZsum; ++p)
    if (p < np) v[p] = part[p * stride + i];
  z64 acc = v[0];
#pragma unroll
  for (int p = 1; p < kMaxZsum; ++p)
    if (p < np) {
      acc.x += v[p].x;
      acc.y += v[p].y;
    }
  out[i] = {s * acc.x, s * acc.y};
}

// part[i] = sum_p part[p stride + i], the partials added in order (in place into the first)
__global__ void __launch_bounds__(256) zsum_inplace_kernel(z64 *part, size_t stride, int np, size_t count) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= count) return;
  z64 acc = part[i];
  for (int p = 1; p < np; ++p) {
    const z64 v = part[p * stride + i];
    acc.x += v.x;
    acc.y += v.y;
  }
  part[i] = acc;
}

template <bool TA, bool CA, bool TB, bool CB>
hipError_t zgemm(const z64 *a, int lda, const z64 *b, int ldb, z64 *c, int ldc, int M, int N, int K, double s,
                 hipStream_t st, const LaunchHook &hook, const char *name, int split = 1, int sa = 1,
                 size_t a_split = 0) {
  hook(st, name, 1, 0);
  const int kc = ((K + split - 1) / split + kDepth - 1) / kDepth * kDepth;
  const size_t c_split = size_t(M) * size_t(ldc);
  hipLaunchKernelGGL((zgemm_mfma_kernel<TA, CA, TB, CB>), dim3((N + 63) / 64, (M + 63) / 64, split), dim3(256), 0,
                     st, a, lda, b, ldb, c, ldc, M, N, K, s, kc, c_split, sa, a_split);
  hipError_t e = hipGetLastError();
  hook(st, name, 1, 1);
  return e;
}

uint64_t dbits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof u);
  return u;
}

// W[k][x] = exp(-2 pi i (k - m/2)(x - n/2) du / n_d), m x n float64 pairs; the index product is
// an exact integer, its turns reduced to [-1/2, 1/2] before the exponential
int mft64_matrix(Ctx *ctx, int m, int n, double n_d, double du, hipStream_t s, const z64 **out) {
  const TableKey key{kMft64, m, uint64_t(n), dbits(n_d), dbits(du), 0};
  if (auto it = ctx->tables.find(key); it != ctx->tables.end()) {
    *out = static_cast<const z64 *>(it->second);
    return FR_OK;
  }
  std::vector<double> w(size_t(2) * m * n);
  const double r = du / n_d;
  for (int k = 0; k < m; ++k)
    for (int x = 0; x < n; ++x) {
      const double p = double(int64_t(k - m / 2) * int64_t(x - n / 2));
      double t = p * r;
      t -= std::rint(t);
      w[2 * (size_t(k) * n + x)] = std::cos(2.0 * M_PI * t);
      w[2 * (size_t(k) * n + x) + 1] = -std::sin(2.0 * M_PI * t);
    }
  void *d = nullptr;
  const int st = ctx->upload(key, w.data(), w.size() * sizeof(double), s, &d);
  *out = static_cast<const z64 *>(d);
  return st;
}

}  // namespace
}  // namespace fr

extern "C" size_t mft_f64_workspace_bytes(int32_t n_pupil, int32_t m_focal) {
  if (n_pupil <= 0 || m_focal <= 0) return 0;
  const int s2 = fr::f64_split2(n_pupil, m_focal);
  return sizeof(fr_c128) * (size_t(n_pupil) * size_t(m_focal) * size_t(fr::f64_split(n_pupil, m_focal)) +
                            (s2 > 1 ? size_t(m_focal) * size_t(m_focal) * size_t(s2) : 0));
}

extern "C" int mft_f64(fr_ctx *ctx_, const fr_c128 *in, fr_c128 *out, int32_t n_pupil, int32_t m_focal,
                       double n_d, double du, int32_t flags, fr_c128 *ws, size_t ws_bytes, void *stream) {
  if (!in || !out || !ws || n_pupil <= 0 || m_focal <= 0 || (flags & ~FR_ADJOINT)) return FR_EINVAL;
  if (!(n_d > 0) || !std::isfinite(n_d) || !(du > 0) || !std::isfinite(du)) return FR_EINVAL;
  if (ws_bytes < mft_f64_workspace_bytes(n_pupil, m_focal)) return FR_EWORKSPACE;
  fr::Ctx *ctx = reinterpret_cast<fr::Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  const int n = n_pupil, m = m_focal;
  const fr::z64 *w;
  int st = fr::mft64_matrix(ctx, m, n, n_d, du, s, &w);
  if (st != FR_OK) return st;
  const auto *src = reinterpret_cast<const fr::z64 *>(in);
  auto *dst = reinterpret_cast<fr::z64 *>(out);
  auto *t = reinterpret_cast<fr::z64 *>(ws);
  const double scale = du / n_d;
  const fr::LaunchHook hook = ctx->hook();
  if (!(flags & FR_ADJOINT)) {
    // T = W in (m x n, in `split` partial sums over k, added in order into the first by
    // zsum_kernel); out = scale T W^T (m x m), that product in turn split over k into `split2`
    // partials after T in the workspace, added in order by zsum_kernel. (Adding T's partials as
    // the second product reads them made each of its column tiles read all of them: 0.78 ms
    // against 0.71 ms for the forward transform at the occulter shape.)
    const int split = fr::f64_split(n, m), split2 = fr::f64_split2(n, m);
    const size_t part = size_t(m) * size_t(n), part2 = size_t(m) * size_t(m);
    e = fr::zgemm<false, false, false, false>(w, n, src, n, t, n, m, n, n, 1.0, s, hook, "zgemm_mft64_1", split);
    if (e == hipSuccess && split > 1) {
      hook(s, "zsum_mft64_t", 1, 0);
      hipLaunchKernelGGL(fr::zsum_inplace_kernel, dim3(unsigned((part + 255) / 256)), dim3(256), 0, s, t, part,
                         split, part);
      e = hipGetLastError();
      hook(s, "zsum_mft64_t", 1, 1);
    }
    if (e == hipSuccess && split2 == 1)
      e = fr::zgemm<false, false, true, false>(t, n, w, n, dst, m, m, m, n, scale, s, hook, "zgemm_mft64_2");
    if (e == hipSuccess && split2 > 1) {
      fr::z64 *t2 = t + part * split;
      e = fr::zgemm<false, false, true, false>(t, n, w, n, t2, m, m, m, n, 1.0, s, hook, "zgemm_mft64_2", split2);
      if (e == hipSuccess) {
        hook(s, "zsum_mft64", 1, 0);
        hipLaunchKernelGGL(fr::zsum_kernel, dim3(unsigned((part2 + 255) / 256)), dim3(256), 0, s, t2, part2, split2,
                           dst, part2, scale);
        e = hipGetLastError();
        hook(s, "zsum_mft64", 1, 1);
      }
    }
  } else {
    // T = W^H in (n x m); out = scale T conj(W) (n x n). (T in split-K partials would be summed
    // by every column tile of the second product: 0.99 ms against 0.62 ms for it at the occulter
    // shape.)
    e = fr::zgemm<true, true, false, false>(w, n, src, m, t, m, n, m, m, 1.0, s, hook, "zgemm_mft64_adj_1");
    if (e == hipSuccess)
      e = fr::zgemm<false, false, false, true>(t, m, w, n, dst, n, n, n, m, scale, s, hook, "zgemm_mft64_adj_2");
  }
  if (e != hipSuccess) return fr::record_hip(e);
  return FR_OK;
}
