// Matrix Fourier transform as two complex GEMMs on FP32 MFMA (Sec. 1.1: the semi-analytic
// coronagraph of Soummer et al. uses matrix DFTs; Sec. 2.3: the sin/cos arrays of that
// matrix DFT). Unlike the FFT sweeps this step really is a dense contraction, so it runs on
// the matrix cores.
//
// Complex product with real MFMA: per complex k-step, Cr += Ar Br - Ai Bi and
// Ci += Ar Bi + Ai Br (four v_mfma_f32_32x32x2f32, A/B fragments from LDS).
// Block tile 64 x 64, four waves in 2 x 2, each wave one 32 x 32 real and imaginary
// accumulator per 16-deep k tile, added into float64 totals (the long Fourier sums of the
// coronagraph cancel to tiny values in the dark hole, so their rounding must not grow with K).
// Operands may be transposed and/or conjugated on load. Small outputs with
// long K are split over K; the partial sums go to the workspace and one epilogue kernel adds
// them in a fixed order (deterministic), applies alpha, beta and the mask.
#include <hip/hip_runtime.h>

#include "fr_internal.h"

namespace fr {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int PAD = 4;

struct GemmParams {
  CGemmArgs a;
  int split;        // number of K slices (gridDim.z)
  int k_per_split;  // multiple of BK
  float2 *partial;  // split x M x N when split > 1
};

// result (i, j) = alpha acc + beta Cin, times mask; written to C and/or accumulated as
// weight |result|^2 into the intensity map
__device__ __forceinline__ void epilogue(const CGemmArgs &a, int i, int j, float cr, float ci) {
  float2 outv = make_float2(a.alpha_re * cr - a.alpha_im * ci, a.alpha_re * ci + a.alpha_im * cr);
  if (a.beta != 0.f) {
    const float2 old = a.Cin ? a.Cin[size_t(i) * a.ldcin + j] : a.C[size_t(i) * a.ldc + j];
    outv.x += a.beta * old.x;
    outv.y += a.beta * old.y;
  }
  if (a.mask) {
    const float mk = a.mask[size_t(i) * a.ldm + j];
    outv.x *= mk;
    outv.y *= mk;
  }
  if (!a.skip_c) a.C[size_t(i) * a.ldc + j] = outv;
  if (a.intensity) {
    float *ip = a.intensity + size_t(i) * a.ldi + j;
    *ip += a.weight * (outv.x * outv.x + outv.y * outv.y);
  }
}

__device__ __forceinline__ float2 load_op(const float2 *p, int ld, int r, int c, int rows, int cols,
                                          bool trans, bool conj) {
  // element (r, c) of op(X) where X is stored row-major rows x cols (or transposed)
  if (r >= rows || c >= cols) return make_float2(0.f, 0.f);
  float2 v = trans ? p[size_t(c) * ld + r] : p[size_t(r) * ld + c];
  if (conj) v.y = -v.y;
  return v;
}

__global__ void __launch_bounds__(256) cgemm_kernel(GemmParams gp) {
  const CGemmArgs &a = gp.a;
  __shared__ float2 As[BK][BM + PAD];
  __shared__ float2 Bs[BK][BN + PAD];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * gp.k_per_split;
  const int kend = min(a.K, kbeg + gp.k_per_split);
  // each BK-deep tile is summed by the MFMAs in float32, then added into float64 totals
  double totr[16], toti[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) totr[r] = toti[r] = 0.0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    floatx16 accr = {0.f}, acci = {0.f};
    // A tile: op(A)[i0 + i][k0 + k]; op(A) = A (M x K) or A^T with A stored K x M.
    // The thread mapping walks memory contiguously in either case.
#pragma unroll
    for (int e = tid; e < BM * BK; e += 256) {
      int i, k;
      if (a.transA) {
        i = e % BM;
        k = e / BM;
      } else {
        k = e % BK;
        i = e / BK;
      }
      As[k][i] = load_op(a.A, a.lda, i0 + i, k0 + k, a.M, kend, a.transA != 0, a.conjA != 0);
    }
#pragma unroll
    for (int e = tid; e < BK * BN; e += 256) {
      int k, j;
      if (a.transB) {  // B stored N x K: contiguous along k
        k = e % BK;
        j = e / BK;
      } else {
        j = e % BN;
        k = e / BN;
      }
      float2 v = load_op(a.B, a.ldb, k0 + k, j0 + j, kend, a.N, a.transB != 0, a.conjB != 0);
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int k = kk + (lane >> 5);
      const float2 av = As[k][wm * 32 + (lane & 31)];
      const float2 bv = Bs[k][wn * 32 + (lane & 31)];
      accr = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f32_32x32x2f32(-av.y, bv.y, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.y, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.x, acci, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      totr[r] += double(accr[r]);
      toti[r] += double(acci[r]);
    }
    __syncthreads();
  }
  // accumulator r of lane l sits at row (r/4)*8 + (l/32)*4 + r%4, column l%32 of the wave tile
  const int j = j0 + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = i0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    if (i >= a.M || j >= a.N) continue;
    const float cr = float(totr[r]), ci = float(toti[r]);
    if (gp.split > 1) {
      gp.partial[(size_t(blockIdx.z) * a.M + i) * a.N + j] = make_float2(cr, ci);
    } else {
      epilogue(a, i, j, cr, ci);
    }
  }
}

__global__ void __launch_bounds__(256) split_reduce(GemmParams gp) {
  const CGemmArgs &a = gp.a;
  const size_t total = size_t(a.M) * a.N;
  for (size_t e = size_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += size_t(gridDim.x) * 256) {
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < gp.split; ++s) {
      const float2 v = gp.partial[size_t(s) * total + e];
      sr += v.x;
      si += v.y;
    }
    const int i = int(e / a.N), j = int(e % a.N);
    epilogue(a, i, j, float(sr), float(si));
  }
}

}  // namespace

int cgemm_split_for(int M, int N, int K) {
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int s = 1;
  while (tiles * s < 512 && (K / (BK * (s * 2))) >= 8 && s < kMaxSplit) s *= 2;
  return s;
}

hipError_t launch_cgemm_split(const CGemmArgs &a, int split, float2 *partial, hipStream_t stream,
                              const LaunchHook &hook) {
  GemmParams gp;
  gp.a = a;
  gp.split = split;
  int kps = (a.K + split - 1) / split;
  kps = (kps + BK - 1) / BK * BK;
  gp.k_per_split = kps;
  gp.partial = partial;
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, split);
  hook(stream, "cgemm", a.K, 0);
  hipLaunchKernelGGL(cgemm_kernel, grid, dim3(256), 0, stream, gp);
  hipError_t e = hipGetLastError();
  hook(stream, "cgemm", a.K, 1);
  if (e != hipSuccess || split == 1) return e;
  const size_t total = size_t(a.M) * a.N;
  int blocks = int(std::min<size_t>((total + 255) / 256, 4096));
  hook(stream, "split_reduce", a.K, 0);
  hipLaunchKernelGGL(split_reduce, dim3(blocks), dim3(256), 0, stream, gp);
  e = hipGetLastError();
  hook(stream, "split_reduce", a.K, 1);
  return e;
}

}  // namespace fr
