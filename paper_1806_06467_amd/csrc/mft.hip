// Matrix Fourier transform as two complex GEMMs on FP32 MFMA (Sec. 1.1: the semi-analytic
// coronagraph of Soummer et al. uses matrix DFTs; Sec. 2.3: the sin/cos arrays of that
// matrix DFT). Unlike the FFT sweeps this step really is a dense contraction, so it runs on
// the matrix cores.
//
// Complex product with real MFMA: per complex k-step, Cr += Ar Br - Ai Bi and
// Ci += Ar Bi + Ai Br (four v_mfma_f32_32x32x2f32 per 32 x 32 tile, fragments from LDS), or
// with three products (Gauss) P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), Cr = P1 - P2,
// Ci = P3 - P1 - P2, the differences taken in float64 at each fold.
// Block tile 64 x 128 (four waves in 2 x 2, each a 32 x 64 piece made of two 32 x 32 MFMA
// tiles) or 64 x 64 for small outputs. Two or three blocks share a compute unit; as their
// barriers are independent, one block's float64 folds overlap another block's MFMAs. Operand tiles 16 deep are staged through double-buffered LDS, the next tile's
// global loads in flight while the current one is multiplied (one barrier per tile). Each
// 16-deep tile (32-deep group for the three-product tiles) is summed by the MFMAs in float32 and
// then added into float64 totals (the long Fourier sums of the coronagraph cancel to tiny values
// in the dark hole, so their rounding must not grow with K); the epilogue (alpha, beta, mask,
// intensity) runs in float64.
// Operands may be transposed (template) and/or conjugated (on the LDS store). Outputs with few
// tiles and long K are split over K; the float64 partial sums go to the workspace and one
// epilogue kernel adds them in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "fr_internal.h"

namespace fr {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BK = 16;
constexpr int PAD = 4;

struct GemmParams {
  CGemmArgs a;
  int split;        // number of K slices (gridDim.z)
  int k_per_split;  // multiple of BK
  double2 *partial; // split x M x N when split > 1
};

// result (i, j) = alpha acc + beta Cin, times mask, in float64; written to C and/or
// accumulated as weight |result|^2 into the float64 intensity map
__device__ __forceinline__ void epilogue(const CGemmArgs &a, int i, int j, double cr, double ci) {
  double orr = a.alpha_re * cr - a.alpha_im * ci;
  double oi = a.alpha_re * ci + a.alpha_im * cr;
  if (a.beta != 0.f) {
    const float2 old = a.Cin ? a.Cin[size_t(i) * a.ldcin + j] : a.C[size_t(i) * a.ldc + j];
    orr += double(a.beta) * double(old.x);
    oi += double(a.beta) * double(old.y);
  }
  if (a.mask) {
    const double mk = a.mask[size_t(i) * a.ldm + j];
    orr *= mk;
    oi *= mk;
  }
  if (!a.skip_c) a.C[size_t(i) * a.ldc + j] = make_float2(float(orr), float(oi));
  if (a.intensity) {
    double *ip = a.intensity + size_t(i) * a.ldi + j;
    *ip += a.weight * (orr * orr + oi * oi);
  }
}

// Tile configuration: WM x WN waves, each wave a 32 x (32 TN) piece of the block tile; the
// operand tiles of the next PD stages are in flight while a stage is multiplied. G3: three real
// products per complex k-step instead of four (Gauss): P1 = sum Ar Br, P2 = sum Ai Bi,
// P3 = sum (Ar + Ai)(Br + Bi), combined per stage in float64 as Cr = P1 - P2, Ci = P3 - P1 - P2.
template <int WM_, int WN_, int TN_, int PD_ = 1, bool G3_ = false, int FOLD_ = 1>
struct Cfg {
  static constexpr int WM = WM_, WN = WN_, TN = TN_, PD = PD_;
  static constexpr bool G3 = G3_;
  static constexpr int FOLD = FOLD_;  // 16-deep stages summed in float32 between float64 folds
  // waves per SIMD the register budget targets (the three-product 32 x 64 wave tile holds three
  // float32 and two float64 accumulator sets, so it gets the whole register file)
  static constexpr int waves = TN == 1 ? 3 : (G3 ? 1 : 2);
  static constexpr int BM = 32 * WM, BN = 32 * TN * WN;
  static constexpr int threads = 64 * WM * WN;
  static constexpr int la = BM * BK / threads;  // A elements per thread per tile
  static constexpr int lb = BK * BN / threads;  // B elements per thread per tile
  static_assert(BM * BK % threads == 0 && BK * BN % threads == 0, "tile not divisible");
  static_assert(threads % BK == 0 && threads % BM == 0 && threads % BN == 0, "thread mapping");
};
using CfgL = Cfg<2, 2, 2>;  // 64 x 128, 256 threads: two blocks share a compute unit
using CfgS = Cfg<2, 2, 1>;  // 64 x 64, 256 threads
using CfgX = Cfg<4, 2, 2>;  // 128 x 128, 512 threads
using CfgP = Cfg<2, 2, 1, 2>;  // 64 x 64, 256 threads, two stages of loads in flight
// three products per complex step, float32 sums over 32-deep groups between float64 folds
using CfgS3 = Cfg<2, 2, 1, 1, true, 2>;  // 64 x 64
using CfgL3 = Cfg<2, 2, 2, 1, true, 2>;  // 64 x 128

// Per-thread share of one BK-deep operand tile, mapped so that consecutive threads walk
// memory contiguously.
template <class C, bool TA, bool TB>
struct TileLoad {
  float2 ra[C::la], rb[C::lb];
  __device__ __forceinline__ static void a_coord(int t, int r, int &i, int &k) {
    if (TA) {  // A stored K x M: contiguous along i
      i = t % C::BM;
      k = t / C::BM + (C::threads / C::BM) * r;
    } else {   // A stored M x K: contiguous along k
      k = t % BK;
      i = t / BK + (C::threads / BK) * r;
    }
  }
  __device__ __forceinline__ static void b_coord(int t, int r, int &k, int &j) {
    if (TB) {  // B stored N x K: contiguous along k
      k = t % BK;
      j = t / BK + (C::threads / BK) * r;
    } else {   // B stored K x N: contiguous along j
      j = t % C::BN;
      k = t / C::BN + (C::threads / C::BN) * r;
    }
  }
  __device__ __forceinline__ void load(const CGemmArgs &a, int t, int i0, int j0, int k0, int kend) {
#pragma unroll
    for (int r = 0; r < C::la; ++r) {
      int i, k;
      a_coord(t, r, i, k);
      const int gi = i0 + i, gk = k0 + k;
      ra[r] = (gi < a.M && gk < kend) ? (TA ? a.A[size_t(gk) * a.lda + gi] : a.A[size_t(gi) * a.lda + gk])
                                      : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < C::lb; ++r) {
      int k, j;
      b_coord(t, r, k, j);
      const int gk = k0 + k, gj = j0 + j;
      rb[r] = (gj < a.N && gk < kend) ? (TB ? a.B[size_t(gj) * a.ldb + gk] : a.B[size_t(gk) * a.ldb + gj])
                                      : make_float2(0.f, 0.f);
    }
  }
  __device__ __forceinline__ void store(float2 (*As)[C::BM + PAD], float2 (*Bs)[C::BN + PAD], int t, float sa,
                                        float sb) const {
#pragma unroll
    for (int r = 0; r < C::la; ++r) {
      int i, k;
      a_coord(t, r, i, k);
      As[k][i] = make_float2(ra[r].x, sa * ra[r].y);
    }
#pragma unroll
    for (int r = 0; r < C::lb; ++r) {
      int k, j;
      b_coord(t, r, k, j);
      Bs[k][j] = make_float2(rb[r].x, sb * rb[r].y);
    }
  }
};

template <class C, bool TA, bool TB>
__global__ void __launch_bounds__(C::threads) __attribute__((amdgpu_waves_per_eu(C::waves)))
cgemm_kernel(GemmParams gp) {
  static_assert(C::threads <= 512, "block too large");
  constexpr int TN = C::TN;
  const CGemmArgs &a = gp.a;
  __shared__ float2 As[2][BK][C::BM + PAD];
  __shared__ float2 Bs[2][BK][C::BN + PAD];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / C::WN, wn = wave % C::WN;
  // Blocks are dealt round-robin to the 8 XCDs (each with its own L2). Renumber them so that
  // each XCD runs a contiguous range of tiles; inside a K slice the range is walked in groups of
  // kGroupRows tile rows, column by column, so that the blocks resident on an XCD at one time
  // share a few operand row panels of A and column panels of B in that XCD's L2 (walking whole
  // tile rows instead streams all of B once per tile row).
  int bx, by, bz;
  {
    constexpr int kGroupRows = 8;
    const int gx = gridDim.x, gy = gridDim.y;
    const int total = gx * gy * gridDim.z;
    const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int tile = total % 8 == 0 ? (lin & 7) * (total >> 3) + (lin >> 3) : lin;
    bz = tile / (gx * gy);
    const int t = tile % (gx * gy);
    const int g = t / (kGroupRows * gx);             // group of tile rows
    const int rows = min(kGroupRows, gy - g * kGroupRows);
    const int u = t % (kGroupRows * gx);             // position inside the group
    bx = u / rows;
    by = g * kGroupRows + u % rows;
  }
  const int i0 = by * C::BM, j0 = bx * C::BN;
  const int kbeg = bz * gp.k_per_split;
  const int kend = min(a.K, kbeg + gp.k_per_split);
  const float sa = a.conjA ? -1.f : 1.f, sb = a.conjB ? -1.f : 1.f;
  double totr[TN][16], toti[TN][16];
#pragma unroll
  for (int t = 0; t < TN; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) totr[t][r] = toti[t][r] = 0.0;
  const int arow = wm * 32 + (lane & 31);
  const int bcol = wn * 32 * TN + (lane & 31);
  const int kl = lane >> 5;
  // float32 sums of the current fold group: (P1, P2, P3) for three products, (Cr, Ci) else
  floatx16 acc[C::G3 ? 3 : 2][TN];
  auto clear = [&] {
#pragma unroll
    for (int q = 0; q < (C::G3 ? 3 : 2); ++q)
#pragma unroll
      for (int t = 0; t < TN; ++t) acc[q][t] = floatx16{0.f};
  };
  clear();
  // one stage: multiply the LDS tile `buf` into the float32 sums
  auto multiply = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const float2 av = As[buf][kk + kl][arow];
      float2 bv[TN];
#pragma unroll
      for (int t = 0; t < TN; ++t) bv[t] = Bs[buf][kk + kl][bcol + 32 * t];
      if constexpr (C::G3) {
        const float as = av.x + av.y;
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          acc[0][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv[t].x, acc[0][t], 0, 0, 0);
          acc[1][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv[t].y, acc[1][t], 0, 0, 0);
          acc[2][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(as, bv[t].x + bv[t].y, acc[2][t], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          acc[0][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv[t].x, acc[0][t], 0, 0, 0);
          acc[1][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv[t].y, acc[1][t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          acc[0][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(-av.y, bv[t].y, acc[0][t], 0, 0, 0);
          acc[1][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv[t].x, acc[1][t], 0, 0, 0);
        }
      }
    }
  };
  // add the float32 sums into the float64 totals and restart them
  auto fold = [&] {
#pragma unroll
    for (int t = 0; t < TN; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if constexpr (C::G3) {
          const double d1 = double(acc[0][t][r]), d2 = double(acc[1][t][r]);
          totr[t][r] += d1 - d2;
          toti[t][r] += double(acc[2][t][r]) - d1 - d2;
        } else {
          totr[t][r] += double(acc[0][t][r]);
          toti[t][r] += double(acc[1][t][r]);
        }
      }
    clear();
  };
  int pending = 0;  // stages multiplied since the last fold
  auto after_stage = [&](bool last) {
    if (++pending == C::FOLD || last) {
      fold();
      pending = 0;
    }
  };
  if constexpr (C::PD == 1) {
    TileLoad<C, TA, TB> ld;
    if (kbeg < kend) {
      ld.load(a, tid, i0, j0, kbeg, kend);
      ld.store(As[0], Bs[0], tid, sa, sb);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) ld.load(a, tid, i0, j0, k0 + BK, kend);
      multiply(buf);
      after_stage(!more);
      if (more) ld.store(As[buf ^ 1], Bs[buf ^ 1], tid, sa, sb);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    // two register sets: while stage s is multiplied, one set receives stage s + 2 and the
    // other holds stage s + 1 (stored to the other LDS buffer at the end of the stage)
    TileLoad<C, TA, TB> l0, l1;
    if (kbeg < kend) {
      l0.load(a, tid, i0, j0, kbeg, kend);
      l0.store(As[0], Bs[0], tid, sa, sb);
    }
    if (kbeg + BK < kend) l1.load(a, tid, i0, j0, kbeg + BK, kend);
    __syncthreads();
    auto step = [&](int k0, int buf, TileLoad<C, TA, TB> &fill, const TileLoad<C, TA, TB> &ready) {
      if (k0 + 2 * BK < kend) fill.load(a, tid, i0, j0, k0 + 2 * BK, kend);
      multiply(buf);
      after_stage(k0 + BK >= kend);
      if (k0 + BK < kend) ready.store(As[buf ^ 1], Bs[buf ^ 1], tid, sa, sb);
      __syncthreads();
    };
    for (int k0 = kbeg; k0 < kend; k0 += 2 * BK) {
      step(k0, 0, l0, l1);
      if (k0 + BK < kend) step(k0 + BK, 1, l1, l0);
    }
  }
  // the last stage of the slice ended with a fold, so the float64 totals hold everything
  // accumulator r of lane l sits at row (r/4)*8 + (l/32)*4 + r%4, column l%32 of a 32 x 32 tile
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    const int j = j0 + wn * 32 * TN + t * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = i0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
      if (i >= a.M || j >= a.N) continue;
      if (gp.split > 1) {
        gp.partial[(size_t(bz) * a.M + i) * a.N + j] = make_double2(totr[t][r], toti[t][r]);
      } else {
        epilogue(a, i, j, totr[t][r], toti[t][r]);
      }
    }
  }
}

__global__ void __launch_bounds__(256) split_reduce(GemmParams gp) {
  const CGemmArgs &a = gp.a;
  const size_t total = size_t(a.M) * a.N;
  for (size_t e = size_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += size_t(gridDim.x) * 256) {
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < gp.split; ++s) {
      const double2 v = gp.partial[size_t(s) * total + e];
      sr += v.x;
      si += v.y;
    }
    const int i = int(e / a.N), j = int(e % a.N);
    epilogue(a, i, j, sr, si);
  }
}

template <class C>
hipError_t launch_cfg(const GemmParams &gp, hipStream_t stream) {
  const CGemmArgs &a = gp.a;
  dim3 grid((a.N + C::BN - 1) / C::BN, (a.M + C::BM - 1) / C::BM, gp.split);
  if (a.transA) {
    if (a.transB) hipLaunchKernelGGL((cgemm_kernel<C, true, true>), grid, dim3(C::threads), 0, stream, gp);
    else hipLaunchKernelGGL((cgemm_kernel<C, true, false>), grid, dim3(C::threads), 0, stream, gp);
  } else {
    if (a.transB) hipLaunchKernelGGL((cgemm_kernel<C, false, true>), grid, dim3(C::threads), 0, stream, gp);
    else hipLaunchKernelGGL((cgemm_kernel<C, false, false>), grid, dim3(C::threads), 0, stream, gp);
  }
  return hipGetLastError();
}

template <class C>
int tiles_of(int M, int N) {
  return ((M + C::BM - 1) / C::BM) * ((N + C::BN - 1) / C::BN);
}

// K slices so that the grid holds about two blocks per compute unit, each slice at least
// 128 deep
int split_for(int tiles, int K) {
  int s = 1;
  while (tiles * s < 512 && K / (s * 2) >= 128 && s < kMaxSplit) s *= 2;
  return s;
}

// the large tile when it (with its split) still gives about one block per compute unit
bool use_large(int M, int N, int K) {
  const int t = tiles_of<CfgL>(M, N);
  return t * split_for(t, K) >= 256;
}

// tile configuration: 0 small, 1 large, 2 extra large, 3 small with deeper prefetch, 4 small and
// 5 large with three products per complex step; `cfg` >= 0 is a choice made by the autotuner,
// else FR_GEMM_TILE (s, l, x, p, t, u) overrides the default for manual tuning runs
int tile_choice(int M, int N, int K, int cfg) {
  if (cfg >= 0 && cfg < kGemmTiles) return cfg;
  static const int forced = [] {
    const char *v = std::getenv("FR_GEMM_TILE");
    if (!v) return -1;
    return v[0] == 's' ? 0 : v[0] == 'l' ? 1 : v[0] == 'x' ? 2 : v[0] == 'p' ? 3 : v[0] == 't' ? 4 : v[0] == 'u' ? 5 : -1;
  }();
  if (forced >= 0) return forced;
  return use_large(M, N, K) ? 1 : 0;
}

}  // namespace

int cgemm_split_for(int M, int N, int K, int cfg) {
  switch (tile_choice(M, N, K, cfg)) {
    case 1: return split_for(tiles_of<CfgL>(M, N), K);
    case 2: return split_for(tiles_of<CfgX>(M, N), K);
    case 3: return split_for(tiles_of<CfgP>(M, N), K);
    case 4: return split_for(tiles_of<CfgS3>(M, N), K);
    case 5: return split_for(tiles_of<CfgL3>(M, N), K);
    default: return split_for(tiles_of<CfgS>(M, N), K);
  }
}

hipError_t launch_cgemm_split(const CGemmArgs &a, int split, int cfg_choice, void *partial, hipStream_t stream,
                              const LaunchHook &hook) {
  GemmParams gp;
  gp.a = a;
  gp.split = split;
  int kps = (a.K + split - 1) / split;
  kps = (kps + BK - 1) / BK * BK;
  gp.k_per_split = kps;
  gp.partial = static_cast<double2 *>(partial);
  const int cfg = tile_choice(a.M, a.N, a.K, cfg_choice);
  char name[64];
  static const char *const tag[kGemmTiles] = {"S", "L", "X", "P", "S3", "L3"};
  std::snprintf(name, sizeof name, "cgemm%s_%dx%dx%d_s%d", tag[cfg], a.M, a.N, a.K, split);
  hook(stream, name, a.K, 0);
  hipError_t e = cfg == 1 ? launch_cfg<CfgL>(gp, stream)
                 : cfg == 2 ? launch_cfg<CfgX>(gp, stream)
                 : cfg == 3 ? launch_cfg<CfgP>(gp, stream)
                 : cfg == 4 ? launch_cfg<CfgS3>(gp, stream)
                 : cfg == 5 ? launch_cfg<CfgL3>(gp, stream)
                            : launch_cfg<CfgS>(gp, stream);
  hook(stream, name, a.K, 1);
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
