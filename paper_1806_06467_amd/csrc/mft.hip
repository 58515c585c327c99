// Matrix Fourier transform as two complex GEMMs on the matrix cores (Sec. 1.1: the
// semi-analytic coronagraph of Soummer et al. uses matrix DFTs; Sec. 2.3: the sin/cos arrays of
// that matrix DFT). Unlike the FFT sweeps this step really is a dense contraction, so it runs on
// MFMA.
//
// Complex product with real MFMA: per complex k-step, Cr += Ar Br - Ai Bi and
// Ci += Ar Bi + Ai Br (four v_mfma_f32_32x32x2f32 per 32 x 32 tile, fragments from LDS), or
// with three products (Gauss) P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), Cr = P1 - P2,
// Ci = P3 - P1 - P2, the differences taken in float64 at each fold; or (tile 6) the four real
// products formed on v_mfma_f32_32x32x16_bf16 from exact bfloat16 pieces of the float32
// operands (cgemm_bf_kernel).
// Block tile 64 x 128 (four waves in 2 x 2, each a 32 x 64 piece made of two 32 x 32 MFMA
// tiles) or 64 x 64 for small outputs. Two or three blocks share a compute unit; as their
// barriers are independent, one block's float64 folds overlap another block's MFMAs. Operand
// tiles 16 deep are staged through double-buffered LDS, the next tile's global loads in flight
// while the current one is multiplied (one barrier per tile). Each 16-deep tile (32-deep group
// for the float32 three-product tiles, 128-deep for the bfloat16-split tile, whose sums round
// once per 16 k) is summed by the MFMAs in float32 and then added into float64 totals (the long
// Fourier sums of the coronagraph cancel to tiny values in the dark hole, so their rounding must
// not grow with K); the epilogue (alpha, beta, mask, intensity) runs in float64.
// Operands may be transposed (template) and/or conjugated (on the LDS store). Outputs with few
// tiles and long K are split over K; the float64 partial sums go to the workspace and one
// epilogue kernel adds them in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <type_traits>

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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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

// Blocks are dealt round-robin to the 8 XCDs (each with its own L2). Renumber them so that each
// XCD runs a contiguous range of tiles; inside a K slice the range is walked in groups of
// kGroupRows tile rows, column by column, so that the blocks resident on an XCD at one time share
// a few operand row panels of A and column panels of B in that XCD's L2 (walking whole tile rows
// instead streams all of B once per tile row).
__device__ __forceinline__ void block_tile(int &bx, int &by, int &bz) {
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
  int bx, by, bz;
  block_tile(bx, by, bz);
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
  constexpr int kSums = C::G3 ? 3 : 2;
  floatx16 acc[kSums][TN];
  auto clear = [&] {
#pragma unroll
    for (int q = 0; q < kSums; ++q)
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
  // operand tile from the loader's registers into LDS (imaginary parts conjugated as asked)
  auto stage_store = [&](const TileLoad<C, TA, TB> &ld, int buf) { ld.store(As[buf], Bs[buf], tid, sa, sb); };
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
      stage_store(ld, 0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) ld.load(a, tid, i0, j0, k0 + BK, kend);
      multiply(buf);
      after_stage(!more);
      if (more) stage_store(ld, buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    // two register sets: while stage s is multiplied, one set receives stage s + 2 and the
    // other holds stage s + 1 (stored to the other LDS buffer at the end of the stage)
    TileLoad<C, TA, TB> l0, l1;
    if (kbeg < kend) {
      l0.load(a, tid, i0, j0, kbeg, kend);
      stage_store(l0, 0);
    }
    if (kbeg + BK < kend) l1.load(a, tid, i0, j0, kbeg + BK, kend);
    __syncthreads();
    auto step = [&](int k0, int buf, TileLoad<C, TA, TB> &fill, const TileLoad<C, TA, TB> &ready) {
      if (k0 + 2 * BK < kend) fill.load(a, tid, i0, j0, k0 + 2 * BK, kend);
      multiply(buf);
      after_stage(k0 + BK >= kend);
      if (k0 + BK < kend) stage_store(ready, buf ^ 1);
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

// The bfloat16-split tile (tile 6). Each float32 operand value x (real and imaginary parts, the
// imaginary part's sign flipped when the operand is conjugated) is split exactly into three
// bfloat16 pieces x = hi + mid + lo by rounding to nearest: hi = bf16(x), mid = bf16(x - hi),
// lo = x - hi - mid. Both differences are exact in float32 (each operand pair is within a factor
// of two), and lo has at most eight significant bits, so it is a bfloat16 too; |mid| <= 2^-8 |x|
// and |lo| <= 2^-16 |x|. A real product a b is the sum of the nine piece products, each exact in
// float32; the tile forms the six down to 2^-16 |a b| (hi hi, hi mid, mid hi, mid mid, hi lo,
// lo hi) on v_mfma_f32_32x32x16_bf16, which sums each 16-term dot fused and rounds once. The
// three left out (mid lo, lo mid, lo lo) are below 2^-23 |a b| together and, as round-to-nearest
// residuals, of either sign. The complex product takes four real products per k
// (Cr = Ar Br - Ai Bi, Ci = Ar Bi + Ai Br; -Ai by a sign flip of its pieces), so only two real
// streams per operand are split. The hi hi products and the correction products go to separate
// float32 sums, so that the corrections are never rounded at the scale of the running total;
// every kBfFold stages the sums are added into float64 totals.
// Block tile 64 x 64, four waves of 32 x 32, 16-deep stages through double-buffered LDS. Each
// thread loads four consecutive k of one operand row per stage, two stages ahead of the one
// being multiplied, and while the MFMAs of stage s run it splits stage s + 1 and writes its
// pieces to the other LDS buffer (one 8-byte store per piece, contiguous across the wave).
constexpr int kBfRows = 64;     // block tile edge (M and N)
constexpr int kBfThreads = 256;
constexpr int kBfFold = 8;      // 16-deep stages per float64 fold
constexpr int kBfPieces = 6;    // re hi, re mid, re lo, im hi, im mid, im lo

struct BfRegs {
  float2 a[4], b[4];
};

// LDS row of 16 k as two 8-k halves; rows alternate the halves' order in a pattern that keeps a
// wave's 16-byte fragment reads free of bank conflicts
__device__ __forceinline__ int bf_swz(int row) { return (((row >> 2) ^ (row >> 3)) & 1) * 8; }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// two values as packed bfloat16 pairs of their pieces (first value in the low half), x = hi +
// mid + lo exactly for each (see above)
__device__ __forceinline__ void bf_split2(float x0, float x1, unsigned &hi, unsigned &mid, unsigned &lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(floatx2{x0, x1}, bf16x2));
  const float r0 = x0 - __uint_as_float(hi << 16), r1 = x1 - __uint_as_float(hi & 0xffff0000u);
  mid = __builtin_bit_cast(unsigned, __builtin_convertvector(floatx2{r0, r1}, bf16x2));
  const float l0 = r0 - __uint_as_float(mid << 16), l1 = r1 - __uint_as_float(mid & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(floatx2{l0, l1}, bf16x2));
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(kBfThreads) __attribute__((amdgpu_waves_per_eu(2)))
cgemm_bf_kernel(GemmParams gp) {
  const CGemmArgs &a = gp.a;
  // pieces [buffer][piece][row or column][k], k contiguous (with the half swizzle), so that a
  // lane's eight k values of one piece are one 16-byte read
  __shared__ __attribute__((aligned(16))) unsigned short Ap[2][kBfPieces][kBfRows][BK];
  __shared__ __attribute__((aligned(16))) unsigned short Bp[2][kBfPieces][kBfRows][BK];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  int bx, by, bz;
  block_tile(bx, by, bz);
  const int i0 = by * kBfRows, j0 = bx * kBfRows;
  const int kbeg = bz * gp.k_per_split;
  const int kend = min(a.K, kbeg + gp.k_per_split);
  const int nst = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  const unsigned sma = a.conjA ? 0x80000000u : 0u, smb = a.conjB ? 0x80000000u : 0u;
  // this thread's operand row (A) / column (B) in the tile and its first k of four
  const int lrow = tid >> 2, lk = (tid & 3) * 4;

  // four consecutive complex values base[e .. e + 3] as two 16-byte buffer loads (wave-uniform
  // descriptor, per-lane byte offset; operands below 2^31 bytes)
  auto load_run = [](const float2 *base, unsigned e, float2 *dst) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(base), (short)0, 0x7fffffff, 0x00020000);
    typedef float f4 __attribute__((ext_vector_type(4)));
    const unsigned o = e * 8u;
    const f4 lo = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
    const f4 hi = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u, 0, 0));
    dst[0] = make_float2(lo[0], lo[1]);
    dst[1] = make_float2(lo[2], lo[3]);
    dst[2] = make_float2(hi[0], hi[1]);
    dst[3] = make_float2(hi[2], hi[3]);
  };
  // `full`: the block's tile lies inside M x N and its K slice is a whole number of stages, so
  // no load needs a bounds check (and every path issues the same loads, which keeps the
  // prefetch's wait counts exact)
  auto load = [&](auto full, BfRegs &rg, int k0) {
    constexpr bool F = decltype(full)::value;
    const int gk = k0 + lk;
    const int gi = i0 + lrow, gj = j0 + lrow;
    if (F) {
      if (!TA) {
        load_run(a.A, unsigned(gi) * unsigned(a.lda) + unsigned(gk), rg.a);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) rg.a[r] = a.A[size_t(gk + r) * a.lda + gi];
      }
      if (TB) {
        load_run(a.B, unsigned(gj) * unsigned(a.ldb) + unsigned(gk), rg.b);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) rg.b[r] = a.B[size_t(gk + r) * a.ldb + gj];
      }
      return;
    }
    if (!TA && gi < a.M && gk + 4 <= kend) {
      load_run(a.A, unsigned(gi) * unsigned(a.lda) + unsigned(gk), rg.a);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rg.a[r] = (gi < a.M && gk + r < kend)
                      ? (TA ? a.A[size_t(gk + r) * a.lda + gi] : a.A[size_t(gi) * a.lda + gk + r])
                      : make_float2(0.f, 0.f);
    }
    if (TB && gj < a.N && gk + 4 <= kend) {
      load_run(a.B, unsigned(gj) * unsigned(a.ldb) + unsigned(gk), rg.b);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rg.b[r] = (gj < a.N && gk + r < kend)
                      ? (TB ? a.B[size_t(gj) * a.ldb + gk + r] : a.B[size_t(gk + r) * a.ldb + gj])
                      : make_float2(0.f, 0.f);
    }
  };
  // split four values of one operand row and write the six pieces (8 bytes each) to LDS
  auto put = [&](unsigned short (*dst)[kBfRows][BK], const float2 *v, unsigned sm) {
    unsigned w[kBfPieces][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf_split2(v[2 * h].x, v[2 * h + 1].x, w[0][h], w[1][h], w[2][h]);
      bf_split2(__uint_as_float(__float_as_uint(v[2 * h].y) ^ sm), __uint_as_float(__float_as_uint(v[2 * h + 1].y) ^ sm),
                w[3][h], w[4][h], w[5][h]);
    }
    const int k = lk ^ bf_swz(lrow);
#pragma unroll
    for (int q = 0; q < kBfPieces; ++q) *reinterpret_cast<uint2 *>(&dst[q][lrow][k]) = make_uint2(w[q][0], w[q][1]);
  };

  // float32 sums of the current fold group: Cr and Ci, each as hi hi and correction sums
  floatx16 crh, crc, cih, cic;
  double totr[16], toti[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) totr[r] = toti[r] = 0.0;
  auto clear = [&] {
    crh = floatx16{0.f};
    crc = floatx16{0.f};
    cih = floatx16{0.f};
    cic = floatx16{0.f};
  };
  clear();
  // fragment rows: lane % 32 of the wave's 32 rows (columns), k = 8 (lane / 32) .. + 7
  const int ra = wm * 32 + (lane & 31), rb = wn * 32 + (lane & 31);
  const int ka = 8 * (lane >> 5) ^ bf_swz(ra), kb = 8 * (lane >> 5) ^ bf_swz(rb);
  auto multiply = [&](int buf) {
    bf16x8 fa[kBfPieces], fb[kBfPieces], na[3];
#pragma unroll
    for (int q = 0; q < kBfPieces; ++q) {
      fa[q] = *reinterpret_cast<const bf16x8 *>(&Ap[buf][q][ra][ka]);
      fb[q] = *reinterpret_cast<const bf16x8 *>(&Bp[buf][q][rb][kb]);
    }
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < 3; ++q)
      na[q] = __builtin_bit_cast(bf16x8, __builtin_bit_cast(u4, fa[3 + q]) ^ u4{0x80008000u, 0x80008000u,
                                                                                 0x80008000u, 0x80008000u});
    // the five corrections smallest first (mid mid, lo hi, hi lo, mid hi, hi mid), then hi hi;
    // the Cr and Ci chains alternate so consecutive MFMAs are independent
    constexpr int lx[5] = {1, 2, 0, 1, 0}, ly[5] = {1, 0, 2, 0, 1};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int x = lx[q], y = ly[q];
      crc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[x], fb[y], crc, 0, 0, 0);
      cic = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[x], fb[3 + y], cic, 0, 0, 0);
      crc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[x], fb[3 + y], crc, 0, 0, 0);
      cic = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[3 + x], fb[y], cic, 0, 0, 0);
    }
    crh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], fb[0], crh, 0, 0, 0);
    cih = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], fb[3], cih, 0, 0, 0);
    crh = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[0], fb[3], crh, 0, 0, 0);
    cih = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[3], fb[0], cih, 0, 0, 0);
  };
  auto fold = [&] {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      totr[r] += double(crh[r]) + double(crc[r]);
      toti[r] += double(cih[r]) + double(cic[r]);
    }
    clear();
  };

  // stage s: multiply LDS buffer `buf` while `ready` (stage s + 1) is split into the other
  // buffer and `fill` receives stage s + 2. At the last stage the split writes a repeated stage
  // to a buffer nobody reads again.
  auto run = [&](auto full) {
    BfRegs r0, r1;
#pragma unroll
    for (int r = 0; r < 4; ++r) r0.a[r] = r0.b[r] = r1.a[r] = r1.b[r] = make_float2(0.f, 0.f);
    if (nst == 0) return;
    load(full, r0, kbeg);
    put(Ap[0], r0.a, sma);
    put(Bp[0], r0.b, smb);
    load(full, r1, kbeg + min(1, nst - 1) * BK);
    __syncthreads();
    int pending = 0;
    // the loads are issued unconditionally (the last stages reload the last stage) so that the
    // wait before the split counts only the previous stage's loads
    auto stage = [&](int s, int buf, BfRegs &fill, const BfRegs &ready) {
      load(full, fill, kbeg + min(s + 2, nst - 1) * BK);
      multiply(buf);
      put(Ap[buf ^ 1], ready.a, sma);
      put(Bp[buf ^ 1], ready.b, smb);
      if (++pending == kBfFold || s + 1 == nst) {
        fold();
        pending = 0;
      }
      __syncthreads();
    };
    for (int s = 0; s < nst; s += 2) {
      stage(s, 0, r0, r1);
      if (s + 1 < nst) stage(s + 1, 1, r1, r0);
    }
  };
  const bool full = i0 + kBfRows <= a.M && j0 + kBfRows <= a.N && (kend - kbeg) % BK == 0;
  if (full) run(std::true_type{});
  else run(std::false_type{});
  // accumulator r of lane l sits at row (r/4)*8 + (l/32)*4 + r%4, column l%32 of the wave's tile
  const int j = j0 + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = i0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    if (i >= a.M || j >= a.N) continue;
    if (gp.split > 1) {
      gp.partial[(size_t(bz) * a.M + i) * a.N + j] = make_double2(totr[r], toti[r]);
    } else {
      epilogue(a, i, j, totr[r], toti[r]);
    }
  }
}

// output rows over blockIdx.y, columns over blockIdx.x and the threads (no index division),
// the partials added in slice order
__global__ void __launch_bounds__(256) split_reduce(GemmParams gp) {
  const CGemmArgs &a = gp.a;
  const size_t total = size_t(a.M) * a.N;
  for (int i = blockIdx.y; i < a.M; i += gridDim.y) {
    for (int j = blockIdx.x * 256 + threadIdx.x; j < a.N; j += gridDim.x * 256) {
      const size_t e = size_t(i) * a.N + j;
      double sr = 0.0, si = 0.0;
      for (int s = 0; s < gp.split; ++s) {
        const double2 v = gp.partial[size_t(s) * total + e];
        sr += v.x;
        si += v.y;
      }
      epilogue(a, i, j, sr, si);
    }
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

hipError_t launch_bf(const GemmParams &gp, hipStream_t stream) {
  const CGemmArgs &a = gp.a;
  dim3 grid((a.N + kBfRows - 1) / kBfRows, (a.M + kBfRows - 1) / kBfRows, gp.split);
  if (a.transA) {
    if (a.transB) hipLaunchKernelGGL((cgemm_bf_kernel<true, true>), grid, dim3(kBfThreads), 0, stream, gp);
    else hipLaunchKernelGGL((cgemm_bf_kernel<true, false>), grid, dim3(kBfThreads), 0, stream, gp);
  } else {
    if (a.transB) hipLaunchKernelGGL((cgemm_bf_kernel<false, true>), grid, dim3(kBfThreads), 0, stream, gp);
    else hipLaunchKernelGGL((cgemm_bf_kernel<false, false>), grid, dim3(kBfThreads), 0, stream, gp);
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
// 5 large with three products per complex step, 6 small on bfloat16 pieces; `cfg` >= 0 is a
// choice made by the autotuner (or a tuning file), else the default by shape
int tile_choice(int M, int N, int K, int cfg) {
  if (cfg >= 0 && cfg < kGemmTiles) return cfg;
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
    case 6: return split_for(tiles_of<CfgS>(M, N), K);  // 64 x 64 like the small tile
    default: return split_for(tiles_of<CfgS>(M, N), K);
  }
}

// the bfloat16 tile reads k-contiguous operands through a buffer descriptor with 32-bit byte
// offsets: both operands' extents must stay below 2^31 bytes
bool bf_offsets_fit(const CGemmArgs &a) {
  const long long ea = (a.transA ? (long long)(a.K - 1) * a.lda + a.M : (long long)(a.M - 1) * a.lda + a.K);
  const long long eb = (a.transB ? (long long)(a.N - 1) * a.ldb + a.K : (long long)(a.K - 1) * a.ldb + a.N);
  return ea * 8 < (1ll << 31) - 64 && eb * 8 < (1ll << 31) - 64;
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
  int cfg = tile_choice(a.M, a.N, a.K, cfg_choice);
  if (cfg == 6 && !bf_offsets_fit(a)) cfg = 4;  // the same products on float32 operands
  char name[64];
  static const char *const tag[kGemmTiles] = {"S", "L", "X", "P", "S3", "L3", "B"};
  std::snprintf(name, sizeof name, "cgemm%s_%dx%dx%d_s%d", tag[cfg], a.M, a.N, a.K, split);
  hook(stream, name, a.K, 0);
  hipError_t e = cfg == 1 ? launch_cfg<CfgL>(gp, stream)
                 : cfg == 2 ? launch_cfg<CfgX>(gp, stream)
                 : cfg == 3 ? launch_cfg<CfgP>(gp, stream)
                 : cfg == 4 ? launch_cfg<CfgS3>(gp, stream)
                 : cfg == 5 ? launch_cfg<CfgL3>(gp, stream)
                 : cfg == 6 ? launch_bf(gp, stream)
                            : launch_cfg<CfgS>(gp, stream);
  hook(stream, name, a.K, 1);
  if (e != hipSuccess || split == 1) return e;
  hook(stream, "split_reduce", a.K, 0);
  hipLaunchKernelGGL(split_reduce, dim3(std::min((a.N + 255) / 256, 16), std::min(a.M, 65535)), dim3(256), 0, stream, gp);
  e = hipGetLastError();
  hook(stream, "split_reduce", a.K, 1);
  return e;
}

}  // namespace fr
