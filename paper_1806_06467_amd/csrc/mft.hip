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
// 16-deep tile (32-deep group for the float32 three-product tiles, 128-deep for the bfloat16-split
// tile, whose leading sum rounds once per 16 k) is summed by the MFMAs in float32 and
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
template <int WM_, int WN_, int TN_, int PD_ = 1, bool G3_ = false, int FOLD_ = 1, bool BF_ = false>
struct Cfg {
  static constexpr int WM = WM_, WN = WN_, TN = TN_, PD = PD_;
  static constexpr bool G3 = G3_;
  static constexpr int FOLD = FOLD_;  // 16-deep stages summed in float32 between float64 folds
  // BF: the three real operand streams (re, im, re + im) are split exactly into three bfloat16
  // pieces each (hi, mid below 2^-7 and lo below 2^-15 of the value) and multiplied on
  // v_mfma_f32_32x32x16_bf16: every piece product except lo lo (below 2^-30 of the leading
  // one), each exact in float32
  static constexpr bool BF = BF_;
  static_assert(!BF || (G3 && TN == 1), "bfloat16 split tiles: three products, 32 x 32 per wave");
  // waves per SIMD the register budget targets (the three-product 32 x 64 wave tile holds three
  // float32 and two float64 accumulator sets, so it gets the whole register file)
  static constexpr int waves = BF ? 2 : TN == 1 ? 3 : (G3 ? 1 : 2);
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
// three products on bfloat16 pieces, 64 x 64
using CfgB = Cfg<2, 2, 1, 1, true, 8, true>;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Per-thread share of one BK-deep operand tile, mapped so that consecutive threads walk
// memory contiguously.
template <class C, bool TA, bool TB>
struct TileLoad {
  float2 ra[C::la], rb[C::lb];
  // For the bfloat16 tiles every thread holds la (lb) consecutive k of one row (column), so that
  // each of its pieces goes to LDS as one 8-byte write: an operand stored with i (j) contiguous
  // keeps its loads contiguous along i (j) for every r; one stored with k contiguous is read as
  // 32-byte runs (four threads per 16-deep row).
  static constexpr int kRun = BK / 4;  // threads per row of a k-contiguous bfloat16 operand
  __device__ __forceinline__ static void a_coord(int t, int r, int &i, int &k) {
    if (TA) {  // A stored K x M: contiguous along i
      i = t % C::BM;
      k = C::BF ? (t / C::BM) * C::la + r : t / C::BM + (C::threads / C::BM) * r;
    } else if (C::BF) {
      i = t / kRun;
      k = (t % kRun) * 4 + r;
    } else {   // A stored M x K: contiguous along k
      k = t % BK;
      i = t / BK + (C::threads / BK) * r;
    }
  }
  __device__ __forceinline__ static void b_coord(int t, int r, int &k, int &j) {
    if (TB) {  // B stored N x K: contiguous along k
      if (C::BF) {
        j = t / kRun;
        k = (t % kRun) * 4 + r;
      } else {
        k = t % BK;
        j = t / BK + (C::threads / BK) * r;
      }
    } else {   // B stored K x N: contiguous along j
      j = t % C::BN;
      k = C::BF ? (t / C::BN) * C::lb + r : t / C::BN + (C::threads / C::BN) * r;
    }
  }
  // four consecutive complex values base[e .. e + 3] (32 bytes, 8-byte aligned) as two 16-byte
  // buffer loads; the descriptor is the operand's (wave-uniform), e the per-lane element offset
  // (operands up to 2^28 elements, so the byte offset fits 32 bits)
  __device__ __forceinline__ static void load_run(const float2 *base, size_t e, float2 *dst) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(base), (short)0, 0x7fffffff, 0x00020000);
    typedef float f4 __attribute__((ext_vector_type(4)));
    const unsigned o = unsigned(e) * 8u;
    const f4 lo = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
    const f4 hi = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u, 0, 0));
    dst[0] = make_float2(lo[0], lo[1]);
    dst[1] = make_float2(lo[2], lo[3]);
    dst[2] = make_float2(hi[0], hi[1]);
    dst[3] = make_float2(hi[2], hi[3]);
  }
  __device__ __forceinline__ void load(const CGemmArgs &a, int t, int i0, int j0, int k0, int kend) {
    if constexpr (C::BF && !TA) {
      static_assert(C::la == 4, "one 4-run per thread");
      int i, k;
      a_coord(t, 0, i, k);
      const int gi = i0 + i, gk = k0 + k;
      if (gi < a.M && gk + 4 <= kend) {
        load_run(a.A, size_t(gi) * a.lda + gk, ra);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ra[r] = (gi < a.M && gk + r < kend) ? a.A[size_t(gi) * a.lda + gk + r] : make_float2(0.f, 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < C::la; ++r) {
        int i, k;
        a_coord(t, r, i, k);
        const int gi = i0 + i, gk = k0 + k;
        ra[r] = (gi < a.M && gk < kend) ? (TA ? a.A[size_t(gk) * a.lda + gi] : a.A[size_t(gi) * a.lda + gk])
                                        : make_float2(0.f, 0.f);
      }
    }
    if constexpr (C::BF && TB) {
      static_assert(C::lb == 4, "one 4-run per thread");
      int k, j;
      b_coord(t, 0, k, j);
      const int gk = k0 + k, gj = j0 + j;
      if (gj < a.N && gk + 4 <= kend) {
        load_run(a.B, size_t(gj) * a.ldb + gk, rb);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          rb[r] = (gj < a.N && gk + r < kend) ? a.B[size_t(gj) * a.ldb + gk + r] : make_float2(0.f, 0.f);
      }
    } else {
#pragma unroll
      for (int r = 0; r < C::lb; ++r) {
        int k, j;
        b_coord(t, r, k, j);
        const int gk = k0 + k, gj = j0 + j;
        rb[r] = (gj < a.N && gk < kend) ? (TB ? a.B[size_t(gj) * a.ldb + gk] : a.B[size_t(gk) * a.ldb + gj])
                                        : make_float2(0.f, 0.f);
      }
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
  __shared__ float2 As[C::BF ? 1 : 2][BK][C::BM + PAD];
  __shared__ float2 Bs[C::BF ? 1 : 2][BK][C::BN + PAD];
  // bfloat16 pieces, [buffer][stream * 3 + level][row or column][k], k contiguous so that a
  // lane's eight k values of one piece are one 16-byte read
  constexpr int kPieces = 9;
  __shared__ __attribute__((aligned(16))) unsigned short Ab[C::BF ? 2 : 1][C::BF ? kPieces : 1][C::BF ? C::BM : 1][BK];
  __shared__ __attribute__((aligned(16))) unsigned short Bb[C::BF ? 2 : 1][C::BF ? kPieces : 1][C::BF ? C::BN : 1][BK];
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
  // float32 sums of the current fold group: (P1, P2, P3) for three products, (Cr, Ci) else; the
  // bfloat16 tile keeps each P in two sums, the hi hi products and the (at least 2^-7 smaller)
  // correction products, so that the correction terms are not rounded at the scale of the total
  constexpr int kSums = C::BF ? 6 : (C::G3 ? 3 : 2);
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
    if constexpr (C::BF) {
      // lane: row (column) lane % 32 of the wave's piece, k = 8 (lane / 32) .. + 7
      const int kh = 8 * (lane >> 5);
      bf16x8 ap[3][3], bp[3][3];
#pragma unroll
      for (int st = 0; st < 3; ++st)
#pragma unroll
        for (int lv = 0; lv < 3; ++lv) {
          ap[st][lv] = *reinterpret_cast<const bf16x8 *>(&Ab[buf][st * 3 + lv][arow][kh]);
          bp[st][lv] = *reinterpret_cast<const bf16x8 *>(&Bb[buf][st * 3 + lv][bcol][kh]);
        }
      // eight piece products: the seven corrections smallest first (lo mid, mid lo, lo hi,
      // mid mid, hi lo, mid hi, hi mid) into the correction sum, then hi hi into the main sum;
      // only lo lo (below 2^-28 of the leading product) is left out. The three streams' chains
      // are interleaved so that consecutive MFMAs are independent.
      constexpr int la_[7] = {2, 1, 2, 1, 0, 1, 0}, lb_[7] = {1, 2, 0, 1, 2, 0, 1};
#pragma unroll
      for (int q = 0; q < 7; ++q)
#pragma unroll
        for (int st = 0; st < 3; ++st)
          acc[2 * st + 1][0] =
              __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap[st][la_[q]], bp[st][lb_[q]], acc[2 * st + 1][0], 0, 0, 0);
#pragma unroll
      for (int st = 0; st < 3; ++st)
        acc[2 * st][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap[st][0], bp[st][0], acc[2 * st][0], 0, 0, 0);
      return;
    }
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
  // operand tile from the loader's registers into LDS: float32 complex, or for BF the three
  // streams (re, im, re + im; imaginary parts conjugated as asked) in bfloat16 pieces
  auto stage_store = [&](const TileLoad<C, TA, TB> &ld, int buf) {
    if constexpr (C::BF) {
      // one operand's elements: pieces of the three streams, as 2-byte writes (k contiguous
      // across lanes) or, when a thread holds n consecutive k of one row, as one 2n-byte write
      // the four consecutive-k values v[0..3] of one row. Each stream value x = hi + mid + lo
      // exactly, each piece a bfloat16 (the upper 16 bits of a float32 bit pattern): hi and mid
      // by truncation, the remainders r = x - hi and r - mid being exact in float32, lo holding
      // the last at most eight significant bits. Pairs of upper halves are packed by one byte
      // permute each and written as one 8-byte store per piece.
      auto put = [&](unsigned short(*dst)[C::BF ? C::BM : 1][BK], const float2 *v, float sc, int row, int k0) {
        unsigned bits[3][3][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float re = v[r].x, im = sc * v[r].y;
          const float x3[3] = {re, im, re + im};
#pragma unroll
          for (int st = 0; st < 3; ++st) {
            const unsigned xb = __float_as_uint(x3[st]);
            const float rr = x3[st] - __uint_as_float(xb & 0xffff0000u);
            const unsigned rb = __float_as_uint(rr);
            bits[st][0][r] = xb;
            bits[st][1][r] = rb;
            bits[st][2][r] = __float_as_uint(rr - __uint_as_float(rb & 0xffff0000u));
          }
        }
#pragma unroll
        for (int st = 0; st < 3; ++st)
#pragma unroll
          for (int lv = 0; lv < 3; ++lv) {
            // upper half of the second operand in the low half, of the first in the high half
            const unsigned w0 = __builtin_amdgcn_perm(bits[st][lv][1], bits[st][lv][0], 0x07060302u);
            const unsigned w1 = __builtin_amdgcn_perm(bits[st][lv][3], bits[st][lv][2], 0x07060302u);
            *reinterpret_cast<uint2 *>(&dst[st * 3 + lv][row][k0]) = make_uint2(w0, w1);
          }
      };
      static_assert(C::la == 4 && C::lb == 4, "bfloat16 tiles: four elements per thread per operand");
      {
        int i, k;
        TileLoad<C, TA, TB>::a_coord(tid, 0, i, k);
        put(Ab[buf], ld.ra, sa, i, k);
      }
      {
        int k, j;
        TileLoad<C, TA, TB>::b_coord(tid, 0, k, j);
        put(Bb[buf], ld.rb, sb, j, k);
      }
    } else {
      ld.store(As[buf], Bs[buf], tid, sa, sb);
    }
  };
  // add the float32 sums into the float64 totals and restart them
  auto fold = [&] {
#pragma unroll
    for (int t = 0; t < TN; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if constexpr (C::BF) {
          const double d1 = double(acc[0][t][r]) + double(acc[1][t][r]);
          const double d2 = double(acc[2][t][r]) + double(acc[3][t][r]);
          const double d3 = double(acc[4][t][r]) + double(acc[5][t][r]);
          totr[t][r] += d1 - d2;
          toti[t][r] += d3 - d1 - d2;
        } else if constexpr (C::G3) {
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
// 5 large with three products per complex step, 6 small with three products on bfloat16 pieces;
// `cfg` >= 0 is a choice made by the autotuner, else FR_GEMM_TILE (s, l, x, p, t, u, b)
// overrides the default for manual tuning runs
int tile_choice(int M, int N, int K, int cfg) {
  if (cfg >= 0 && cfg < kGemmTiles) return cfg;
  static const int forced = [] {
    const char *v = std::getenv("FR_GEMM_TILE");
    if (!v) return -1;
    return v[0] == 's' ? 0 : v[0] == 'l' ? 1 : v[0] == 'x' ? 2 : v[0] == 'p' ? 3 : v[0] == 't' ? 4 : v[0] == 'u' ? 5 : v[0] == 'b' ? 6 : -1;
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
    case 6: return split_for(tiles_of<CfgB>(M, N), K);
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
                 : cfg == 6 ? launch_cfg<CfgB>(gp, stream)
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
