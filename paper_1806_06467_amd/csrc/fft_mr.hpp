// Runtime-planned Stockham FFT of one line held in LDS, for line lengths that factor into
// radices up to 16 (2-10, 12, 14, 15, 16).
//
// Pass with radix R after span P (P = product of earlier radices), over L = n / R butterflies
// dealt round-robin to the T threads of the line: butterfly b reads elements b + r L, twiddles
// leg r by w_{P R}^{r (b mod P)}, runs DFT_R, and (after a barrier) writes output r to
// (b / P) P R + (b mod P) + r P. The result is in natural order (autosort). Twiddles come from
// per-pass float32 tables [r - 1][k] built in float64 on the host (mr_twiddle_build).
#pragma once
#include "fft_line.hpp"

namespace fr {

template <int R, bool INV, int T, int MAXN>
__device__ __forceinline__ void mr_pass_r(c32 *lds, int n, int P, const float2 *__restrict__ tw, int t,
                                          const float2 *__restrict__ h, bool hconj) {
  const int nr = n / R;
  constexpr int NBMAX = (MAXN / R + T - 1) / T;
  c32 u[NBMAX][R];
#pragma unroll
  for (int i = 0; i < NBMAX; ++i) {
    const int b = t + i * T;
    if (b < nr) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = b + r * nr;
        c32 x = lds[lds_pad(e)];
        if (h) x = hconj ? cmulc(x, c32{h[e].x, h[e].y}) : cmul(x, c32{h[e].x, h[e].y});
        u[i][r] = x;
      }
      if (P > 1) {
        const int k = b % P;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 q = tw[(r - 1) * P + k];
          u[i][r] = INV ? cmulc(u[i][r], c32{q.x, q.y}) : cmul(u[i][r], c32{q.x, q.y});
        }
      }
      DftDir<R, INV>::run(u[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NBMAX; ++i) {
    const int b = t + i * T;
    if (b < nr) {
      const int base = (b / P) * (P * R) + (b % P);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(base + r * P)] = u[i][r];
    }
  }
  __syncthreads();
}

template <bool INV, int T, int MAXN>
__device__ __forceinline__ void mr_pass(int R, c32 *lds, int n, int P, const float2 *tw, int t,
                                        const float2 *h, bool hconj) {
  switch (R) {
    case 2: mr_pass_r<2, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 3: mr_pass_r<3, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 4: mr_pass_r<4, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 5: mr_pass_r<5, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 6: mr_pass_r<6, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 7: mr_pass_r<7, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 8: mr_pass_r<8, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 9: mr_pass_r<9, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 10: mr_pass_r<10, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 12: mr_pass_r<12, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 14: mr_pass_r<14, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    case 15: mr_pass_r<15, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
    default: mr_pass_r<16, INV, T, MAXN>(lds, n, P, tw, t, h, hconj); break;
  }
}

// Opaque copy of the lane index: without it the compiler hoists the lane-dependent LDS
// addresses of every radix's pass out of the pass loop (and out of persistent loops around it)
// and spills them.
__device__ __forceinline__ int mr_opaque(int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(v));
#endif
  return v;
}

// radix of pass s of a plan packed 5 bits per pass (mr_plan_pack)
__host__ __device__ __forceinline__ int mr_radix(unsigned plan, int s) { return int((plan >> (5 * s)) & 31u); }

// Unnormalised DFT (INV: inverse kernel) of the n-point line in LDS (padded, natural order in
// and out), with a packed plan of npass radices and its twiddle table. With h != null the first pass
// multiplies its inputs by h (conj(h) when hconj): the frequency product of a convolution.
template <bool INV, int T, int MAXN>
__device__ __forceinline__ void mr_fft(c32 *lds, int n, int npass, unsigned plan, const float2 *tw,
                                       int t, const float2 *h, bool hconj) {
  int P = 1;
  for (int s = 0; s < npass; ++s) {
    const int R = mr_radix(plan, s);
    mr_pass<INV, T, MAXN>(R, lds, n, P, tw, mr_opaque(t), s == 0 ? h : nullptr, hconj);
    if (P > 1) tw += (R - 1) * P;
    P *= R;
  }
}

// The same passes with the line length, the radices and the spans known at compile time (the
// plans of the broadband grids): no runtime radix switch, divisions by constants, no bounds
// checks where the butterflies fill the threads. Same twiddle table layout as mr_fft's for the
// same radix order, same arithmetic per butterfly.
template <int N, int R, int P, bool INV, int T>
__device__ __forceinline__ void mr_pass_ct(c32 *lds, const float2 *__restrict__ tw, int t,
                                           const float2 *__restrict__ h, bool hconj) {
  constexpr int NR = N / R;
  constexpr int NB = (NR + T - 1) / T;
  c32 u[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + i * T;
    if (NR % T == 0 || b < NR) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = b + r * NR;
        c32 x = lds[lds_pad(e)];
        if (h) x = hconj ? cmulc(x, c32{h[e].x, h[e].y}) : cmul(x, c32{h[e].x, h[e].y});
        u[i][r] = x;
      }
      if constexpr (P > 1) {
        const int k = b % P;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 q = tw[(r - 1) * P + k];
          u[i][r] = INV ? cmulc(u[i][r], c32{q.x, q.y}) : cmul(u[i][r], c32{q.x, q.y});
        }
      }
      DftDir<R, INV>::run(u[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + i * T;
    if (NR % T == 0 || b < NR) {
      const int base = (b / P) * (P * R) + (b % P);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(base + r * P)] = u[i][r];
    }
  }
  __syncthreads();
}

template <bool INV, int T, int N, int P, int R, int... Rest>
__device__ __forceinline__ void mr_fft_ct(c32 *lds, const float2 *tw, int t, const float2 *h, bool hconj) {
  mr_pass_ct<N, R, P, INV, T>(lds, tw, t, h, hconj);
  if constexpr (sizeof...(Rest) > 0)
    mr_fft_ct<INV, T, N, P * R, Rest...>(lds, tw + (P > 1 ? (R - 1) * P : 0), t, nullptr, false);
}

// a compile-time plan: edge N, radices Rs in pass order
template <int N_, int... Rs>
struct MrCt {
  static constexpr int N = N_;
  static constexpr unsigned packed() {
    unsigned p = 0;
    int s = 0;
    for (int r : {Rs...}) p |= unsigned(r) << (5 * s++);
    return p;
  }
  template <bool INV, int T>
  __device__ __forceinline__ static void fft(c32 *lds, const float2 *tw, int t, const float2 *h, bool hconj) {
    mr_fft_ct<INV, T, N_, 1, Rs...>(lds, tw, t, h, hconj);
  }
};

// Register-resident form of a compile-time plan: the line is held E elements per thread (slot m
// of thread t is element t + T m, T = N / E threads), as in the power-of-two sweeps. The first
// pass (span 1) takes its butterflies from the registers and the last pass leaves its outputs
// in them (in the same slot order), which needs E divisible by the first and the last radix;
// the passes between go through the LDS as above. So a transform costs the LDS traffic of the
// power-of-two plans of the same pass count, and a forward transform, a product in frequency
// and an inverse transform chain without touching the LDS in between. Same twiddle table layout
// and the same arithmetic per butterfly as mr_fft for the same radix order.
// A middle pass through the LDS that holds only its butterflies' inputs across the barrier
// between reading and writing the line: the twiddles are read and the butterflies run after it,
// one at a time (the same arithmetic as mr_pass_ct, fewer registers).
template <int N, int R, int P, bool INV, int T>
__device__ __forceinline__ void mrr_mid_pass(c32 *lds, const float2 *__restrict__ tw, int t) {
  constexpr int NR = N / R;
  constexpr int NB = (NR + T - 1) / T;
  c32 u[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + i * T;
    if (NR % T == 0 || b < NR) {
#pragma unroll
      for (int r = 0; r < R; ++r) u[i][r] = lds[lds_pad(b + r * NR)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + i * T;
    if (NR % T == 0 || b < NR) {
      const int k = b % P;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 q = tw[(r - 1) * P + k];
        u[i][r] = INV ? cmulc(u[i][r], c32{q.x, q.y}) : cmul(u[i][r], c32{q.x, q.y});
      }
      DftDir<R, INV>::run(u[i]);
      const int base = (b / P) * (P * R) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(base + r * P)] = u[i][r];
    }
  }
  __syncthreads();
}

template <int N, int E, bool INV, int P, int R, int... Rest>
__device__ __forceinline__ void mrr_passes(c32 (&v)[E], c32 *lds, int t, const float2 *__restrict__ tw) {
  constexpr int T = N / E;
  if constexpr (sizeof...(Rest) > 0) {
    mrr_mid_pass<N, R, P, INV, T>(lds, tw, t);
    mrr_passes<N, E, INV, P * R, Rest...>(v, lds, t, tw + (R - 1) * P);
  } else {
    // last pass: span P = N / R, butterfly b = t + j T < P reads elements b + r P (slot j + r NB)
    // and leaves output r in the same slot
    static_assert(P * R == N && E % R == 0, "the last radix must divide the elements per thread");
    constexpr int NB = E / R;
    c32 u[NB][R];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < R; ++r) u[j][r] = lds[lds_pad(t + T * (j + r * NB))];
    __syncthreads();  // the line is read out: the LDS is free for the next transform
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = t + j * T;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 q = tw[(r - 1) * P + k];
        u[j][r] = INV ? cmulc(u[j][r], c32{q.x, q.y}) : cmul(u[j][r], c32{q.x, q.y});
      }
      DftDir<R, INV>::run(u[j]);
#pragma unroll
      for (int r = 0; r < R; ++r) v[j + r * NB] = u[j][r];
    }
  }
}

template <int N, int E, bool INV, int R1, int... Rest>
__device__ __forceinline__ void mrr_fft(c32 (&v)[E], c32 *lds, int t, const float2 *__restrict__ tw) {
  constexpr int T = N / E;
  static_assert(N % E == 0 && E % R1 == 0, "the first radix must divide the elements per thread");
  static_assert(sizeof...(Rest) >= 2, "first, middle and last passes");
  // first pass (span 1): butterfly b = t + j T reads elements b + r N / R1 (slot j + r NB) and
  // writes output r to b R1 + r
  constexpr int NB = E / R1;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    c32 u[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) u[r] = v[j + r * NB];
    DftDir<R1, INV>::run(u);
    const int b = t + j * T;
#pragma unroll
    for (int r = 0; r < R1; ++r) lds[lds_pad(b * R1 + r)] = u[r];
  }
  __syncthreads();
  mrr_passes<N, E, INV, R1, Rest...>(v, lds, t, tw);
}

// a register-resident plan: edge N, E elements per thread, radices Rs in pass order
template <int N_, int E_, int... Rs>
struct MrReg {
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int T = N_ / E_;
  static constexpr unsigned packed() {
    unsigned p = 0;
    int s = 0;
    for (int r : {Rs...}) p |= unsigned(r) << (5 * s++);
    return p;
  }
  template <bool INV>
  __device__ __forceinline__ static void fft(c32 (&v)[E_], c32 *lds, int t, const float2 *tw) {
    mrr_fft<N_, E_, INV, Rs...>(v, lds, t, tw);
  }
};

// Host side. Greedy radix plan of an n-point line: the largest supported radix that divides
// what is left, at most maxpass passes; false if n does not factor that way.
inline bool mr_plan_build(int n, int maxn, int maxpass, int *npass, int *radix) {
  static const int rs[] = {16, 15, 14, 12, 10, 9, 8, 7, 6, 5, 4, 3, 2};
  if (n < 2 || n > maxn) return false;
  int left = n, k = 0;
  while (left > 1) {
    int pick = 0;
    for (int r : rs)
      if (left % r == 0) {
        pick = r;
        break;
      }
    if (!pick || k >= maxpass) return false;
    radix[k++] = pick;
    left /= pick;
  }
  *npass = k;
  return true;
}

inline unsigned mr_plan_pack(int npass, const int *radix) {
  unsigned p = 0;
  for (int s = 0; s < npass; ++s) p |= unsigned(radix[s]) << (5 * s);
  return p;
}

// entries of the twiddle table of a plan
inline int mr_twiddle_size(int npass, const int *radix) {
  int P = 1, total = 0;
  for (int s = 0; s < npass; ++s) {
    if (P > 1) total += (radix[s] - 1) * P;
    P *= radix[s];
  }
  return total;
}

// per pass with span P > 1: block [r - 1][k] = exp(-2 pi i r k / (P R)), built in float64 and
// rounded once
inline void mr_twiddle_fill(int npass, const int *radix, float2 *out) {
  int P = 1;
  for (int s = 0; s < npass; ++s) {
    const int R = radix[s];
    if (P > 1) {
      for (int r = 1; r < R; ++r)
        for (int k = 0; k < P; ++k) {
          const long long num = (long long)r * k % (P * R);
          const double turn = -double(num) / double(P * R);
          out[(r - 1) * P + k] = make_float2(float(__builtin_cos(2.0 * kPi * turn)),
                                             float(__builtin_sin(2.0 * kPi * turn)));
        }
      out += (R - 1) * P;
    }
    P *= R;
  }
}

}  // namespace fr
