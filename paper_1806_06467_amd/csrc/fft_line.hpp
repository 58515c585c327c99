// LDS-staged Stockham FFT of one line of N complex values held by T = N / E threads.
//
// Register-slot convention: thread t holds slots m = 0..E-1, slot m being element t + T*m.
// That is the coalesced global-load pattern, the input pattern of every Stockham pass
// (butterfly b reads b + r*N/R, with b = t + j*T and slot m = j + r*E/R), and the output
// pattern of the last pass. So a forward FFT, a pointwise product in frequency and a second
// FFT chain without any reordering: the spectrum leaves the first transform with slot m
// holding frequency t + T*m, and the second transform takes it from the same registers.
//
// Pass with radix R after span P (P = product of earlier radices): butterfly b twiddles leg r
// by w_{P R}^{r (b mod P)}, runs DFT_R and writes output r to (b / P) P R + (b mod P) + r P.
// Twiddles come from per-pass tables built in float64 on the host (exact to half an ulp).
#pragma once
#include "dft_small.hpp"

namespace fr {

// one float2 of padding every 16 keeps the power-of-two strides of the exchanges spread
// over the LDS banks
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
template <int N>
struct LdsLine {
  static constexpr int size = N + N / 16;
};

// Padded LDS index of output r of butterfly b in a pass of span P and radix R, written as a
// per-thread base plus a compile-time offset per r (so the stores use immediate offsets).
template <int P, int R>
struct PassOut {
  int base;  // padded index of r = 0
  __device__ __forceinline__ explicit PassOut(int b) {
    const int i0 = (b / P) * (P * R) + (b % P);
    base = lds_pad(i0);
  }
  // valid when P % 16 == 0 (the pad of i0 + rP is pad(i0) + 17 rP/16), or P == 1 and
  // 16 % R == 0 with i0 = b R (then (b R + r) / 16 = b R / 16 for r < R)
  __device__ __forceinline__ static constexpr int off(int r) {
    if constexpr (P % 16 == 0) return r * (P + P / 16);
    return r;  // P == 1
  }
  static constexpr bool exact = (P % 16 == 0) || (P == 1 && 16 % R == 0);
};

// Twiddles of one pass for the NB butterflies a thread owns: leg r of butterfly b is
// multiplied by w_{PR}^{r (b mod P)}, read from the pass's float32 (or float64) table laid out
// [r - 1][k], k = b mod P, so that for each leg the lanes of a wavefront read consecutive
// entries (the table is built in float64 on the host; each entry is within half an ulp).
template <int P, int R, int NB, int T, class C = c32, class TW = float2>
struct PassTw {
  // with several butterflies per thread and long lines (32 elements per thread) the twiddles
  // are read per butterfly inside the pass instead (register budget)
  static constexpr bool lazy = NB > 1 && NB * R >= 32;
  C w[lazy ? 1 : NB][R > 1 ? R - 1 : 1];
  __device__ __forceinline__ void load(const TW* __restrict__ tw, int t) {
    if constexpr (P > 1 && !lazy) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int k = (t + j * T) % P;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const TW q = tw[(r - 1) * P + k];
          w[j][r - 1] = {q.x, q.y};
        }
      }
    }
  }
};

template <int R0, int... Rs>
struct FirstOf {
  static constexpr int value = R0;
};

// Pass with radix R after span P. The twiddles of the next pass are loaded before this
// pass's LDS exchange, so their latency overlaps the exchange.
//
// HALF exchanges move the line through an LDS buffer of N/2 (+ padding) in two rounds: the
// outputs at positions below N/2 (butterflies b < N/(2R): threads t < T/2 when each thread owns
// one butterfly, else the first half of each thread's butterflies), then the upper half. Every
// non-last pass has P R <= N/2, so the N/2 boundary never splits a butterfly's outputs, and the
// reading slots split the same way (slot m < E/2 is position t + T m < N/2).
// C: the element type (c32 or c64d); TW: the twiddle table's (float2 or double2)
template <class C, class TW, bool INV, bool HALF, int N, int E, int P, int R, int... Rest>
__device__ __forceinline__ void fft_passes(C (&v)[E], C* __restrict__ lds, int t,
                                           const TW* __restrict__ tw,
                                           const PassTw<P, R, E / R, N / E, C, TW>& cur) {
  constexpr int T = N / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide the elements per thread");
  static_assert(N % (P * R) == 0, "plan does not factor N");
  static_assert(!HALF || NB == 1 || NB % 2 == 0, "half exchanges split each thread's butterflies in two");
  constexpr bool last = sizeof...(Rest) == 0;
  constexpr bool lazy = PassTw<P, R, NB, T>::lazy;
  // outputs of the second half-round, held until the first half has been exchanged
  constexpr int HOLD = !HALF || last ? 1 : (NB == 1 ? 1 : NB / 2);
  C hold[HOLD][R];
  // write output r of butterfly b (positions shifted down by `shift`)
  auto put = [&](int b, int shift, const C (&u)[R]) {
    if constexpr (PassOut<P, R>::exact) {
      const PassOut<P, R> o(b - shift / R);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[o.base + PassOut<P, R>::off(r)] = u[r];
    } else {
      const int base = (b / P) * (P * R) + (b % P) - shift;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(base + r * P)] = u[r];
    }
  };
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    C u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[j + r * NB];
    const int b = t + j * T;
    if constexpr (P > 1) {
      if constexpr (lazy) {
        const int k = b % P;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const TW q = tw[(r - 1) * P + k];
          u[r] = INV ? cmulc(u[r], C{q.x, q.y}) : cmul(u[r], C{q.x, q.y});
        }
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) u[r] = INV ? cmulc(u[r], cur.w[j][r - 1]) : cmul(u[r], cur.w[j][r - 1]);
      }
    }
    DftDir<R, INV>::run(u);
    if constexpr (last) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[j + r * NB] = u[r];
    } else if constexpr (!HALF) {
      put(b, 0, u);
    } else if constexpr (NB == 1) {
      if (t < T / 2) {
        put(b, 0, u);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) hold[0][r] = u[r];
      }
    } else {
      if (j < NB / 2) {
        put(b, 0, u);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) hold[j - NB / 2][r] = u[r];
      }
    }
  }
  if constexpr (!last) {
    constexpr int R2 = FirstOf<Rest...>::value;
    const TW* tw_next = tw + (P > 1 ? (R - 1) * P : 0);
    PassTw<P * R, R2, E / R2, T, C, TW> nxt;
    nxt.load(tw_next, t);
    // read slots [m0, m1), whose positions start at T m0
    auto get = [&](int m0, int m1) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        if (m < m0 || m >= m1) continue;
        if constexpr (T % 16 == 0) {
          v[m] = lds[lds_pad(t) + (m - m0) * (T + T / 16)];
        } else {
          v[m] = lds[lds_pad(t + T * (m - m0))];
        }
      }
    };
    __syncthreads();
    if constexpr (!HALF) {
      get(0, E);
      __syncthreads();
    } else {
      get(0, E / 2);
      __syncthreads();
      if constexpr (NB == 1) {
        if (t >= T / 2) put(t, N / 2, hold[0]);
      } else {
#pragma unroll
        for (int j = NB / 2; j < NB; ++j) put(t + j * T, N / 2, hold[j - NB / 2]);
      }
      __syncthreads();
      get(E / 2, E);
      __syncthreads();
    }
    fft_passes<C, TW, INV, HALF, N, E, P * R, Rest...>(v, lds, t, tw_next, nxt);
  }
}

// float64-built twiddle table of a plan: for each pass with span P > 1 and radix R, the block
// [r - 1][k] = exp(-2 pi i r k / (P R)), r = 1..R-1, k = 0..P-1 (rounded once to float for a
// float2 table, kept in float64 for a double2 table)
inline void tw_store(float2* p, double c, double s) { *p = make_float2(float(c), float(s)); }
inline void tw_store(double2* p, double c, double s) { *p = make_double2(c, s); }
template <int N, int P, int R, int... Rest>
struct TwiddleTable {
  template <class TW>
  static void build(TW* out) {
    if (P > 1) {
      for (int r = 1; r < R; ++r)
        for (int k = 0; k < P; ++k) {
          const long long num = (long long)r * k % (P * R);
          const double turn = -double(num) / double(P * R);
          tw_store(out + (r - 1) * P + k, __builtin_cos(2.0 * kPi * turn), __builtin_sin(2.0 * kPi * turn));
        }
    }
    if constexpr (sizeof...(Rest) > 0) TwiddleTable<N, P * R, Rest...>::build(out + (P > 1 ? (R - 1) * P : 0));
  }
  static constexpr int size() {
    int s = P > 1 ? (R - 1) * P : 0;
    if constexpr (sizeof...(Rest) > 0) s += TwiddleTable<N, P * R, Rest...>::size();
    return s;
  }
};

// compile-time FFT plan: N = product of Rs, E elements per thread
template <int N_, int E_, int... Rs>
struct Plan {
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int T = N_ / E_;
  static constexpr int twiddles = TwiddleTable<N_, 1, Rs...>::size();
  static constexpr int R0 = FirstOf<Rs...>::value;
  template <class TW>
  static void build_twiddles(TW* out) { TwiddleTable<N_, 1, Rs...>::build(out); }
  // unnormalised DFT of the line, kernel exp(-2 pi i nk/N); tw = the plan's twiddle table (float2
  // for c32 elements, double2 for c64d). HALF: exchanges through an LDS line of N/2
  // (LdsLine<N/2>), in two rounds each.
  template <bool HALF = false, class C, class TW>
  __device__ __forceinline__ static void forward(C (&v)[E_], C* lds, int t, const TW* tw) {
    PassTw<1, R0, E_ / R0, N_ / E_, C, TW> none;
    fft_passes<C, TW, false, HALF, N_, E_, 1, Rs...>(v, lds, t, tw, none);
  }
  // unnormalised inverse DFT, kernel exp(+2 pi i nk/N)
  template <bool HALF = false, class C, class TW>
  __device__ __forceinline__ static void inverse(C (&v)[E_], C* lds, int t, const TW* tw) {
    PassTw<1, R0, E_ / R0, N_ / E_, C, TW> none;
    fft_passes<C, TW, true, HALF, N_, E_, 1, Rs...>(v, lds, t, tw, none);
  }
};

}  // namespace fr
