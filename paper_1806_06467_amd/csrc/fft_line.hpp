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
// Twiddles come from a float64 table of the N roots exp(-2 pi i m / N) built on the host.
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

template <bool INV, int N, int E, int P, int R, int... Rest>
__device__ __forceinline__ void fft_passes(c32 (&v)[E], c32* __restrict__ lds, int t,
                                           const c64d* __restrict__ root) {
  constexpr int T = N / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide the elements per thread");
  static_assert(N % (P * R) == 0, "plan does not factor N");
  constexpr bool last = sizeof...(Rest) == 0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    c32 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[j + r * NB];
    const int b = t + j * T;
    if constexpr (P > 1) {
      // leg r of butterfly b is twiddled by w_{PR}^{r k}, k = b mod P; w_{PR}^k is root[k N/(PR)]
      constexpr int S = N / (P * R);
      apply_twiddle_powers<R, INV>(u, root[(b % P) * S]);
    }
    DftDir<R, INV>::run(u);
    if constexpr (last) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[j + r * NB] = u[r];
    } else {
      const int base = (b / P) * (P * R) + (b % P);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(base + r * P)] = u[r];
    }
  }
  if constexpr (!last) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[lds_pad(t + T * m)];
    __syncthreads();
    fft_passes<INV, N, E, P * R, Rest...>(v, lds, t, root);
  }
}

// compile-time FFT plan: N = product of Rs, E elements per thread
template <int N_, int E_, int... Rs>
struct Plan {
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int T = N_ / E_;
  // unnormalised DFT of the line, kernel exp(-2 pi i nk/N)
  __device__ __forceinline__ static void forward(c32 (&v)[E_], c32* lds, int t, const c64d* root) {
    fft_passes<false, N_, E_, 1, Rs...>(v, lds, t, root);
  }
  // unnormalised inverse DFT, kernel exp(+2 pi i nk/N)
  __device__ __forceinline__ static void inverse(c32 (&v)[E_], c32* lds, int t, const c64d* root) {
    fft_passes<true, N_, E_, 1, Rs...>(v, lds, t, root);
  }
};

}  // namespace fr
