// Register-resident small DFTs (radix 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 15, 16) and
// compile-time twiddles.
//
// These are the butterflies of the Cooley-Tukey FFT that the paper relies on for its
// O(n log n) plane transforms (Sec. 1.2). Sign convention: forward kernel exp(-2 pi i nk/R).
// Constants are computed here at compile time from their definition (a Taylor series of
// cos/sin about 0 after reduction to |x| <= pi/4); no library constants are used.
#pragma once
#include <hip/hip_runtime.h>

namespace fr {

struct c32 {
  float x, y;
};

// float64 complex (the float64 sweeps; float64 twiddle powers)
struct c64d {
  double x, y;
};

// complex arithmetic for either element type (c32 or c64d)
template <class C>
__device__ __forceinline__ C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <class C>
__device__ __forceinline__ C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <class C>
__device__ __forceinline__ C cmul(C a, C b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class C>
__device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <class C>
__device__ __forceinline__ C cconj(C a) { return {a.x, -a.y}; }
__device__ __forceinline__ c32 csq(c32 a) { return {a.x * a.x - a.y * a.y, 2.0f * a.x * a.y}; }
__device__ __forceinline__ c32 cscale(c32 a, float s) { return {a.x * s, a.y * s}; }
template <class C>
__device__ __forceinline__ C mul_mi(C a) { return {a.y, -a.x}; }  // a * (-i)
template <class C>
__device__ __forceinline__ C mul_pi(C a) { return {-a.y, a.x}; }  // a * (+i)

// ---- compile-time trig ------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin_small(double x) {  // |x| <= pi/4
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_small(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi k / m for integers (exact octant reduction)
constexpr double ct_cos_turn(long k, long m) {
  k %= m;
  if (k < 0) k += m;
  // reduce to the first octant using symmetries of the circle
  const double t = double(k) / double(m);  // in [0, 1)
  const double q = t * 8.0;
  const int oct = int(q);
  const double f = (t - oct / 8.0) * 2.0 * kPi;  // angle inside the octant, [0, pi/4)
  switch (oct) {
    case 0: return ct_cos_small(f);
    case 1: return ct_sin_small(kPi / 4 - f);
    case 2: return -ct_sin_small(f);
    case 3: return -ct_cos_small(kPi / 4 - f);
    case 4: return -ct_cos_small(f);
    case 5: return -ct_sin_small(kPi / 4 - f);
    case 6: return ct_sin_small(f);
    default: return ct_cos_small(kPi / 4 - f);
  }
}
constexpr double ct_sin_turn(long k, long m) {
  k %= m;
  if (k < 0) k += m;
  const double t = double(k) / double(m);
  const double q = t * 8.0;
  const int oct = int(q);
  const double f = (t - oct / 8.0) * 2.0 * kPi;
  switch (oct) {
    case 0: return ct_sin_small(f);
    case 1: return ct_cos_small(kPi / 4 - f);
    case 2: return ct_cos_small(f);
    case 3: return ct_sin_small(kPi / 4 - f);
    case 4: return -ct_sin_small(f);
    case 5: return -ct_cos_small(kPi / 4 - f);
    case 6: return -ct_cos_small(f);
    default: return -ct_sin_small(kPi / 4 - f);
  }
}

// v * exp(-2 pi i K / M), with the multiples of pi/4 done without multiplications; the
// constants in the element type's precision
template <int K, int M, class C>
__device__ __forceinline__ C twmul(C v) {
  using S = decltype(v.x);
  constexpr int k = ((K % M) + M) % M;
  constexpr S h = S(0.70710678118654752440);
  if constexpr (k == 0) {
    return v;
  } else if constexpr (2 * k == M) {
    return {-v.x, -v.y};
  } else if constexpr (4 * k == M) {
    return mul_mi(v);
  } else if constexpr (4 * k == 3 * M) {
    return mul_pi(v);
  } else if constexpr (8 * k == M) {  // (1 - i)/sqrt2
    return {(v.x + v.y) * h, (v.y - v.x) * h};
  } else if constexpr (8 * k == 3 * M) {  // (-1 - i)/sqrt2
    return {(v.y - v.x) * h, -(v.x + v.y) * h};
  } else if constexpr (8 * k == 5 * M) {  // (-1 + i)/sqrt2
    return {-(v.x + v.y) * h, (v.x - v.y) * h};
  } else if constexpr (8 * k == 7 * M) {  // (1 + i)/sqrt2
    return {(v.x - v.y) * h, (v.x + v.y) * h};
  } else {
    constexpr S c = S(ct_cos_turn(k, M));
    constexpr S s = S(-ct_sin_turn(k, M));
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// ---- small DFTs in place on u[0..R) (natural order in, natural order out) --------------
template <int R>
struct Dft;

template <>
struct Dft<1> {
  template <class C>
  __device__ __forceinline__ static void run(C*) {}
};

template <>
struct Dft<2> {
  template <class C>
  __device__ __forceinline__ static void run(C* u) {
    C a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  template <class C>
  __device__ __forceinline__ static void run(C* u) {
    C t0 = cadd(u[0], u[2]), t1 = csub(u[0], u[2]);
    C t2 = cadd(u[1], u[3]), t3 = csub(u[1], u[3]);
    u[0] = cadd(t0, t2);
    u[2] = csub(t0, t2);
    u[1] = cadd(t1, mul_mi(t3));
    u[3] = csub(t1, mul_mi(t3));
  }
};

template <>
struct Dft<3> {
  template <class C>
  __device__ __forceinline__ static void run(C* u) {
    using S = decltype(u->x);
    constexpr S s3 = S(0.86602540378443864676);  // sqrt(3)/2
    C t = cadd(u[1], u[2]), d = csub(u[1], u[2]);
    C a = u[0];
    C m = {a.x - S(0.5) * t.x, a.y - S(0.5) * t.y};
    C r = {d.x * s3, d.y * s3};
    u[0] = cadd(a, t);
    u[1] = cadd(m, mul_mi(r));
    u[2] = csub(m, mul_mi(r));
  }
};

// odd prime R: pair n with R - n; X_k = x0 + sum s_n cos - i sum d_n sin, X_{R-k} with +i
template <int R>
struct DftOdd {
  template <class C>
  __device__ __forceinline__ static void run(C* u) {
    constexpr int H = (R - 1) / 2;
    C s[H], d[H];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      s[n - 1] = cadd(u[n], u[R - n]);
      d[n - 1] = csub(u[n], u[R - n]);
    }
    C x0 = u[0];
    C sum = x0;
#pragma unroll
    for (int n = 0; n < H; ++n) sum = cadd(sum, s[n]);
    C out[R];
    out[0] = sum;
    run_k<1>(x0, s, d, out);
#pragma unroll
    for (int k = 0; k < R; ++k) u[k] = out[k];
  }
  template <int K, class C>
  __device__ __forceinline__ static void run_k(C x0, const C* s, const C* d, C* out) {
    constexpr int H = (R - 1) / 2;
    if constexpr (K <= H) {
      C a = x0, b = {0, 0};
      acc<K, 1>(a, b, s, d);
      out[K] = cadd(a, mul_mi(b));
      out[R - K] = csub(a, mul_mi(b));
      run_k<K + 1>(x0, s, d, out);
    }
  }
  template <int K, int N1, class C>
  __device__ __forceinline__ static void acc(C& a, C& b, const C* s, const C* d) {
    using S = decltype(a.x);
    constexpr int H = (R - 1) / 2;
    if constexpr (N1 <= H) {
      constexpr S c = S(ct_cos_turn(long(K) * N1, R));
      constexpr S sn = S(ct_sin_turn(long(K) * N1, R));
      a.x += s[N1 - 1].x * c;
      a.y += s[N1 - 1].y * c;
      b.x += d[N1 - 1].x * sn;
      b.y += d[N1 - 1].y * sn;
      acc<K, N1 + 1>(a, b, s, d);
    }
  }
};

template <>
struct Dft<5> : DftOdd<5> {};
template <>
struct Dft<7> : DftOdd<7> {};

// composite R = A * B: n = B*n1 + n2, k = k1 + A*k2
//   step 1: for each n2, DFT_A over n1; twiddle by w_R^(n2 k1); step 2: for each k1, DFT_B over n2
template <int A, int B>
struct DftComposite {
  template <class C>
  __device__ __forceinline__ static void run(C* u) {
    constexpr int R = A * B;
    C t[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      C a[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) a[n1] = u[B * n1 + n2];
      Dft<A>::run(a);
      tw_row<0>(a, n2);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) t[k1 * B + n2] = a[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      C b[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) b[n2] = t[k1 * B + n2];
      Dft<B>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) u[k1 + A * k2] = b[k2];
    }
  }
  // a[k1] *= w_R^(n2 k1); n2 is a loop index that unrolls to a constant
  template <int K1, class C>
  __device__ __forceinline__ static void tw_row(C* a, int n2) {
    if constexpr (K1 < A) {
      a[K1] = tw_dispatch<K1, 0>(a[K1], n2);
      tw_row<K1 + 1>(a, n2);
    }
  }
  template <int K1, int N2, class C>
  __device__ __forceinline__ static C tw_dispatch(C v, int n2) {
    if constexpr (N2 < B) {
      if (n2 == N2) return twmul<K1 * N2, A * B>(v);
      return tw_dispatch<K1, N2 + 1>(v, n2);
    } else {
      return v;
    }
  }
};

template <>
struct Dft<6> : DftComposite<2, 3> {};
template <>
struct Dft<9> : DftComposite<3, 3> {};
template <>
struct Dft<10> : DftComposite<2, 5> {};
template <>
struct Dft<12> : DftComposite<4, 3> {};
template <>
struct Dft<14> : DftComposite<2, 7> {};
template <>
struct Dft<15> : DftComposite<3, 5> {};
template <>
struct Dft<8> : DftComposite<2, 4> {};
template <>
struct Dft<16> : DftComposite<4, 4> {};
template <>
struct Dft<32> : DftComposite<4, 8> {};

// Inverse-direction DFT (kernel exp(+2 pi i nk/R)): X_inv[k] = X_fwd[(R - k) mod R], so the
// forward butterfly is reused and its outputs are renamed (no arithmetic).
template <int R, bool INV>
struct DftDir {
  template <class C>
  __device__ __forceinline__ static void run(C *u) {
    Dft<R>::run(u);
    if constexpr (INV) {
#pragma unroll
      for (int k = 1; k < (R + 1) / 2; ++k) {
        const C t = u[k];
        u[k] = u[R - k];
        u[R - k] = t;
      }
    }
  }
};

// u[r] *= w1^r (or conj(w1)^r for the inverse), r = 1..R-1. The powers are accumulated in
// float64 (full rate on CDNA, like non-packed float32), p_r = p_{r-1} w1, whose rounding
// (~r 1e-16) stays far below float resolution, then rounded once to float: every twiddle is
// within half an ulp from one table value per butterfly, with two float64 values live.
__device__ __forceinline__ c64d dmul(c64d a, c64d b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}

template <bool INV>
__device__ __forceinline__ void twiddle_leg(c32 &u, c64d p) {
  const c32 w = {float(p.x), float(p.y)};
  u = INV ? cmulc(u, w) : cmul(u, w);
}

template <int R, bool INV>
__device__ __forceinline__ void apply_twiddle_powers(c32 *u, c64d w1) {
  c64d p = w1;
#pragma unroll
  for (int r = 1; r < R; ++r) {
    if (r > 1) p = dmul(p, w1);
    twiddle_leg<INV>(u[r], p);
  }
}

// sin and cos of 2 pi t for t in turns: the reduction t - rint(t) to [-1/2, 1/2] is exact in
// float32, then the hardware sine and cosine, which take their argument in turns (measured on
// gfx950 against float64 at every 2^-24 step of [-1/2, 1/2): within 1.3e-7 of the exact values,
// rms 3.5e-8; a degree-9/8 Taylor evaluation on the octant costs about 20 VALU instructions per
// pair against two transcendental issues here).
__device__ __forceinline__ void sincos_turns(float t, float *s, float *c) {
  t -= rintf(t);
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}

}  // namespace fr
