// Register-resident small DFTs and the four-step line FFT.
//
// dft<N, INV>(v): in-place DFT of N values held in registers, natural order
// in and out, by recursive mixed-radix Cooley-Tukey (N = A*B: B DFTs of
// size A over stride-B subsequences, twiddle exp(-+2 pi i b ka / N), A DFTs
// of size B; output index ka + A*kb).  All indices are compile-time, so the
// data stays in VGPRs.  Twiddles are compile-time constants from a double
// precision Taylor series, rounded once to float.
//
// Four-step line FFT of length K = K1*K2 (the classic decomposition
// n = n1*K2 + n2, k = k1 + K1*k2):
//   step 1  thread n2 (< K2) holds x[n1*K2 + n2], n1 < K1, does dft<K1>,
//           multiplies output k1 by W_K^(n2*k1) (FP64-tabulated table),
//   transpose through LDS,
//   step 2  thread k1 (< K1) holds the K2 values of row k1, does dft<K2> and
//           owns outputs X[k1 + K1*k2], k2 < K2.
#pragma once

#include "common.hpp"

namespace pnp {
namespace reg {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_sin(double x) {
  // Taylor series, |x| <= pi: terms shrink fast; 30 terms reach double precision
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// exp(-2 pi i t / N) reduced to |angle| <= pi
constexpr double tw_angle(int t, int N) {
  int r = t % N;
  if (2 * r > N) r -= N;
  return -2.0 * kPi * (double)r / (double)N;
}
template <int N, int T>
struct Tw {
  static constexpr float re = (float)cx_cos(tw_angle(T, N));
  static constexpr float im = (float)cx_sin(tw_angle(T, N));
};

template <bool INV>
__host__ __device__ __forceinline__ float2 mul_tw(float2 v, float wr, float wi) {
  if (INV) wi = -wi;
  return make_float2(v.x * wr - v.y * wi, v.x * wi + v.y * wr);
}

template <bool INV>
__host__ __device__ __forceinline__ float2 mul_mi(float2 v) {
  return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
}

// smallest "first radix" used to split N
template <int N>
struct Split {
  static constexpr int A = (N % 4 == 0 && N != 4 && N != 8) ? 4
                         : (N % 2 == 0 && N != 2 && N != 4 && N != 8) ? 2
                         : (N % 3 == 0 && N != 3) ? 3
                         : (N % 5 == 0 && N != 5) ? 5
                         : N;
};

template <int N, bool INV>
struct DFT;

template <bool INV>
struct DFT<1, INV> {
  template <int S>
  __host__ __device__ __forceinline__ static void run(float2*) {}
};

template <bool INV>
struct DFT<2, INV> {
  template <int S>
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[S];
    v[0] = cadd(a, b);
    v[S] = csub(a, b);
  }
};

template <bool INV>
struct DFT<3, INV> {
  template <int S>
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float h = 0.86602540378443864676f;
    float2 s = cadd(v[S], v[2 * S]);
    float2 d = mul_mi<INV>(csub(v[S], v[2 * S]));
    float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
    v[0] = cadd(v[0], s);
    v[S] = make_float2(m.x + h * d.x, m.y + h * d.y);
    v[2 * S] = make_float2(m.x - h * d.x, m.y - h * d.y);
  }
};

template <bool INV>
struct DFT<4, INV> {
  template <int S>
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 a0 = v[0], a1 = v[S], a2 = v[2 * S], a3 = v[3 * S];
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
    v[0] = cadd(t0, t2);
    v[2 * S] = csub(t0, t2);
    v[S] = cadd(t1, t3);
    v[3 * S] = csub(t1, t3);
  }
};

template <bool INV>
struct DFT<5, INV> {
  template <int S>
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    float2 a0 = v[0];
    float2 sa = cadd(v[S], v[4 * S]), da = csub(v[S], v[4 * S]);
    float2 sb = cadd(v[2 * S], v[3 * S]), db = csub(v[2 * S], v[3 * S]);
    float2 b1 = make_float2(a0.x + c1 * sa.x + c2 * sb.x, a0.y + c1 * sa.y + c2 * sb.y);
    float2 b2 = make_float2(a0.x + c2 * sa.x + c1 * sb.x, a0.y + c2 * sa.y + c1 * sb.y);
    float2 e1 = mul_mi<INV>(make_float2(s1 * da.x + s2 * db.x, s1 * da.y + s2 * db.y));
    float2 e2 = mul_mi<INV>(make_float2(s2 * da.x - s1 * db.x, s2 * da.y - s1 * db.y));
    v[0] = make_float2(a0.x + sa.x + sb.x, a0.y + sa.y + sb.y);
    v[S] = cadd(b1, e1);
    v[4 * S] = csub(b1, e1);
    v[2 * S] = cadd(b2, e2);
    v[3 * S] = csub(b2, e2);
  }
};

template <bool INV>
struct DFT<8, INV> {
  template <int S>
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 e[4] = {v[0], v[2 * S], v[4 * S], v[6 * S]};
    float2 o[4] = {v[S], v[3 * S], v[5 * S], v[7 * S]};
    DFT<4, INV>::template run<1>(e);
    DFT<4, INV>::template run<1>(o);
    const float h = 0.70710678118654752440f;
    float2 w1 = mul_tw<INV>(o[1], h, -h);
    float2 w2 = mul_mi<INV>(o[2]);
    float2 w3 = mul_tw<INV>(o[3], -h, -h);
    v[0] = cadd(e[0], o[0]);
    v[4 * S] = csub(e[0], o[0]);
    v[S] = cadd(e[1], w1);
    v[5 * S] = csub(e[1], w1);
    v[2 * S] = cadd(e[2], w2);
    v[6 * S] = csub(e[2], w2);
    v[3 * S] = cadd(e[3], w3);
    v[7 * S] = csub(e[3], w3);
  }
};

// Generic composite N = A * B (A = Split<N>::A), operating on elements
// v[0], v[S], ..., v[(N-1) S].
template <int N, bool INV>
struct DFT {
  static constexpr int A = Split<N>::A;
  static constexpr int B = N / A;
  static_assert(A > 1 && A < N, "unsupported register DFT size");

  template <int b, int ka, int S>
  __host__ __device__ __forceinline__ static void twiddle(float2* v) {
    if constexpr (b * ka % N != 0) {
      constexpr float wr = Tw<N, b * ka>::re;
      constexpr float wi = Tw<N, b * ka>::im;
      v[(ka * B + b) * S] = mul_tw<INV>(v[(ka * B + b) * S], wr, wi);
    }
  }

  template <int b, int S>
  __host__ __device__ __forceinline__ static void col(float2* v) {
    // DFT of size A over v[(a*B + b) S], a < A  (stride B*S)
    DFT<A, INV>::template run<B * S>(v + b * S);
    // twiddles W_N^{b ka}
    tw_row<b, 0, S>(v);
  }
  template <int b, int ka, int S>
  __host__ __device__ __forceinline__ static void tw_row(float2* v) {
    if constexpr (ka < A) {
      twiddle<b, ka, S>(v);
      tw_row<b, ka + 1, S>(v);
    }
  }
  template <int b, int S>
  __host__ __device__ __forceinline__ static void cols(float2* v) {
    if constexpr (b < B) {
      col<b, S>(v);
      cols<b + 1, S>(v);
    }
  }
  template <int ka, int S>
  __host__ __device__ __forceinline__ static void rows(float2* v) {
    if constexpr (ka < A) {
      // DFT of size B over v[(ka*B + b) S], b < B (contiguous in steps of S)
      DFT<B, INV>::template run<S>(v + ka * B * S);
      rows<ka + 1, S>(v);
    }
  }

  // HZ: inputs a = 1, 2 of every first-level column (the middle half of
  // the sequence) are zero -- a forward transform of a zero-padded line.
  // The size-4 column DFTs of (x0, 0, 0, x3) reduce to x0 +- x3 and
  // x0 -+ i x3 (the general form cannot drop the zero terms itself: x + 0
  // is not x for x = -0 in IEEE arithmetic).
  template <int b, int S>
  __host__ __device__ __forceinline__ static void col_hz(float2* v) {
    float2* c = v + b * S;
    const float2 x0 = c[0], x3 = c[3 * B * S];
    const float2 m = mul_mi<INV>(x3);
    c[0] = cadd(x0, x3);
    c[2 * B * S] = csub(x0, x3);
    c[B * S] = csub(x0, m);
    c[3 * B * S] = cadd(x0, m);
    tw_row<b, 0, S>(v);
  }
  template <int b, int S>
  __host__ __device__ __forceinline__ static void cols_hz(float2* v) {
    if constexpr (b < B) {
      col_hz<b, S>(v);
      cols_hz<b + 1, S>(v);
    }
  }

  template <int S, bool HZ = false>
  __host__ __device__ __forceinline__ static void run(float2* v) {
    if constexpr (HZ) {
      static_assert(A == 4, "zero-padded first level needs a radix-4 split");
      cols_hz<0, S>(v);
    } else {
      cols<0, S>(v);
    }
    rows<0, S>(v);
    // now v[(ka*B + kb) S] holds X[ka + A*kb]; reorder to natural order
    float2 t[N];
#pragma unroll
    for (int ka = 0; ka < A; ++ka)
#pragma unroll
      for (int kb = 0; kb < B; ++kb) t[ka + A * kb] = v[(ka * B + kb) * S];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i * S] = t[i];
  }
};

template <int N, bool INV>
__host__ __device__ __forceinline__ void dft(float2* v) {
  DFT<N, INV>::template run<1>(v);
}

// dft of a line whose middle half (indices N/4 .. 3N/4-1) is zero
template <int N, bool INV>
__host__ __device__ __forceinline__ void dft_halfzero(float2* v) {
  DFT<N, INV>::template run<1, true>(v);
}

}  // namespace reg

// Supported four-step factorisations K = K1 * K2 (K1 >= K2, both <= 32).
// Returns 0 when K has no register path (the LDS Stockham path is used).
inline int four_step_k1(int K) {
  switch (K) {
    case 128: return 16;
    case 192: return 16;
    case 256: return 16;
    case 512: return 32;
    case 640: return 32;
    case 768: return 32;
    case 1024: return 32;
    default: return 0;
  }
}

}  // namespace pnp
