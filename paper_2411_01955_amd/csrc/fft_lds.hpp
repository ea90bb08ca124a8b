// Batched mixed-radix (8, 4, 2, 5, 3) Stockham FFT over lines held in LDS.
//
// A workgroup transforms `nl` lines of length K that sit in LDS at
// `a + line*LS` (LS >= K is the line stride, padded against bank
// conflicts).  Each stage reads from one LDS buffer and writes the other
// (autosort: natural order in and out, no bit reversal).  Stage with radix R
// after a product Ns of earlier radices: butterfly j (0 <= j < K/R) reads
// x[j + r*K/R], multiplies by exp(-+2*pi*i*(j mod Ns)*r/(Ns*R)) and writes
// its radix-R DFT to x'[(j/Ns)*Ns*R + (j mod Ns) + r*Ns].
//
// Forward = kernel exp(-2*pi*i*j*t/K); inverse = exp(+...) without 1/K.
#pragma once

#include "common.hpp"

namespace pnp {

template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 v) {
  // forward: multiply by -i; inverse: by +i
  return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  const float h = 0.70710678118654752440f;
  // w^1, w^2, w^3 with w = exp(-+2*pi*i/8)
  float2 w1o = INV ? make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y))
                   : make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
  float2 w2o = mul_mi<INV>(o2);
  float2 w3o = INV ? make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y))
                   : make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1o);
  v[5] = csub(e1, w1o);
  v[2] = cadd(e2, w2o);
  v[6] = csub(e2, w2o);
  v[3] = cadd(e3, w3o);
  v[7] = csub(e3, w3o);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
  const float h = 0.86602540378443864676f;  // sqrt(3)/2
  float2 s = cadd(v[1], v[2]);
  float2 d = mul_mi<INV>(csub(v[1], v[2]));
  float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
  v[0] = cadd(v[0], s);
  v[1] = make_float2(m.x + h * d.x, m.y + h * d.y);
  v[2] = make_float2(m.x - h * d.x, m.y - h * d.y);
}

template <bool INV>
__device__ __forceinline__ void dft5(float2* v) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
  float2 a0 = v[0];
  float2 sa = cadd(v[1], v[4]), da = csub(v[1], v[4]);
  float2 sb = cadd(v[2], v[3]), db = csub(v[2], v[3]);
  float2 b1 = make_float2(a0.x + c1 * sa.x + c2 * sb.x, a0.y + c1 * sa.y + c2 * sb.y);
  float2 b2 = make_float2(a0.x + c2 * sa.x + c1 * sb.x, a0.y + c2 * sa.y + c1 * sb.y);
  float2 e1 = mul_mi<INV>(make_float2(s1 * da.x + s2 * db.x, s1 * da.y + s2 * db.y));
  float2 e2 = mul_mi<INV>(make_float2(s2 * da.x - s1 * db.x, s2 * da.y - s1 * db.y));
  v[0] = make_float2(a0.x + sa.x + sb.x, a0.y + sa.y + sb.y);
  v[1] = cadd(b1, e1);
  v[4] = csub(b1, e1);
  v[2] = cadd(b2, e2);
  v[3] = csub(b2, e2);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<INV>(v);
  else dft8<INV>(v);
}

template <int R, bool INV>
__device__ __forceinline__ void stockham_stage(const float2* __restrict__ a, float2* __restrict__ b,
                                               int nl, int K, int LS, int Ns,
                                               const float2* __restrict__ tw) {
  const int KR = K / R;
  const int total = nl * KR;
  const int twstep = K / (Ns * R);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int line = t / KR;
    const int j = t - line * KR;
    const float2* src = a + line * LS;
    float2* dst = b + line * LS;
    const int k = j % Ns;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * KR];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[k * r * twstep];
        if (INV) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    dftR<R, INV>(v);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
}

// Transforms nl lines (stride LS) starting in buffer `a`, using `b` as the
// second buffer.  Returns the buffer holding the result.  Contains
// __syncthreads(); every thread of the block must call it.
template <bool INV>
__device__ float2* lds_fft(float2* a, float2* b, int nl, int LS, const FFTDesc& d) {
  int Ns = 1;
  for (int s = 0; s < d.nrad; ++s) {
    const int R = d.rad[s];
    switch (R) {
      case 8: stockham_stage<8, INV>(a, b, nl, d.K, LS, Ns, d.tw); break;
      case 4: stockham_stage<4, INV>(a, b, nl, d.K, LS, Ns, d.tw); break;
      case 2: stockham_stage<2, INV>(a, b, nl, d.K, LS, Ns, d.tw); break;
      case 5: stockham_stage<5, INV>(a, b, nl, d.K, LS, Ns, d.tw); break;
      default: stockham_stage<3, INV>(a, b, nl, d.K, LS, Ns, d.tw); break;
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

}  // namespace pnp
