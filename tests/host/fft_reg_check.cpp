// Host harness for the register DFTs and the four-step composition of
// fft_reg.hpp: reads nothing, writes "name re im ..." lines for random
// inputs generated from a fixed LCG; the Python test compares with numpy.
#include <cmath>
#include <cstdio>
#include <vector>

#include "fft_reg.hpp"

using namespace pnp;

static unsigned long long g_state = 12345;
static float rnd() {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (float)((g_state >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;
}

template <int N, bool INV>
static void one() {
  float2 v[N], in[N];
  for (int i = 0; i < N; ++i) in[i] = v[i] = make_float2(rnd(), rnd());
  reg::dft<N, INV>(v);
  printf("dft %d %d", N, INV ? 1 : 0);
  for (int i = 0; i < N; ++i) printf(" %.9g %.9g", in[i].x, in[i].y);
  for (int i = 0; i < N; ++i) printf(" %.9g %.9g", v[i].x, v[i].y);
  printf("\n");
}

// dft of a line whose middle half is zero (the zero-padded forward lines)
template <int N>
static void halfzero() {
  float2 v[N], in[N];
  for (int i = 0; i < N; ++i) {
    const bool pad = i >= N / 4 && i < 3 * N / 4;
    in[i] = v[i] = pad ? make_float2(0.f, 0.f) : make_float2(rnd(), rnd());
  }
  reg::dft_halfzero<N, false>(v);
  printf("hz %d 0", N);
  for (int i = 0; i < N; ++i) printf(" %.9g %.9g", in[i].x, in[i].y);
  for (int i = 0; i < N; ++i) printf(" %.9g %.9g", v[i].x, v[i].y);
  printf("\n");
}

// four-step with a double-tabulated twiddle table, emulating the kernels:
// thread n2 < K2 runs step 1, thread k1 < K1 runs step 2
template <int K1, int K2, bool INV>
static void four() {
  constexpr int K = K1 * K2;
  std::vector<float2> x(K), tw(K), A(K1 * (K2 + 1)), X(K);
  for (int i = 0; i < K; ++i) x[i] = make_float2(rnd(), rnd());
  for (int t = 0; t < K; ++t)
    tw[t] = make_float2((float)std::cos(-2.0 * M_PI * t / K), (float)std::sin(-2.0 * M_PI * t / K));
  for (int n2 = 0; n2 < K2; ++n2) {
    float2 v[K1];
    for (int n1 = 0; n1 < K1; ++n1) v[n1] = x[n1 * K2 + n2];
    reg::dft<K1, INV>(v);
    for (int k1 = 1; k1 < K1; ++k1) {
      float2 w = tw[n2 * k1];
      if (INV) w.y = -w.y;
      v[k1] = cmul(v[k1], w);
    }
    for (int k1 = 0; k1 < K1; ++k1) A[k1 * (K2 + 1) + n2] = v[k1];
  }
  for (int k1 = 0; k1 < K1; ++k1) {
    float2 u[K2];
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = A[k1 * (K2 + 1) + n2];
    reg::dft<K2, INV>(u);
    for (int k2 = 0; k2 < K2; ++k2) X[k1 + K1 * k2] = u[k2];
  }
  printf("four %d %d", K, INV ? 1 : 0);
  for (int i = 0; i < K; ++i) printf(" %.9g %.9g", x[i].x, x[i].y);
  for (int i = 0; i < K; ++i) printf(" %.9g %.9g", X[i].x, X[i].y);
  printf("\n");
}

// Toeplitz column chain as the kernel runs it: forward four-step, multiply
// by a real T[k], inverse with k = k1 + K1*k2, r = r2 + K2*r1 (inverse DFT
// over k2 by thread k1, twiddle exp(+2 pi i k1 r2/K), inverse DFT over k1
// by thread r2).  Prints input, T and y = sum_k T[k] X[k] exp(+2 pi i k r/K).
template <int K1, int K2>
static void toep() {
  constexpr int K = K1 * K2;
  std::vector<float2> x(K), tw(K), A(K1 * (K2 + 1)), B(K2 * (K1 + 1)), Y(K);
  std::vector<float> T(K);
  for (int i = 0; i < K; ++i) x[i] = make_float2(rnd(), rnd());
  for (int i = 0; i < K; ++i) T[i] = rnd();
  for (int t = 0; t < K; ++t)
    tw[t] = make_float2((float)std::cos(-2.0 * M_PI * t / K), (float)std::sin(-2.0 * M_PI * t / K));
  for (int n2 = 0; n2 < K2; ++n2) {
    float2 v[K1];
    for (int n1 = 0; n1 < K1; ++n1) v[n1] = x[n1 * K2 + n2];
    reg::dft<K1, false>(v);
    for (int k1 = 1; k1 < K1; ++k1) v[k1] = cmul(v[k1], tw[n2 * k1]);
    for (int k1 = 0; k1 < K1; ++k1) A[k1 * (K2 + 1) + n2] = v[k1];
  }
  for (int k1 = 0; k1 < K1; ++k1) {
    float2 u[K2];
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = A[k1 * (K2 + 1) + n2];
    reg::dft<K2, false>(u);
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = cscale(u[k2], T[k1 + K1 * k2]);
    reg::dft<K2, true>(u);
    for (int r2 = 1; r2 < K2; ++r2) {
      float2 w = tw[k1 * r2];
      w.y = -w.y;
      u[r2] = cmul(u[r2], w);
    }
    for (int r2 = 0; r2 < K2; ++r2) B[r2 * (K1 + 1) + k1] = u[r2];
  }
  for (int r2 = 0; r2 < K2; ++r2) {
    float2 z[K1];
    for (int k1 = 0; k1 < K1; ++k1) z[k1] = B[r2 * (K1 + 1) + k1];
    reg::dft<K1, true>(z);
    for (int r1 = 0; r1 < K1; ++r1) Y[r2 + K2 * r1] = z[r1];
  }
  printf("toep %d 0", K);
  for (int i = 0; i < K; ++i) printf(" %.9g %.9g", x[i].x, x[i].y);
  for (int i = 0; i < K; ++i) printf(" %.9g 0", T[i]);
  for (int i = 0; i < K; ++i) printf(" %.9g %.9g", Y[i].x, Y[i].y);
  printf("\n");
}

int main() {
  toep<16, 8>(); toep<32, 20>(); toep<32, 24>(); toep<32, 32>();
  one<2, false>(); one<3, false>(); one<4, false>(); one<5, false>(); one<6, false>();
  one<8, false>(); one<10, false>(); one<12, false>(); one<16, false>(); one<20, false>();
  one<24, false>(); one<32, false>();
  one<8, true>(); one<12, true>(); one<20, true>(); one<32, true>();
  four<16, 8, false>(); four<16, 12, false>(); four<16, 16, false>(); four<32, 16, false>();
  four<32, 20, false>(); four<32, 24, false>(); four<32, 32, false>();
  four<16, 8, true>(); four<32, 20, true>(); four<32, 24, true>();
  halfzero<16>(); halfzero<32>();
  return 0;
}
