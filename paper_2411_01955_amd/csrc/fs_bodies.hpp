// Register four-step FFT pass bodies (K = K1*K2, fft_reg.hpp) shared by the
// 2D and 3D operators and the batched kernels: the row passes (pre /
// zero-pad / FFT along x, and inverse FFT / crop / coil sum) and the column
// passes along a strided axis.  Pixel r = i - n/2 of an image axis sits at
// grid index r mod K; grid index j is frequency j (mod K).
#pragma once

#include "common.hpp"
#include "fft_reg.hpp"

namespace pnp {

__device__ __forceinline__ int img_of_grid(int j, int n, int K) {
  // grid index j -> image index i (or -1 when j is in the zero padding)
  const int h = n >> 1;
  if (j < h) return j + h;
  if (j >= K - h) return j - (K - h);
  return -1;
}

__device__ __forceinline__ int grid_of_img(int i, int n, int K) {
  const int r = i - (n >> 1);
  return r < 0 ? r + K : r;
}

// Image input of the forward row pass: the image x, or -- inside CG -- the
// direction update p' = r + beta p computed on the fly (x = p, beta read
// from the device scalars); the workgroups of coil group 0 store p'.
struct ImgIn {
  const float2* x;
  CGUpdate cg;   // cg.r == nullptr: plain image input
};

struct ImgScal {
  float alpha, beta;
};
__device__ __forceinline__ ImgScal img_scal(const ImgIn& in) {
  return in.cg.r ? ImgScal{(float)*in.cg.alpha, (float)*in.cg.beta} : ImgScal{0.f, 0.f};
}
__device__ __forceinline__ float2 img_at(const ImgIn& in, long long pix, ImgScal sc, bool store) {
  if (!in.cg.r) return in.x[pix];
  // every reader needs r' = r - alpha (w + beta s); the storing workgroup
  // also forms and writes p', s', u'
  const CGUpdate& c = in.cg;
  const float2 rv = c.r[pix], sv = c.s[pix], wv = c.w[pix];
  const float2 sn = make_float2(fmaf(sc.beta, sv.x, wv.x), fmaf(sc.beta, sv.y, wv.y));
  const float2 rn = make_float2(fmaf(-sc.alpha, sn.x, rv.x), fmaf(-sc.alpha, sn.y, rv.y));
  if (store) {
    const float2 pv = c.p[pix], uv = c.u[pix];
    const float2 pn = make_float2(fmaf(sc.beta, pv.x, rv.x), fmaf(sc.beta, pv.y, rv.y));
    c.p2[pix] = pn;
    c.s2[pix] = sn;
    c.u2[pix] = make_float2(fmaf(sc.alpha, pn.x, uv.x), fmaf(sc.alpha, pn.y, uv.y));
    c.r2[pix] = rn;
  }
  return rn;
}

template <int K1, int K2>
struct FS {
  static constexpr int K = K1 * K2;
  static constexpr int AS = K2 + 1;                 // LDS row stride of the transpose
  static constexpr int LA = K1 * AS;                // one line's transpose block
  static constexpr int CS = ((LA + 13) / 16) * 16 + 2;   // column stride, = 2 mod 16
  static constexpr int GS = ((K + 13) / 16) * 16 + 2;    // grid column stride, = 2 mod 16
  static constexpr int CSTR = CS > GS ? CS : GS;         // strip LDS per column
};

template <int K1, int K2, bool INV>
__device__ __forceinline__ void fs_twiddle(float2 (&v)[K1], int t, const float2* __restrict__ tw) {
#pragma unroll
  for (int k1 = 1; k1 < K1; ++k1) {
    float2 w = tw[t * k1];
    if (INV) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
}

// Row pass of the forward operator for image row iy and coil group g
// (RC coils, one line of K1 threads each: blockDim = RC * K1); A: RC LA
// blocks of float2 LDS.  Shared by the single-slice, batched and 3D kernels.
template <int K1, int K2, int RC = 4>
__device__ __forceinline__ void rows_fwd_body(const ImgIn& in, const float2* __restrict__ S, int L, int nx,
                                              int ny, const float* __restrict__ dax,
                                              const float* __restrict__ day, const float2* __restrict__ tw,
                                              float2* __restrict__ mid, int iy, int g, float2* A) {
  using F = FS<K1, K2>;
  constexpr int rc = RC;
  const int line = threadIdx.x / K1;
  const int t = threadIdx.x % K1;
  const int l = g * rc + line;
  const bool active = l < L;
  const long long N = (long long)nx * ny;
  float2* Al = A + line * F::LA;
  if (active && t < K2) {
    float2 v[K1];
    const float sy = day ? day[iy] : 1.f;     // no deapodisation table: Toeplitz operator
    const ImgScal bt = img_scal(in);
    const bool store = line == 0 && g == 0;
    const float2* Sl = S ? S + (long long)l * N + (long long)iy * nx : nullptr;
    const long long row0 = (long long)iy * nx;
#pragma unroll
    for (int n1 = 0; n1 < K1; ++n1) {
      const int ix = img_of_grid(n1 * K2 + t, nx, F::K);
      v[n1] = ix >= 0 ? cscale(S ? cmul(Sl[ix], img_at(in, row0 + ix, bt, store))
                                  : img_at(in, row0 + ix, bt, store),
                                (dax ? dax[ix] : 1.f) * sy)
                      : make_float2(0.f, 0.f);
    }
    reg::dft<K1, false>(v);
    fs_twiddle<K1, K2, false>(v, t, tw);
#pragma unroll
    for (int k1 = 0; k1 < K1; ++k1) Al[k1 * F::AS + t] = v[k1];
  }
  __syncthreads();
  if (active) {
    float2 u[K2];
#pragma unroll
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = Al[t * F::AS + n2];
    reg::dft<K2, false>(u);
    float2* dst = mid + ((long long)l * ny + iy) * F::K;
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) dst[t + K1 * k2] = u[k2];
  }
}

// Row pass of the adjoint for image row iy and coil group g: inverse row
// FFT, crop, deapodisation, conj(S_l) and the sum over the group's RC coils
// into part[g]; A: RC LA blocks of float2 LDS.
template <int K1, int K2, int RC = 4>
__device__ __forceinline__ void rows_adj_body(const float2* __restrict__ mid, const float2* __restrict__ S, int L,
                                              int nx, int ny, const float* __restrict__ dax,
                                              const float* __restrict__ day, const float2* __restrict__ tw,
                                              float2* __restrict__ part, int iy, int g, float2* A) {
  using F = FS<K1, K2>;
  constexpr int rc = RC;
  const int line = threadIdx.x / K1;
  const int t = threadIdx.x % K1;
  const int l = g * rc + line;
  const bool active = l < L;
  const long long N = (long long)nx * ny;
  float2* Al = A + line * F::LA;
  if (active && t < K2) {
    float2 v[K1];
    const float2* src = mid + ((long long)l * ny + iy) * F::K;
#pragma unroll
    for (int n1 = 0; n1 < K1; ++n1) v[n1] = src[n1 * K2 + t];
    reg::dft<K1, true>(v);
    fs_twiddle<K1, K2, true>(v, t, tw);
#pragma unroll
    for (int k1 = 0; k1 < K1; ++k1) Al[k1 * F::AS + t] = v[k1];
  }
  __syncthreads();
  float2 u[K2];
  if (active) {
#pragma unroll
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = Al[t * F::AS + n2];
    reg::dft<K2, true>(u);
  }
  __syncthreads();
  // per-coil contributions conj(S_l) * crop(row) into LDS (reusing A), then coil sum
  float2* Z = A;
  if (active) {
    const float2* Sl = S ? S + (long long)l * N + (long long)iy * nx : nullptr;
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) {
      const int ix = img_of_grid(t + K1 * k2, nx, F::K);
      if (ix >= 0) Z[line * nx + ix] = S ? cmulc(Sl[ix], u[k2]) : u[k2];
    }
  }
  __syncthreads();
  const int nl = min(rc, L - g * rc);
  const float sy = day ? day[iy] : 1.f;     // no deapodisation table: Toeplitz operator
  for (int ix = threadIdx.x; ix < nx; ix += blockDim.x) {
    float2 acc = Z[ix];
    for (int li = 1; li < nl; ++li) acc = cadd(acc, Z[li * nx + ix]);
    part[(long long)g * N + (long long)iy * nx + ix] = cscale(acc, (dax ? dax[ix] : 1.f) * sy);
  }
}

// Column passes over a strip of 8 grid columns (one thread column c per
// grid column, threads t < K1 along the column), in registers with LDS
// transposes; `col` points at the strip's column c, grid row j sits at
// col[j * rs].  The column is the zero-padded image of `nimg` rows
// (img_of_grid placement) on the input side of the forward transform and
// on the output side of the inverse one.
//   forward   n = n1*K2 + n2, k = k1 + K1*k2: thread n2 runs the DFT over n1,
//             twiddle, transpose, thread k1 runs the DFT over n2
//             -> u[k2] = X[t + K1*k2]
//   inverse   k = k1 + K1*k2, r = r2 + K2*r1: thread k1 runs the inverse DFT
//             over k2, twiddle exp(+2 pi i k1 r2 / K), transpose, thread r2
//             runs the inverse DFT over k1 -> y[r2 + K2*r1]
// lds: 8 * CS float2.  Every thread of the workgroup must call these.
template <int K1, int K2>
__device__ __forceinline__ void col_fwd(const float2* __restrict__ col, long long rs, int nimg, bool colok,
                                        const float2* __restrict__ tw, float2* lds, float2 (&u)[K2]) {
  using F = FS<K1, K2>;
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  if (colok && t < K2) {
    float2 v[K1];
#pragma unroll
    for (int n1 = 0; n1 < K1; ++n1) {
      const int iy = img_of_grid(n1 * K2 + t, nimg, F::K);
      v[n1] = iy >= 0 ? col[(long long)iy * rs] : make_float2(0.f, 0.f);
    }
    reg::dft<K1, false>(v);
    fs_twiddle<K1, K2, false>(v, t, tw);
#pragma unroll
    for (int k1 = 0; k1 < K1; ++k1) lds[c * F::CS + k1 * F::AS + t] = v[k1];
  }
  __syncthreads();
  if (colok) {
#pragma unroll
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = lds[c * F::CS + t * F::AS + n2];
    reg::dft<K2, false>(u);
  }
  __syncthreads();
}

template <int K1, int K2>
__device__ __forceinline__ void col_inv(float2* __restrict__ col, long long rs, int nimg, bool colok,
                                        const float2* __restrict__ tw, float2* lds, float2 (&u)[K2]) {
  using F = FS<K1, K2>;
  constexpr int AS2 = K1 + 1;          // row stride of the second transpose
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  if (colok) {
    reg::dft<K2, true>(u);
#pragma unroll
    for (int r2 = 1; r2 < K2; ++r2) {
      float2 w = tw[t * r2];
      w.y = -w.y;
      u[r2] = cmul(u[r2], w);
    }
#pragma unroll
    for (int r2 = 0; r2 < K2; ++r2) lds[c * F::CS + r2 * AS2 + t] = u[r2];
  }
  __syncthreads();
  if (colok && t < K2) {
    float2 z[K1];
#pragma unroll
    for (int k1 = 0; k1 < K1; ++k1) z[k1] = lds[c * F::CS + t * AS2 + k1];
    reg::dft<K1, true>(z);
#pragma unroll
    for (int r1 = 0; r1 < K1; ++r1) {
      const int iy = img_of_grid(t + K2 * r1, nimg, F::K);
      if (iy >= 0) col[(long long)iy * rs] = z[r1];
    }
  }
  __syncthreads();
}

// Toeplitz column pass (2D): zero-padded column FFT, multiplication by the
// real transfer function T, inverse FFT, for grid columns [c0, c0 + tile) of
// coil l; only the ny image rows of mid are read and written (in place).
template <int K1, int K2>
__device__ __forceinline__ void cols_toep_body(float2* __restrict__ mid, int ny, int Kx,
                                               const float2* __restrict__ tw, int tile,
                                               const float* __restrict__ T, int c0, int l, float2* lds) {
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  const bool colok = c < tile;
  float2* col = mid + (long long)l * ny * Kx + c0 + c;
  float2 u[K2];
  col_fwd<K1, K2>(col, Kx, ny, colok, tw, lds, u);
  if (colok) {
    const float* Tc = T + c0 + c;
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = cscale(u[k2], Tc[(long long)(t + K1 * k2) * Kx]);
  }
  col_inv<K1, K2>(col, Kx, ny, colok, tw, lds, u);
}

}  // namespace pnp
