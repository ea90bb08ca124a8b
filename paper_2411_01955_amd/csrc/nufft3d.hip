// Multicoil 3D non-Cartesian operator (Eq. 1 with a 3D trajectory) on the
// register four-step FFT sizes, and its Toeplitz-embedded normal operator.
//
// Layouts (K = 2n per axis, image [nz][ny][nx], coil-major):
//   mid  [L][nz][ny][Kx]   after the x pass (image rows only)
//   g2   [L][nz][Ky][Kx]   after the y pass (image z planes only)
//   grid [L][Kz][Ky][Kx]   the full oversampled grid (gridded operator only)
//
//   forward  A x:  x pass (pre: x * S_l * deapod, zero pad, FFT)  -> mid
//                  y pass (image rows -> all Ky)                  -> g2
//                  z pass (image planes -> all Kz)                -> grid
//                  type-2 interpolation, 6^3 taps per sample     -> y
//   adjoint:       type-1 spread (FP32 atomics into grid), then the inverse
//                  z / y / x passes with crops, deapodisation, conj(S_l) and
//                  the coil-group sums
//   Toeplitz normal operator: x pass -> y pass -> z pass in place on g2
//                  (zero-padded FFT along z, times T, inverse, crop) ->
//                  inverse y pass -> inverse x pass with the coil sums; the
//                  full grid is never formed.
// The transfer function T is the DFT of the point-spread function
// psf[d] = N^{-1} sum_m w_m exp(i <k_m, d>), |d_a| < n_a, evaluated by the
// type-1 gridding of the weights onto a (2n)^3 image.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "fft_reg.hpp"
#include "fs_bodies.hpp"
#include "trace.hpp"

namespace pnp {

namespace {

constexpr int kRowCoils3 = 4;

// Per-thread byte offsets in the 3D passes are 32-bit where every offset of
// the launch fits (up to 256^3 grids), else 64-bit (a coil group's mid
// exceeds 4 GB at 384^3).  HALF: the axis is zero-padded from n = K/2
// (every operator pass); without it the pass transforms a full grid-sized
// array (the transfer function's DFT).
using Off3 = unsigned long long;
inline bool fits32(double max_bytes) { return max_bytes < 4294967296.0 - 1024.0; }

// x pass (forward): rows are the nz*ny image lines
template <int K1, int K2, bool HALF, typename OFF>
__global__ void __launch_bounds__(kRowCoils3 * K1)
k3_rows_fwd(ImgIn in, const float2* __restrict__ S, int L, int nx, int nrows, const float* __restrict__ dax,
            const float* __restrict__ dyz, const float2* __restrict__ tw, float2* __restrict__ mid) {
  __shared__ float2 A[kRowCoils3 * FS<K1, K2>::LA];
  __shared__ float2 X[FS<K1, K2>::K];
  rows_fwd_body<K1, K2, kRowCoils3, HALF, OFF>(in, S, L, nx, nrows, dax, dyz, tw, mid, blockIdx.x, blockIdx.y, A, X);
}

template <int K1, int K2, bool HALF, typename OFF>
__global__ void __launch_bounds__(kRowCoils3 * K1)
k3_rows_adj(const float2* __restrict__ mid, const float2* __restrict__ S, int L, int nx, int nrows,
            const float* __restrict__ dax, const float* __restrict__ dyz, const float2* __restrict__ tw,
            float2* __restrict__ part) {
  __shared__ float2 A[kRowCoils3 * FS<K1, K2>::LA];
  rows_adj_body<K1, K2, kRowCoils3, HALF, OFF>(mid, S, L, nx, nrows, dax, dyz, tw, part, blockIdx.x, blockIdx.y, A);
}

// A set of columns: workgroup (strip, set) works on columns c0 .. c0+7 of
// set = a * nb + b, at offset a * sa + b * sb of its array; grid row j of a
// column sits at j * rs.
struct ColSets {
  int nb;
  long long in_sa, in_sb, out_sa, out_sb, rs_in, rs_out;
};

// forward: zero-padded image rows (nimg) -> all K rows
template <int K1, int K2, bool HALF, typename OFF>
__global__ void __launch_bounds__(8 * K1)
k3_cols_fwd(const float2* __restrict__ in, float2* __restrict__ out, ColSets cs, int nimg,
            const float2* __restrict__ tw) {
  __shared__ float2 lds[8 * FS<K1, K2>::CS];
  const int c = threadIdx.x % 8, t = threadIdx.x / 8;
  const int a = blockIdx.y / cs.nb, b = blockIdx.y % cs.nb;
  const int c0 = blockIdx.x * 8;
  const float2* src = in + a * cs.in_sa + b * cs.in_sb + c0;
  float2* dst = out + a * cs.out_sa + b * cs.out_sb + c0;
  float2 u[K2];
  col_fwd<K1, K2, HALF, OFF>(src, (OFF)cs.rs_in, nimg, true, tw, lds, u);
  const OFF rb = (OFF)cs.rs_out * 8u, cb = (OFF)c * 8u + (OFF)t * rb;
#pragma unroll
  for (int k2 = 0; k2 < K2; ++k2) st_off(dst, cb + (OFF)(K1 * k2) * rb, u[k2]);
}

// inverse: all K rows -> image rows (nimg), cropped
template <int K1, int K2, bool HALF, typename OFF>
__global__ void __launch_bounds__(8 * K1)
k3_cols_inv(const float2* __restrict__ in, float2* __restrict__ out, ColSets cs, int nimg,
            const float2* __restrict__ tw) {
  __shared__ float2 lds[8 * FS<K1, K2>::CS];
  const int c = threadIdx.x % 8, t = threadIdx.x / 8;
  const int a = blockIdx.y / cs.nb, b = blockIdx.y % cs.nb;
  const int c0 = blockIdx.x * 8;
  const float2* src = in + a * cs.in_sa + b * cs.in_sb + c0;
  float2* dst = out + a * cs.out_sa + b * cs.out_sb + c0;
  float2 u[K2];
  const OFF rb = (OFF)cs.rs_in * 8u, cb = (OFF)c * 8u + (OFF)t * rb;
#pragma unroll
  for (int k2 = 0; k2 < K2; ++k2) u[k2] = ld_off(src, cb + (OFF)(K1 * k2) * rb);
  col_inv<K1, K2, HALF, OFF>(dst, (OFF)cs.rs_out, nimg, true, tw, lds, u);
}

// z pass of the Toeplitz operator, in place on g2: sets (coil l, row ky),
// visited in XCD order with the coil fastest (T slices shared in L2)
template <int K1, int K2, typename OFF>
__global__ void __launch_bounds__(8 * K1)
k3_cols_toep(float2* __restrict__ g2, int L, int nz, int Ky, int Kx, const float2* __restrict__ tw,
             const float* __restrict__ T) {
  __shared__ float2 lds[8 * FS<K1, K2>::CS];
  const int c = threadIdx.x % 8, t = threadIdx.x / 8;
  const int nstrips = Kx / 8;
  const int lin = xcd_order(blockIdx.x, gridDim.x);
  const int l = lin % L;
  const int rest = lin / L;                 // = ky * nstrips + strip
  const int ky = rest / nstrips, c0 = (rest % nstrips) * 8;
  const long long plane = (long long)Ky * Kx;
  float2* strip = g2 + (long long)l * nz * plane + (long long)ky * Kx + c0;
  float2 u[K2];
  col_fwd<K1, K2, true, OFF>(strip, (OFF)plane, nz, true, tw, lds, u);
  const float* Ts = T + (long long)ky * Kx + c0;
  const OFF tb = (OFF)plane * 4u, cb = (OFF)c * 4u + (OFF)t * tb;
#pragma unroll
  for (int k2 = 0; k2 < K2; ++k2) u[k2] = cscale(u[k2], ld_off(Ts, cb + (OFF)(K1 * k2) * tb));
  col_inv<K1, K2, true, OFF>(strip, (OFF)plane, nz, true, tw, lds, u);
}

// type-2 interpolation: y[l][m] = scale * sum of the 6^3 taps of grid[l]
__global__ void __launch_bounds__(256)
k3_interp(const float2* __restrict__ grid, int Kx, int Ky, int Kz, long long M, const int4* __restrict__ j0,
          const float* __restrict__ wts, float scale, float2* __restrict__ y) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int l = blockIdx.y;
  const int4 j = j0[m];
  float w[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int t = 0; t < 6; ++t) w[a][t] = wts[(m * 3 + a) * 6 + t];
  const float2* g = grid + (long long)l * Kz * Ky * Kx;
  float2 acc = make_float2(0.f, 0.f);
  for (int tz = 0; tz < 6; ++tz) {
    int z = j.z + tz;
    if (z >= Kz) z -= Kz;
    float2 az = make_float2(0.f, 0.f);
#pragma unroll
    for (int ty = 0; ty < 6; ++ty) {
      int yy = j.y + ty;
      if (yy >= Ky) yy -= Ky;
      const float2* row = g + ((long long)z * Ky + yy) * Kx;
      float2 ay = make_float2(0.f, 0.f);
#pragma unroll
      for (int tx = 0; tx < 6; ++tx) {
        int x = j.x + tx;
        if (x >= Kx) x -= Kx;
        ay = cfma(w[0][tx], row[x], ay);
      }
      az = cfma(w[1][ty], ay, az);
    }
    acc = cfma(w[2][tz], az, acc);
  }
  y[(long long)l * M + m] = cscale(acc, scale);
}

// k-space values in the plan's sorted sample order, coils contiguous:
// ys[i][l] = scale * w_m * y[l][m] for m = sorted_m[i]
__global__ void k3_sort_y(long long M, int L, const float2* __restrict__ y, const float* __restrict__ dcf,
                          const int32_t* __restrict__ sorted_m, float scale, float2* __restrict__ ys) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * L) return;
  const long long i = idx / L;
  const int l = (int)(idx - i * L);
  const int32_t m = sorted_m[i];
  ys[idx] = cscale(y[(long long)l * M + m], scale * (dcf ? dcf[m] : 1.f));
}

// type-1 spread as a gather: grid point g receives from every sample whose
// 6^3 window covers it, i.e. whose first tap lies in [g - 5, g] (mod K) on
// every axis.  The samples are sorted by first-tap cell, so for each of the
// 36 (z, y) tap rows the candidates form one contiguous range of the sorted
// order (two across the x wrap).  Workgroup: 8 consecutive grid points
// along x, 32 coil lanes each (coils >= L idle; blockIdx.y picks the chunk
// of 32 coils).  Every grid point is written once: no atomics, no clearing,
// and a summation order fixed by the plan.
__global__ void __launch_bounds__(256)
k3_gather(const float2* __restrict__ ys, int L, const int32_t* __restrict__ cell_off,
          const int32_t* __restrict__ jx, const float* __restrict__ sw, int Kx, int Ky, int Kz, long long nblocks,
          float2* __restrict__ grid) {
  // workgroups are numbered over x and z of the launch (a 512^3 grid needs
  // more than fit along x); the surplus of the last z row exits at once
  const long long b = (long long)blockIdx.z * gridDim.x + blockIdx.x;
  if (b >= nblocks) return;
  const int lane = threadIdx.x & 31;
  const long long g = b * 8 + (threadIdx.x >> 5);
  const int l = blockIdx.y * 32 + lane;
  const bool lok = l < L;
  const int gx = (int)(g % Kx);
  const int gy = (int)((g / Kx) % Ky);
  const int gz = (int)(g / ((long long)Kx * Ky));
  float ax = 0.f, ay = 0.f;
  for (int tz = 0; tz < 6; ++tz) {
    int cz = gz - tz;
    if (cz < 0) cz += Kz;
    for (int ty = 0; ty < 6; ++ty) {
      int cy = gy - ty;
      if (cy < 0) cy += Ky;
      const long long row = ((long long)cz * Ky + cy) * Kx;
      const int nseg = gx >= 5 ? 1 : 2;
      for (int seg = 0; seg < nseg; ++seg) {
        const int x0 = gx >= 5 ? gx - 5 : (seg == 0 ? 0 : Kx + gx - 5);
        const int x1 = gx >= 5 ? gx : (seg == 0 ? gx : Kx - 1);
        const int s0 = cell_off[row + x0], s1 = cell_off[row + x1 + 1];
        for (int i = s0; i < s1; ++i) {
          int tx = gx - jx[i];
          if (tx < 0) tx += Kx;
          const float* w = sw + (long long)i * 18;
          const float f = w[tx] * w[6 + ty] * w[12 + tz];
          if (lok) {
            const float2 v = ys[(long long)i * L + l];
            ax = fmaf(f, v.x, ax);
            ay = fmaf(f, v.y, ay);
          }
        }
      }
    }
  }
  if (lok) grid[(long long)l * Kx * Ky * Kz + g] = make_float2(ax, ay);
}

__global__ void k3_fill_ones(float2* __restrict__ y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = make_float2(1.f, 0.f);
}

__global__ void k3_sum_groups(const float2* __restrict__ part, int G, long long N, float2* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float2 v = part[i];
  for (int g = 1; g < G; ++g) v = cadd(v, part[(long long)g * N + i]);
  out[i] = v;
}

// T = Re(X) * s
__global__ void k3_take_real(const float2* __restrict__ X, long long n, float s, float* __restrict__ T) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) T[i] = X[i].x * s;
}

// psf[i] = s * adj[i], zero where any image index is 0 (offset d_a = -n)
__global__ void k3_psf_prepare(float2* __restrict__ a, int Nx, int Ny, int Nz, float s) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)Nx * Ny * Nz) return;
  const int x = (int)(i % Nx), y = (int)((i / Nx) % Ny), z = (int)(i / ((long long)Nx * Ny));
  a[i] = (x == 0 || y == 0 || z == 0) ? make_float2(0.f, 0.f) : cscale(a[i], s);
}

// ------------------------------------------------------------- launchers
template <int K1, int K2>
struct F3 {
  static constexpr int K = K1 * K2;
  // largest per-thread byte offsets: a coil group's rows of mid or maps, a
  // column of K rows at the row stride
  static bool rows32(int nx, int nrows) {
    return fits32(8.0 * kRowCoils3 * std::max((double)nx * nrows, (double)nrows * K));
  }
  static bool cols32(long long rs_a, long long rs_b) { return fits32(8.0 * K * (double)std::max(rs_a, rs_b) + 64.0); }

  template <bool HALF, typename OFF>
  static void rows_fwd_t(const ImgIn& in, const float2* S, int L, int nx, int nrows, const float* dax,
                         const float* dyz, const float2* tw, float2* mid, hipStream_t s) {
    const int G = (L + kRowCoils3 - 1) / kRowCoils3;
    PNP_LAUNCH((k3_rows_fwd<K1, K2, HALF, OFF>), dim3(nrows, G), dim3(kRowCoils3 * K1), 0, s, in, S, L, nx, nrows,
               dax, dyz, tw, mid);
  }
  template <bool HALF, typename OFF>
  static void rows_adj_t(const float2* mid, const float2* S, int L, int nx, int nrows, const float* dax,
                         const float* dyz, const float2* tw, float2* part, hipStream_t s) {
    const int G = (L + kRowCoils3 - 1) / kRowCoils3;
    PNP_LAUNCH((k3_rows_adj<K1, K2, HALF, OFF>), dim3(nrows, G), dim3(kRowCoils3 * K1), 0, s, mid, S, L, nx, nrows,
               dax, dyz, tw, part);
  }
  static void rows_fwd(const ImgIn& in, const float2* S, int L, int nx, int nrows, const float* dax,
                       const float* dyz, const float2* tw, float2* mid, hipStream_t s) {
    const bool half = 2 * nx == K, n32 = rows32(nx, nrows);
    if (half && n32) rows_fwd_t<true, unsigned>(in, S, L, nx, nrows, dax, dyz, tw, mid, s);
    else if (half) rows_fwd_t<true, Off3>(in, S, L, nx, nrows, dax, dyz, tw, mid, s);
    else if (n32) rows_fwd_t<false, unsigned>(in, S, L, nx, nrows, dax, dyz, tw, mid, s);
    else rows_fwd_t<false, Off3>(in, S, L, nx, nrows, dax, dyz, tw, mid, s);
  }
  static void rows_adj(const float2* mid, const float2* S, int L, int nx, int nrows, const float* dax,
                       const float* dyz, const float2* tw, float2* part, hipStream_t s) {
    const bool half = 2 * nx == K, n32 = rows32(nx, nrows);
    if (half && n32) rows_adj_t<true, unsigned>(mid, S, L, nx, nrows, dax, dyz, tw, part, s);
    else if (half) rows_adj_t<true, Off3>(mid, S, L, nx, nrows, dax, dyz, tw, part, s);
    else if (n32) rows_adj_t<false, unsigned>(mid, S, L, nx, nrows, dax, dyz, tw, part, s);
    else rows_adj_t<false, Off3>(mid, S, L, nx, nrows, dax, dyz, tw, part, s);
  }
  static void cols_fwd(const float2* in, float2* out, const ColSets& cs, int nsets, int Kc, int nimg,
                       const float2* tw, hipStream_t s) {
    const bool half = 2 * nimg == K, n32 = cols32(cs.rs_in, cs.rs_out);
    const dim3 g(Kc / 8, nsets), b(8 * K1);
    if (half && n32) PNP_LAUNCH((k3_cols_fwd<K1, K2, true, unsigned>), g, b, 0, s, in, out, cs, nimg, tw);
    else if (half) PNP_LAUNCH((k3_cols_fwd<K1, K2, true, Off3>), g, b, 0, s, in, out, cs, nimg, tw);
    else if (n32) PNP_LAUNCH((k3_cols_fwd<K1, K2, false, unsigned>), g, b, 0, s, in, out, cs, nimg, tw);
    else PNP_LAUNCH((k3_cols_fwd<K1, K2, false, Off3>), g, b, 0, s, in, out, cs, nimg, tw);
  }
  static void cols_inv(const float2* in, float2* out, const ColSets& cs, int nsets, int Kc, int nimg,
                       const float2* tw, hipStream_t s) {
    const bool half = 2 * nimg == K, n32 = cols32(cs.rs_in, cs.rs_out);
    const dim3 g(Kc / 8, nsets), b(8 * K1);
    if (half && n32) PNP_LAUNCH((k3_cols_inv<K1, K2, true, unsigned>), g, b, 0, s, in, out, cs, nimg, tw);
    else if (half) PNP_LAUNCH((k3_cols_inv<K1, K2, true, Off3>), g, b, 0, s, in, out, cs, nimg, tw);
    else if (n32) PNP_LAUNCH((k3_cols_inv<K1, K2, false, unsigned>), g, b, 0, s, in, out, cs, nimg, tw);
    else PNP_LAUNCH((k3_cols_inv<K1, K2, false, Off3>), g, b, 0, s, in, out, cs, nimg, tw);
  }
  static void cols_toep(float2* g2, int L, int nz, int Ky, int Kx, const float2* tw, const float* T, hipStream_t s) {
    if (2 * nz != K) fail(PNP_ERR_SHAPE, "3D Toeplitz pass needs a grid twice the image along z");
    const dim3 g(L * Ky * (Kx / 8)), b(8 * K1);
    if (cols32((long long)Ky * Kx, 0))
      PNP_LAUNCH((k3_cols_toep<K1, K2, unsigned>), g, b, 0, s, g2, L, nz, Ky, Kx, tw, T);
    else
      PNP_LAUNCH((k3_cols_toep<K1, K2, Off3>), g, b, 0, s, g2, L, nz, Ky, Kx, tw, T);
  }
};

#define PNP_F3_DISPATCH(K, fn, ...)                                      \
  do {                                                                  \
    switch (K) {                                                        \
      case 128: F3<16, 8>::fn(__VA_ARGS__); break;                      \
      case 192: F3<16, 12>::fn(__VA_ARGS__); break;                     \
      case 256: F3<16, 16>::fn(__VA_ARGS__); break;                     \
      case 512: F3<32, 16>::fn(__VA_ARGS__); break;                     \
      case 640: F3<32, 20>::fn(__VA_ARGS__); break;                     \
      case 768: F3<32, 24>::fn(__VA_ARGS__); break;                     \
      case 1024: F3<32, 32>::fn(__VA_ARGS__); break;                    \
      default: fail(PNP_ERR_UNSUPPORTED, "3D grid size %d has no register FFT", K); \
    }                                                                   \
  } while (0)

bool fs_size(int K) {
  return K == 128 || K == 192 || K == 256 || K == 512 || K == 640 || K == 768 || K == 1024;
}

size_t al3(size_t b) { return (b + 255) & ~(size_t)255; }

// dims of one 3D pass set: image (nx, ny, nz), grid (Kx, Ky, Kz)
struct Dims {
  int nx, ny, nz, Kx, Ky, Kz;
  long long N;
};

Dims dims_of(const pnp_plan* p) {
  Dims d{p->ax[0].n, p->ax[1].n, p->ax[2].n, p->ax[0].K, p->ax[1].K, p->ax[2].K, 0};
  d.N = (long long)d.nx * d.ny * d.nz;
  return d;
}

// x, y and z forward passes for "images" of size (nx, ny, nz) within the
// plan's grids: mid -> g2 -> grid (or g2 only when `to_grid` is false)
void passes_fwd(const pnp_plan* p, const Dims& d, const ImgIn& in, const float2* S, int L, const float* dax,
                const float* dyz, float2* mid, float2* g2, float2* grid, hipStream_t s) {
  PNP_F3_DISPATCH(d.Kx, rows_fwd, in, S, L, d.nx, d.nz * d.ny, dax, dyz, p->ax[0].fft.tw, mid, s);
  // y pass: sets (l, z); mid rows y at stride Kx -> g2 rows ky at stride Kx
  {
    const ColSets cs{d.nz, (long long)d.nz * d.ny * d.Kx, (long long)d.ny * d.Kx,
                     (long long)d.nz * d.Ky * d.Kx, (long long)d.Ky * d.Kx, d.Kx, d.Kx};
    PNP_F3_DISPATCH(d.Ky, cols_fwd, mid, g2, cs, L * d.nz, d.Kx, d.ny, p->ax[1].fft.tw, s);
  }
  if (!grid) return;
  // z pass: sets (l, ky); g2 planes z at stride Ky*Kx -> grid planes kz
  {
    const long long plane = (long long)d.Ky * d.Kx;
    const ColSets cs{d.Ky, (long long)d.nz * plane, d.Kx, (long long)d.Kz * plane, d.Kx, plane, plane};
    PNP_F3_DISPATCH(d.Kz, cols_fwd, g2, grid, cs, L * d.Ky, d.Kx, d.nz, p->ax[2].fft.tw, s);
  }
}

// inverse z (from grid, unless grid is null), y and x passes -> part
void passes_adj(const pnp_plan* p, const Dims& d, const float2* S, int L, const float* dax, const float* dyz,
                const float2* grid, float2* g2, float2* mid, float2* part, hipStream_t s) {
  if (grid) {
    const long long plane = (long long)d.Ky * d.Kx;
    const ColSets cs{d.Ky, (long long)d.Kz * plane, d.Kx, (long long)d.nz * plane, d.Kx, plane, plane};
    PNP_F3_DISPATCH(d.Kz, cols_inv, grid, g2, cs, L * d.Ky, d.Kx, d.nz, p->ax[2].fft.tw, s);
  }
  {
    const ColSets cs{d.nz, (long long)d.nz * d.Ky * d.Kx, (long long)d.Ky * d.Kx,
                     (long long)d.nz * d.ny * d.Kx, (long long)d.ny * d.Kx, d.Kx, d.Kx};
    PNP_F3_DISPATCH(d.Ky, cols_inv, g2, mid, cs, L * d.nz, d.Kx, d.ny, p->ax[1].fft.tw, s);
  }
  PNP_F3_DISPATCH(d.Kx, rows_adj, mid, S, L, d.nx, d.nz * d.ny, dax, dyz, p->ax[0].fft.tw, part, s);
}

}  // namespace

bool plan3_supported(const pnp_plan* p) {
  return p->ndim == 3 && fs_size(p->ax[0].K) && fs_size(p->ax[1].K) && fs_size(p->ax[2].K);
}

static void need3(const pnp_plan* p) {
  if (!plan3_supported(p))
    fail(PNP_ERR_UNSUPPORTED, "3D operators need register-FFT grid sizes (n in 64, 96, 128, 256, 320, 384, 512)");
}

int op3_groups(int L) { return (L + kRowCoils3 - 1) / kRowCoils3; }

size_t op3_workspace_bytes(const pnp_plan* p, int L) {
  const Dims d = dims_of(p);
  size_t b = 0;
  b += al3(sizeof(float2) * (size_t)L * d.nz * d.ny * d.Kx);   // mid
  b += al3(sizeof(float2) * (size_t)L * d.nz * d.Ky * d.Kx);   // g2
  b += al3(sizeof(float2) * (size_t)L * d.Kz * d.Ky * d.Kx);   // grid
  b += al3(sizeof(float2) * (size_t)L * p->M);                 // ytmp
  b += al3(sizeof(float2) * (size_t)op3_groups(L) * d.N);      // part
  b += al3(sizeof(float2) * (size_t)L * p->M);                 // ysort
  return b;
}

OpWorkspace op3_workspace(const pnp_plan* p, int L, void* ws) {
  const Dims d = dims_of(p);
  OpWorkspace w{};
  char* c = (char*)ws;
  w.mid = (float2*)c;
  c += al3(sizeof(float2) * (size_t)L * d.nz * d.ny * d.Kx);
  w.g2 = (float2*)c;
  c += al3(sizeof(float2) * (size_t)L * d.nz * d.Ky * d.Kx);
  w.grid = (float2*)c;
  c += al3(sizeof(float2) * (size_t)L * d.Kz * d.Ky * d.Kx);
  w.ytmp = (float2*)c;
  c += al3(sizeof(float2) * (size_t)L * p->M);
  w.part = (float2*)c;
  c += al3(sizeof(float2) * (size_t)op3_groups(L) * d.N);
  w.ysort = (float2*)c;
  w.bytes = op3_workspace_bytes(p, L);
  return w;
}

void op3_forward(const pnp_plan* p, const float2* x, const float2* smaps, int L, float2* y, const OpWorkspace& w,
                 hipStream_t s) {
  need3(p);
  const Dims d = dims_of(p);
  passes_fwd(p, d, ImgIn{x, CGUpdate{}}, smaps, L, p->ax[0].deapod, p->deapod_yz, w.mid, w.g2, w.grid, s);
  PNP_LAUNCH(k3_interp, dim3((unsigned)((p->M + 255) / 256), L), dim3(256), 0, s, w.grid, d.Kx, d.Ky, d.Kz,
             (long long)p->M, p->j0, p->wts, (float)(1.0 / std::sqrt((double)d.N)), y);
}

// k-space y (or w.ytmp) -> coil-group partials in `dst`
static void adjoint_parts3(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf,
                           float scale, float2* dst, const OpWorkspace& w, hipStream_t s) {
  const Dims d = dims_of(p);
  const long long ML = p->M * L;
  PNP_LAUNCH(k3_sort_y, dim3((unsigned)((ML + 255) / 256)), dim3(256), 0, s, (long long)p->M, L, y, dcf,
             p->sorted_m, scale, w.ysort);
  const long long G = (long long)d.Kx * d.Ky * d.Kz;
  const long long nblocks = G / 8;
  const unsigned bx = (unsigned)std::min<long long>(nblocks, 65536);
  const unsigned bz = (unsigned)((nblocks + bx - 1) / bx);
  PNP_LAUNCH(k3_gather, dim3(bx, (unsigned)((L + 31) / 32), bz), dim3(256), 0, s, w.ysort, L, p->cell_off,
             p->sorted_jx, p->sorted_w, d.Kx, d.Ky, d.Kz, nblocks, w.grid);
  passes_adj(p, d, smaps, L, p->ax[0].deapod, p->deapod_yz, w.grid, w.g2, w.mid, dst, s);
}

void op3_adjoint(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf, float2* x,
                 const OpWorkspace& w, hipStream_t s) {
  need3(p);
  const Dims d = dims_of(p);
  adjoint_parts3(p, y, smaps, L, dcf, (float)(1.0 / std::sqrt((double)d.N)), w.part, w, s);
  PNP_LAUNCH(k3_sum_groups, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, s, w.part, op3_groups(L), d.N, x);
}

void op3_normal_parts(const pnp_plan* p, const NormalIn& in, const float2* smaps, int L, const float* dcf,
                      const OpWorkspace& w, hipStream_t s) {
  need3(p);
  const Dims d = dims_of(p);
  passes_fwd(p, d, ImgIn{in.x, in.cg}, smaps, L, p->ax[0].deapod, p->deapod_yz, w.mid, w.g2, w.grid, s);
  PNP_LAUNCH(k3_interp, dim3((unsigned)((p->M + 255) / 256), L), dim3(256), 0, s, w.grid, d.Kx, d.Ky, d.Kz,
             (long long)p->M, p->j0, p->wts, 1.0f, w.ytmp);
  adjoint_parts3(p, w.ytmp, smaps, L, dcf, (float)(1.0 / (double)d.N), w.part, w, s);
}

void op3_normal_toep_parts(const pnp_toeplitz* tp, const NormalIn& in, const float2* smaps, int L,
                           const OpWorkspace& w, hipStream_t s) {
  const pnp_plan* p = tp->plan;
  need3(p);
  const Dims d = dims_of(p);
  passes_fwd(p, d, ImgIn{in.x, in.cg}, smaps, L, nullptr, nullptr, w.mid, w.g2, nullptr, s);
  PNP_F3_DISPATCH(d.Kz, cols_toep, w.g2, L, d.nz, d.Ky, d.Kx, p->ax[2].fft.tw, tp->T, s);
  passes_adj(p, d, smaps, L, nullptr, nullptr, nullptr, w.g2, w.mid, w.part, s);
}

// T = DFT(psf) / (Kx Ky Kz) with psf from the type-1 gridding of the
// weights onto a (2n)^3 image (a helper plan on the same trajectory).
pnp_toeplitz* toeplitz3_create(const pnp_plan* p, const float* dcf, hipStream_t s) {
  need3(p);
  const Dims d = dims_of(p);
  const int32_t hshape[3] = {d.Kz, d.Ky, d.Kx};   // (2n)^3 image, slowest first
  pnp_plan* hp = plan_create(3, hshape, p->M, p->traj, s);
  void* blk = nullptr;
  float* T = nullptr;
  auto cleanup = [&] {
    if (blk) (void)hipFree(blk);
    plan_destroy(hp);
  };
  try {
    need3(hp);
    const Dims h = dims_of(hp);
    // helper adjoint of the weights (one coil, unit map)
    const size_t hw = op3_workspace_bytes(hp, 1);
    const size_t yb = al3(sizeof(float2) * (size_t)p->M), ab = al3(sizeof(float2) * (size_t)h.N);
    PNP_HIP(hipMalloc(&blk, hw + yb + ab));
    char* c = (char*)blk;
    const OpWorkspace w = op3_workspace(hp, 1, c);
    float2* yw = (float2*)(c + hw);
    float2* psf = (float2*)(c + hw + yb);
    // y = 1: the weights enter through the spread's dcf factor
    PNP_LAUNCH(k3_fill_ones, dim3((unsigned)((p->M + 255) / 256)), dim3(256), 0, s, yw, (long long)p->M);
    adjoint_parts3(hp, yw, nullptr, 1, dcf, (float)(1.0 / std::sqrt((double)h.N)), w.part, w, s);
    // psf[r] = adj[r] * sqrt(N_h) / N, planes d_a = -n zeroed
    PNP_LAUNCH(k3_sum_groups, dim3((unsigned)((h.N + 255) / 256)), dim3(256), 0, s, w.part, 1, h.N, psf);
    PNP_LAUNCH(k3_psf_prepare, dim3((unsigned)((h.N + 255) / 256)), dim3(256), 0, s, psf, h.nx, h.ny, h.nz,
               (float)(std::sqrt((double)h.N) / (double)d.N));
    // DFT of psf on the plan's grid: the psf "image" fills the whole grid
    const Dims f{d.Kx, d.Ky, d.Kz, d.Kx, d.Ky, d.Kz, (long long)d.Kx * d.Ky * d.Kz};
    float2* mid = w.mid;       // needs Kz*Ky*Kx (the helper's mid is larger)
    float2* g2 = w.g2;
    float2* grid = w.grid;
    passes_fwd(p, f, ImgIn{psf, CGUpdate{}}, nullptr, 1, nullptr, nullptr, mid, g2, grid, s);
    PNP_HIP(hipMalloc((void**)&T, sizeof(float) * (size_t)f.N));
    PNP_LAUNCH(k3_take_real, dim3((unsigned)((f.N + 255) / 256)), dim3(256), 0, s, grid, f.N,
               (float)(1.0 / (double)f.N), T);
    PNP_HIP(hipStreamSynchronize(s));
  } catch (...) {
    if (T) (void)hipFree(T);
    cleanup();
    throw;
  }
  cleanup();
  auto* tp = new pnp_toeplitz();
  tp->plan = p;
  tp->T = T;
  return tp;
}

}  // namespace pnp
