// Toeplitz embedding of the normal operator A^H D_w A (2D and 3D).
//
// With the orthonormal NDFT of Eq. 1 and the DCF weighting,
//   (F^H D_w F z)[r] = sum_{r'} psf[r - r'] z[r'],
//   psf[d] = N^{-1} sum_m w_m exp(+i <k_m, d>),   d in [-(n-1), n-1]^2,
// a linear convolution.  Embedded circularly in the 2n x 2n grid it becomes
//   F^H D_w F z = crop( IFFT( T * FFT( pad(z) ) ) ),
//   T[j] = sum_d psf[d] exp(-2 pi i <j, d>/K)
//        = N^{-1} sum_m w_m Dx(kx_m - 2 pi jx/Kx) Dy(ky_m - 2 pi jy/Ky),
// with the symmetric Dirichlet kernel D(t) = sum_{d=-(n-1)}^{n-1} exp(i d t)
// = sin((n - 1/2) t) / sin(t/2), which is real, so T is real.  T is formed
// once per (trajectory, DCF) in FP64 -- per-axis Dirichlet tables and one
// real GEMM over the samples -- then scaled by 1/(Kx Ky) (the unnormalised
// inverse FFT) and rounded to FP32.  No Kaiser-Bessel approximation enters:
// the Toeplitz normal operator equals the exact one up to FP32 rounding.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "trace.hpp"

namespace pnp {

namespace {

// D[j][m] for one axis (FP64), j < K
__global__ void k_dirichlet(const float* __restrict__ traj, long long M, int ndim, int axis, int n, int K,
                            double* __restrict__ D) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)K * M) return;
  const int j = (int)(t / M);
  const long long m = t - (long long)j * M;
  double th = (double)traj[m * ndim + axis] - 2.0 * M_PI * (double)j / (double)K;
  // reduce to (-pi, pi]
  th = th - 2.0 * M_PI * rint(th / (2.0 * M_PI));
  const double h = 0.5 * th;
  const double sh = sin(h);
  double v;
  if (fabs(sh) < 1e-12) {
    v = 2.0 * n - 1.0;
  } else {
    v = sin((2.0 * n - 1.0) * h) / sh;
  }
  D[t] = v;
}

// T[jy][jx] = scale * sum_m w_m Dy[jy][m] Dx[jx][m]   (FP64, tiled)
constexpr int kTile = 32;
__global__ void __launch_bounds__(256)
k_psf_gemm(const double* __restrict__ Dy, const double* __restrict__ Dx, const float* __restrict__ w,
           long long M, int Ky, int Kx, double scale, float* __restrict__ T) {
  __shared__ double Ay[kTile][kTile + 1];
  __shared__ double Ax[kTile][kTile + 1];
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;   // 16x16 threads, 2x2 outputs each
  const int jy0 = blockIdx.y * kTile, jx0 = blockIdx.x * kTile;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (long long m0 = 0; m0 < M; m0 += kTile) {
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
      const int r = i / kTile, c = i % kTile;
      const long long m = m0 + c;
      const bool ok = m < M;
      const double wm = ok ? (w ? (double)w[m] : 1.0) : 0.0;
      Ay[r][c] = (ok && jy0 + r < Ky) ? Dy[(long long)(jy0 + r) * M + m] * wm : 0.0;
      Ax[r][c] = (ok && jx0 + r < Kx) ? Dx[(long long)(jx0 + r) * M + m] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < kTile; ++c) {
      const double a0 = Ay[ty][c], a1 = Ay[ty + 16][c];
      const double b0 = Ax[tx][c], b1 = Ax[tx + 16][c];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int jy = jy0 + ty + 16 * a, jx = jx0 + tx + 16 * b;
      if (jy < Ky && jx < Kx) T[(long long)jy * Kx + jx] = (float)(acc[a][b] * scale);
    }
}

// ------------------------------------------------------------------ 3D
// The same construction with three axes:
//   T[jz][jy][jx] = N^{-1} sum_m w_m Dz(kz_m - 2 pi jz/Kz) Dy(ky_m - 2 pi jy/Ky) Dx(kx_m - 2 pi jx/Kx)
// scaled by 1/(Kx Ky Kz).  The tables are stored sample-major (Dt[m][j],
// FP64) so that a chunk of samples loads contiguous rows, and the
// contraction over samples is a GEMM whose left operand
// A[(jz, jy)][m] = w_m Dz[m][jz] Dy[m][jy] is formed while it is staged.

// Dt[m][j] for one axis (FP64), j < K
__global__ void k_dirichlet_t(const float* __restrict__ traj, long long M, int ndim, int axis, int n, int K,
                              double* __restrict__ Dt) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)K * M) return;
  const long long m = t / K;
  const int j = (int)(t - m * K);
  double th = (double)traj[m * ndim + axis] - 2.0 * M_PI * (double)j / (double)K;
  th = th - 2.0 * M_PI * rint(th / (2.0 * M_PI));
  const double h = 0.5 * th;
  const double sh = sin(h);
  Dt[t] = fabs(sh) < 1e-12 ? 2.0 * n - 1.0 : sin((2.0 * n - 1.0) * h) / sh;
}

// T[row][jx] = scale * sum_m A[row][m] Dx[m][jx], row = jz*Ky + jy: a
// 128 x 128 output tile per workgroup, 8 x 8 FP64 accumulators per thread
// (rows ty + 16 i, columns tx + 16 j), samples in chunks of 16 through LDS.
constexpr int kP3 = 128;
constexpr int kP3M = 16;
__global__ void __launch_bounds__(256)
k_psf3_gemm(const double* __restrict__ Dz, const double* __restrict__ Dy, const double* __restrict__ Dx,
            const float* __restrict__ w, long long M, int Kz, int Ky, int Kx, double scale,
            float* __restrict__ T) {
  __shared__ double As[kP3M][kP3];
  __shared__ double Bs[kP3M][kP3];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const long long R = (long long)Kz * Ky;
  const long long r0 = (long long)blockIdx.y * kP3;
  const int c0 = blockIdx.x * kP3;
  double acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
  for (long long m0 = 0; m0 < M; m0 += kP3M) {
    // stage 16 samples: consecutive threads take consecutive rows / columns
    for (int i = threadIdx.x; i < kP3 * kP3M; i += 256) {
      const int mm = i / kP3, r = i % kP3;
      const long long m = m0 + mm;
      const long long row = r0 + r;
      double a = 0.0, b = 0.0;
      if (m < M) {
        if (row < R) {
          const int jz = (int)(row / Ky), jy = (int)(row - (long long)jz * Ky);
          a = (w ? (double)w[m] : 1.0) * Dz[m * Kz + jz] * Dy[m * Ky + jy];
        }
        if (c0 + r < Kx) b = Dx[m * Kx + c0 + r];
      }
      As[mm][r] = a;
      Bs[mm][r] = b;
    }
    __syncthreads();
#pragma unroll 4
    for (int mm = 0; mm < kP3M; ++mm) {
      double a[8], b[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = As[mm][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = Bs[mm][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const long long row = r0 + ty + 16 * i;
    if (row >= R) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int col = c0 + tx + 16 * j;
      if (col < Kx) T[row * Kx + col] = (float)(acc[i][j] * scale);
    }
  }
}

pnp_toeplitz* toeplitz3_create_exact(const pnp_plan* p, const float* traj, const float* dcf, hipStream_t s) {
  auto* tp = new pnp_toeplitz();
  tp->plan = p;
  tp->T = nullptr;
  const int nx = p->ax[0].n, ny = p->ax[1].n, nz = p->ax[2].n;
  const int Kx = p->ax[0].K, Ky = p->ax[1].K, Kz = p->ax[2].K;
  const long long M = p->M;
  struct Tmp {
    double* ptr = nullptr;
    ~Tmp() { if (ptr) (void)hipFree(ptr); }
  } tmp;
  try {
    PNP_HIP(hipMalloc((void**)&tp->T, sizeof(float) * (size_t)Kx * Ky * Kz));
    PNP_HIP(hipMalloc((void**)&tmp.ptr, sizeof(double) * (size_t)(Kx + Ky + Kz) * M));
    double* Dx = tmp.ptr;
    double* Dy = Dx + (size_t)Kx * M;
    double* Dz = Dy + (size_t)Ky * M;
    const int ns[3] = {nx, ny, nz}, Ks[3] = {Kx, Ky, Kz};
    double* Ds[3] = {Dx, Dy, Dz};
    for (int a = 0; a < 3; ++a) {
      const long long tot = (long long)Ks[a] * M;
      PNP_LAUNCH(k_dirichlet_t, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, traj, M, 3, a, ns[a], Ks[a],
                 Ds[a]);
    }
    const double scale = 1.0 / ((double)nx * ny * nz) / ((double)Kx * Ky * Kz);
    const long long R = (long long)Kz * Ky;
    PNP_LAUNCH(k_psf3_gemm, dim3((unsigned)((Kx + kP3 - 1) / kP3), (unsigned)((R + kP3 - 1) / kP3)), dim3(256), 0,
               s, Dz, Dy, Dx, dcf, M, Kz, Ky, Kx, scale, tp->T);
    PNP_HIP(hipStreamSynchronize(s));
  } catch (...) {
    if (tp->T) (void)hipFree(tp->T);
    delete tp;
    throw;
  }
  return tp;
}

}  // namespace

pnp_toeplitz* toeplitz_create(const pnp_plan* p, const float* traj, const float* dcf, hipStream_t s) {
  if (!toeplitz_supported(p))
    fail(PNP_ERR_UNSUPPORTED, "the Toeplitz normal operator needs grid sides in "
                              "{128, 192, 256, 512, 640, 768, 1024}");
  if (p->ndim == 3) return toeplitz3_create_exact(p, traj, dcf, s);
  pnp_toeplitz* tp = new pnp_toeplitz();
  tp->plan = p;
  tp->T = nullptr;
  const int nx = p->ax[0].n, ny = p->ax[1].n, Kx = p->ax[0].K, Ky = p->ax[1].K;
  const long long M = p->M;
  struct Tmp {
    double* ptr = nullptr;
    ~Tmp() { if (ptr) (void)hipFree(ptr); }
  } tmp;
  try {
    PNP_HIP(hipMalloc((void**)&tp->T, sizeof(float) * (size_t)Kx * Ky));
    PNP_HIP(hipMalloc((void**)&tmp.ptr, sizeof(double) * (size_t)(Kx + Ky) * M));
    double* Dx = tmp.ptr;
    double* Dy = tmp.ptr + (size_t)Kx * M;
    const long long tx = (long long)Kx * M, ty = (long long)Ky * M;
    k_dirichlet<<<(unsigned)((tx + 255) / 256), 256, 0, s>>>(traj, M, 2, 0, nx, Kx, Dx);
    PNP_CHECK_LAUNCH();
    k_dirichlet<<<(unsigned)((ty + 255) / 256), 256, 0, s>>>(traj, M, 2, 1, ny, Ky, Dy);
    PNP_CHECK_LAUNCH();
    const double scale = 1.0 / ((double)nx * ny) / ((double)Kx * Ky);
    k_psf_gemm<<<dim3((Kx + kTile - 1) / kTile, (Ky + kTile - 1) / kTile), 256, 0, s>>>(Dy, Dx, dcf, M, Ky,
                                                                                       Kx, scale, tp->T);
    PNP_CHECK_LAUNCH();
    PNP_HIP(hipStreamSynchronize(s));
  } catch (...) {
    if (tp->T) (void)hipFree(tp->T);
    delete tp;
    throw;
  }
  return tp;
}

void toeplitz_destroy(pnp_toeplitz* tp) {
  if (!tp) return;
  if (tp->T) (void)hipFree(tp->T);
  delete tp;
}

}  // namespace pnp
