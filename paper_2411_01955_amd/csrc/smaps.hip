// Coil sensitivity maps from the centre of k-space (Sec. 4.1: a Hamming
// window on the k-space centre, taken to the image domain, masked).
//
// Each sample is weighted by the separable window h(kappa_x) h(kappa_y)
// [h(kappa_z)], kappa = k n / (2 pi) in grid units of its axis,
// h(kappa) = 0.54 + 0.46 cos(pi kappa / c) on |kappa| <= c (c = width/2),
// times the density weight; the low-resolution coil images are the
// adjoint of each coil's weighted data with unit maps; the maps are the
// coil images over their root sum of squares s, zero where
// s <= threshold * max s.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "cg_scalars.hpp"
#include "common.hpp"
#include "trace.hpp"

namespace pnp {

namespace {

__global__ void k_window(long long M, int ndim, const float* __restrict__ traj, int nx, int ny, int nz,
                         float half, const float* __restrict__ dcf, float* __restrict__ w) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int n[3] = {nx, ny, nz};
  float v = dcf ? dcf[m] : 1.f;
  for (int a = 0; a < ndim; ++a) {
    const float kappa = traj[m * ndim + a] * (float)n[a] * 0.15915494309189535f;   // / (2 pi)
    v *= fabsf(kappa) <= half ? 0.54f + 0.46f * cospif(kappa / half) : 0.f;
  }
  w[m] = v;
}

__global__ void k_ones(long long N, float2* __restrict__ o) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    o[i] = make_float2(1.f, 0.f);
}

// s = sqrt(sum_l |z_l|^2) per pixel; block maxima into parts
__global__ void __launch_bounds__(kRedThreads)
k_sos(long long N, int L, const float2* __restrict__ z, float* __restrict__ s, float* __restrict__ parts) {
  __shared__ float sh[kRedThreads / 64];
  float mx = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int l = 0; l < L; ++l) {
      const float2 v = z[(long long)l * N + i];
      acc = fmaf(v.x, v.x, fmaf(v.y, v.y, acc));
    }
    const float r = sqrtf(acc);
    s[i] = r;
    mx = fmaxf(mx, r);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_down(mx, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmaxf(mx, sh[w]);
    parts[blockIdx.x] = fmaxf(mx, sh[0]);
  }
}

// threshold level t = thr * max(parts) (one workgroup)
__global__ void __launch_bounds__(kRedThreads)
k_sos_level(const float* __restrict__ parts, int nb, float thr, float* __restrict__ level) {
  __shared__ float sh[kRedThreads / 64];
  float mx = 0.f;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) mx = fmaxf(mx, parts[b]);
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_down(mx, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmaxf(mx, sh[w]);
    level[0] = thr * fmaxf(mx, sh[0]);
  }
}

// S_l = z_l / s where s > level (and s > 0), else 0; in place
__global__ void k_normalise(long long N, int L, float2* __restrict__ z, const float* __restrict__ s,
                            const float* __restrict__ level) {
  const float t = level[0];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float r = s[i];
    const bool keep = r > t && r > 0.f;
    const float inv = keep ? 1.f / r : 0.f;
    for (int l = 0; l < L; ++l) {
      const long long j = (long long)l * N + i;
      z[j] = keep ? cscale(z[j], inv) : make_float2(0.f, 0.f);
    }
  }
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

unsigned vec_blocks(long long N) {
  const long long b = (N + kRedThreads - 1) / kRedThreads;
  return (unsigned)std::min<long long>(std::max<long long>(b, 1), kRedBlocks);
}

}  // namespace

// coils per adjoint call (2D: the column pass serves them together)
static int smaps_coil_batch(const pnp_plan* p) { return p->ndim == 2 ? 8 : 1; }

size_t smaps_workspace_bytes(const pnp_plan* p) {
  const int64_t N = image_size(p);
  size_t b = al(op_workspace_bytes(p, smaps_coil_batch(p)));
  b += al(sizeof(float2) * N);           // unit map
  b += al(sizeof(float) * p->M);         // window * dcf
  b += al(sizeof(float) * N);            // root sum of squares
  b += al(sizeof(float) * (kRedBlocks + 1));
  return b;
}

void smaps_estimate(const pnp_plan* p, const float2* y, int L, const float* dcf, double width, double threshold,
                    float2* out, void* ws, hipStream_t s) {
  const int64_t N = image_size(p);
  char* c = (char*)ws;
  const int cb = smaps_coil_batch(p);
  const OpWorkspace w = op_workspace(p, cb, c);
  c += al(op_workspace_bytes(p, cb));
  float2* ones = (float2*)c;
  c += al(sizeof(float2) * N);
  float* wts = (float*)c;
  c += al(sizeof(float) * p->M);
  float* sos = (float*)c;
  c += al(sizeof(float) * N);
  float* parts = (float*)c;
  float* level = parts + kRedBlocks;
  const unsigned nb = vec_blocks(N);
  PNP_LAUNCH(k_ones, dim3(nb), dim3(kRedThreads), 0, s, (long long)N, ones);
  PNP_LAUNCH(k_window, dim3((unsigned)((p->M + 255) / 256)), dim3(256), 0, s, (long long)p->M, p->ndim, p->traj,
             p->ax[0].n, p->ax[1].n, p->ax[2].n, (float)(0.5 * width), dcf, wts);
  for (int l = 0; l < L; l += cb)
    op_adjoint_coils(p, y + (long long)l * p->M, std::min(cb, L - l), wts, ones, out + (long long)l * N, w, s);
  PNP_LAUNCH(k_sos, dim3(nb), dim3(kRedThreads), 0, s, (long long)N, L, out, sos, parts);
  PNP_LAUNCH(k_sos_level, dim3(1), dim3(kRedThreads), 0, s, parts, (int)nb, (float)threshold, level);
  PNP_LAUNCH(k_normalise, dim3(nb), dim3(kRedThreads), 0, s, (long long)N, L, out, sos, level);
}

}  // namespace pnp
