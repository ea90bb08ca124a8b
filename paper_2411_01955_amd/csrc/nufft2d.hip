// Multicoil 2D non-Cartesian operator by Kaiser-Bessel gridding, with every
// step fused so that the oversampled grid never travels through HBM:
//
//   forward  A x   (Eq. 1, y_l = F_Omega S_l x)
//     k_rows_fwd       pre (x * S_l * deapod) + zero pad + row FFT (along x)
//                      -> mid[l][iy][Kx]       (only the ny image rows exist)
//     k_cols_fwd_interp  strip of `tile` grid columns: column FFT (along y)
//                      in LDS, then type-2 interpolation of the samples whose
//                      footprint touches the strip -> per-entry partial sums
//     k_gather_entries   y_l[m] = N^{-1/2} * sum of the sample's partials
//   adjoint  A^H D_w y
//     k_cols_adj_spread  strip: type-1 spread of w_m y_l[m] into LDS with LDS
//                      atomics, column inverse FFT, keep the ny image rows
//                      -> mid[l][iy][Kx]
//     k_rows_adj       row inverse FFT, crop, deapod, conj(S_l), coil sum
//                      -> per-coil-group partial images
//     k_sum_groups     out = N^{-1/2} sum over coil groups
//
// Pixel r = i - n/2 sits at grid index r mod K; grid index j is frequency
// j (mod K).  Kernel weights and deapodisation come from the plan.
#include <algorithm>

#include "common.hpp"
#include "fft_lds.hpp"

namespace pnp {

namespace {

constexpr int kThreads = 256;
constexpr int kRowCoils = 4;      // coils per workgroup in the row passes

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

__global__ void __launch_bounds__(kThreads)
k_rows_fwd(const float2* __restrict__ x, const float2* __restrict__ S, int L, int nx, int ny,
           const float* __restrict__ dax, const float* __restrict__ day, FFTDesc fd,
           float2* __restrict__ mid) {
  extern __shared__ float2 lds[];
  const int Kx = fd.K;
  const int iy = blockIdx.x;
  const int l0 = blockIdx.y * kRowCoils;
  const int nl = min(kRowCoils, L - l0);
  const long long N = (long long)nx * ny;
  float2* a = lds;
  float2* b = lds + kRowCoils * Kx;
  const float sy = day[iy];
  for (int t = threadIdx.x; t < nl * Kx; t += blockDim.x) {
    const int li = t / Kx;
    const int j = t - li * Kx;
    const int ix = img_of_grid(j, nx, Kx);
    float2 v = make_float2(0.f, 0.f);
    if (ix >= 0) {
      const long long pix = (long long)iy * nx + ix;
      v = cscale(cmul(S[(long long)(l0 + li) * N + pix], x[pix]), dax[ix] * sy);
    }
    a[li * Kx + j] = v;
  }
  __syncthreads();
  const float2* r = lds_fft<false>(a, b, nl, Kx, fd);
  for (int t = threadIdx.x; t < nl * Kx; t += blockDim.x) {
    const int li = t / Kx;
    const int j = t - li * Kx;
    mid[((long long)(l0 + li) * ny + iy) * Kx + j] = r[li * Kx + j];
  }
}

__global__ void __launch_bounds__(kThreads)
k_cols_fwd_interp(const float2* __restrict__ mid, int nx, int ny, int Kx, FFTDesc fd, int tile,
                  int LS, const int* __restrict__ tile_off, const int* __restrict__ ent_sample,
                  const int4* __restrict__ j0, const float* __restrict__ wts, long long E,
                  float2* __restrict__ ypart) {
  extern __shared__ float2 lds[];
  const int Ky = fd.K;
  const int s = blockIdx.x;
  const int l = blockIdx.y;
  float2* a = lds;
  float2* b = lds + tile * LS;
  const int c0 = s * tile;
  for (int t = threadIdx.x; t < tile * Ky; t += blockDim.x) {
    const int c = t % tile;
    const int jy = t / tile;
    const int iy = img_of_grid(jy, ny, Ky);
    float2 v = make_float2(0.f, 0.f);
    if (iy >= 0) v = mid[((long long)l * ny + iy) * Kx + c0 + c];
    a[c * LS + jy] = v;
  }
  __syncthreads();
  const float2* g = lds_fft<false>(a, b, tile, LS, fd);
  const int e0 = tile_off[s], e1 = tile_off[s + 1];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int m = ent_sample[e];
    const int4 jj = j0[m];
    const float* w = wts + (long long)m * 12;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int ta = 0; ta < 6; ++ta) {
      int col = jj.x + ta;
      if (col >= Kx) col -= Kx;
      const int c = col - c0;
      if ((unsigned)c < (unsigned)tile) {
        float2 sum = make_float2(0.f, 0.f);
#pragma unroll
        for (int tb = 0; tb < 6; ++tb) {
          int row = jj.y + tb;
          if (row >= Ky) row -= Ky;
          sum = cfma(w[6 + tb], g[c * LS + row], sum);
        }
        acc = cfma(w[ta], sum, acc);
      }
    }
    ypart[(long long)l * E + e] = acc;
  }
}

__global__ void k_gather_entries(const float2* __restrict__ ypart, const int* __restrict__ sample_ent,
                                 long long M, long long E, int L, float scale, float2* __restrict__ y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * L) return;
  const int l = (int)(t / M);
  const long long m = t - (long long)l * M;
  const int e0 = sample_ent[m * 2];
  const int e1 = sample_ent[m * 2 + 1];
  float2 v = make_float2(0.f, 0.f);
  if (e0 >= 0) v = ypart[(long long)l * E + e0];
  if (e1 >= 0) v = cadd(v, ypart[(long long)l * E + e1]);
  y[t] = cscale(v, scale);
}

__global__ void __launch_bounds__(kThreads)
k_cols_adj_spread(const float2* __restrict__ y, const float* __restrict__ dcf, float scale,
                  long long M, int nx, int ny, int Kx, FFTDesc fd, int tile, int LS,
                  const int* __restrict__ tile_off, const int* __restrict__ ent_sample,
                  const int4* __restrict__ j0, const float* __restrict__ wts,
                  float2* __restrict__ mid) {
  extern __shared__ float2 lds[];
  const int Ky = fd.K;
  const int s = blockIdx.x;
  const int l = blockIdx.y;
  float2* a = lds;
  float2* b = lds + tile * LS;
  const int c0 = s * tile;
  for (int t = threadIdx.x; t < tile * LS; t += blockDim.x) a[t] = make_float2(0.f, 0.f);
  __syncthreads();
  const int e0 = tile_off[s], e1 = tile_off[s + 1];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int m = ent_sample[e];
    const int4 jj = j0[m];
    const float* w = wts + (long long)m * 12;
    float2 v = y[(long long)l * M + m];
    const float sc = dcf ? dcf[m] * scale : scale;
    v = cscale(v, sc);
#pragma unroll
    for (int ta = 0; ta < 6; ++ta) {
      int col = jj.x + ta;
      if (col >= Kx) col -= Kx;
      const int c = col - c0;
      if ((unsigned)c < (unsigned)tile) {
        const float2 vx = cscale(v, w[ta]);
#pragma unroll
        for (int tb = 0; tb < 6; ++tb) {
          int row = jj.y + tb;
          if (row >= Ky) row -= Ky;
          float* dst = reinterpret_cast<float*>(&a[c * LS + row]);
          atomicAdd(dst, vx.x * w[6 + tb]);
          atomicAdd(dst + 1, vx.y * w[6 + tb]);
        }
      }
    }
  }
  __syncthreads();
  const float2* g = lds_fft<true>(a, b, tile, LS, fd);
  for (int t = threadIdx.x; t < tile * ny; t += blockDim.x) {
    const int c = t % tile;
    const int iy = t / tile;
    const int jy = grid_of_img(iy, ny, Ky);
    mid[((long long)l * ny + iy) * Kx + c0 + c] = g[c * LS + jy];
  }
}

__global__ void __launch_bounds__(kThreads)
k_rows_adj(const float2* __restrict__ mid, const float2* __restrict__ S, int L, int nx, int ny,
           const float* __restrict__ dax, const float* __restrict__ day, FFTDesc fd, float scale,
           float2* __restrict__ part) {
  extern __shared__ float2 lds[];
  const int Kx = fd.K;
  const int iy = blockIdx.x;
  const int g = blockIdx.y;
  const int l0 = g * kRowCoils;
  const int nl = min(kRowCoils, L - l0);
  const long long N = (long long)nx * ny;
  float2* a = lds;
  float2* b = lds + kRowCoils * Kx;
  for (int t = threadIdx.x; t < nl * Kx; t += blockDim.x) {
    const int li = t / Kx;
    const int j = t - li * Kx;
    a[li * Kx + j] = mid[((long long)(l0 + li) * ny + iy) * Kx + j];
  }
  __syncthreads();
  const float2* r = lds_fft<true>(a, b, nl, Kx, fd);
  const float sy = day[iy] * scale;
  for (int ix = threadIdx.x; ix < nx; ix += blockDim.x) {
    const int jx = grid_of_img(ix, nx, Kx);
    const long long pix = (long long)iy * nx + ix;
    float2 acc = make_float2(0.f, 0.f);
    for (int li = 0; li < nl; ++li) {
      const float2 sv = S[(long long)(l0 + li) * N + pix];
      const float2 gv = r[li * Kx + jx];
      acc = cadd(acc, cmulc(sv, gv));
    }
    part[(long long)g * N + pix] = cscale(acc, dax[ix] * sy);
  }
}

__global__ void k_sum_groups(const float2* __restrict__ part, int G, long long N,
                             float2* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float2 v = part[i];
  for (int g = 1; g < G; ++g) v = cadd(v, part[(long long)g * N + i]);
  out[i] = v;
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

int col_stride(int K) { return K + 1; }

size_t rows_lds(int Kx) { return sizeof(float2) * 2 * kRowCoils * Kx; }
size_t cols_lds(const pnp_plan* p) { return sizeof(float2) * 2 * p->tile * col_stride(p->ax[1].K); }

void set_lds_limit(const void* fn, size_t bytes) {
  if (bytes > 65536)
    PNP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

size_t op_workspace_bytes(const pnp_plan* p, int L) {
  const int Kx = p->ax[0].K;
  const int64_t N = image_size(p);
  const int G = (L + kRowCoils - 1) / kRowCoils;
  size_t b = 0;
  b += al(sizeof(float2) * (size_t)L * p->ax[1].n * Kx);   // mid
  b += al(sizeof(float2) * (size_t)L * (size_t)std::max<int64_t>(p->E, 1));  // ypart
  b += al(sizeof(float2) * (size_t)L * p->M);             // ytmp
  b += al(sizeof(float2) * (size_t)G * N);                 // part
  return b;
}

OpWorkspace op_workspace(const pnp_plan* p, int L, void* ws) {
  OpWorkspace w;
  const int Kx = p->ax[0].K;
  const int64_t N = image_size(p);
  const int G = (L + kRowCoils - 1) / kRowCoils;
  char* c = (char*)ws;
  w.mid = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * p->ax[1].n * Kx);
  w.ypart = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * (size_t)std::max<int64_t>(p->E, 1));
  w.ytmp = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * p->M);
  w.part = (float2*)c;
  c += al(sizeof(float2) * (size_t)G * N);
  w.bytes = (size_t)(c - (char*)ws);
  return w;
}

static void check_lds(const pnp_plan* p) {
  const size_t need = std::max(rows_lds(p->ax[0].K), cols_lds(p));
  if (need > 160 * 1024)
    fail(PNP_ERR_UNSUPPORTED, "grid %dx%d needs %zu bytes of LDS per workgroup", p->ax[1].K,
         p->ax[0].K, need);
}

static void launch_forward_grid(const pnp_plan* p, const float2* x, const float2* smaps, int L,
                                const OpWorkspace& w, hipStream_t s) {
  const int nx = p->ax[0].n, ny = p->ax[1].n, Kx = p->ax[0].K;
  const int G = (L + kRowCoils - 1) / kRowCoils;
  check_lds(p);
  {
    const size_t lds = rows_lds(Kx);
    set_lds_limit((const void*)k_rows_fwd, lds);
    hipLaunchKernelGGL(k_rows_fwd, dim3(ny, G), dim3(kThreads), lds, s, x, smaps, L, nx, ny,
                       p->ax[0].deapod, p->ax[1].deapod, p->ax[0].fft, w.mid);
    PNP_CHECK_LAUNCH();
  }
  {
    const size_t lds = cols_lds(p);
    set_lds_limit((const void*)k_cols_fwd_interp, lds);
    hipLaunchKernelGGL(k_cols_fwd_interp, dim3(p->ntx, L), dim3(kThreads), lds, s, w.mid, nx, ny,
                       Kx, p->ax[1].fft, p->tile, col_stride(p->ax[1].K), p->tile_off,
                       p->ent_sample, p->j0, p->wts, (long long)p->E, w.ypart);
    PNP_CHECK_LAUNCH();
  }
}

void op_forward(const pnp_plan* p, const float2* x, const float2* smaps, int L, float2* y,
                const OpWorkspace& w, hipStream_t s) {
  launch_forward_grid(p, x, smaps, L, w, s);
  const long long tot = p->M * L;
  const float scale = (float)(1.0 / std::sqrt((double)image_size(p)));
  hipLaunchKernelGGL(k_gather_entries, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     w.ypart, p->sample_ent, (long long)p->M, (long long)p->E, L, scale, y);
  PNP_CHECK_LAUNCH();
}

void op_adjoint(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf,
                float2* x, const OpWorkspace& w, hipStream_t s) {
  const int nx = p->ax[0].n, ny = p->ax[1].n, Kx = p->ax[0].K;
  const int G = (L + kRowCoils - 1) / kRowCoils;
  const int64_t N = image_size(p);
  const float scale = (float)(1.0 / std::sqrt((double)N));
  check_lds(p);
  {
    const size_t lds = cols_lds(p);
    set_lds_limit((const void*)k_cols_adj_spread, lds);
    hipLaunchKernelGGL(k_cols_adj_spread, dim3(p->ntx, L), dim3(kThreads), lds, s, y, dcf, scale,
                       (long long)p->M, nx, ny, Kx, p->ax[1].fft, p->tile, col_stride(p->ax[1].K),
                       p->tile_off, p->ent_sample, p->j0, p->wts, w.mid);
    PNP_CHECK_LAUNCH();
  }
  {
    const size_t lds = rows_lds(Kx);
    set_lds_limit((const void*)k_rows_adj, lds);
    float2* dst = G == 1 ? x : w.part;
    hipLaunchKernelGGL(k_rows_adj, dim3(ny, G), dim3(kThreads), lds, s, w.mid, smaps, L, nx, ny,
                       p->ax[0].deapod, p->ax[1].deapod, p->ax[0].fft, 1.0f, dst);
    PNP_CHECK_LAUNCH();
  }
  if (G > 1) {
    hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w.part, G,
                       (long long)N, x);
    PNP_CHECK_LAUNCH();
  }
  (void)scale;
}

void op_normal(const pnp_plan* p, const float2* x, const float2* smaps, int L, const float* dcf,
               float2* out, const OpWorkspace& w, hipStream_t s) {
  op_forward(p, x, smaps, L, w.ytmp, w, s);
  op_adjoint(p, w.ytmp, smaps, L, dcf, out, w, s);
}

}  // namespace pnp
