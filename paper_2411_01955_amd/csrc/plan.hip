// Trajectory plan: grid coordinates, kernel weights, tile binning, FFT and
// deapodisation tables.
//
// Kaiser-Bessel gridding (the NUFFT is left open by the paper, Sec. 2.1):
//   grid coordinate  g = k * K / (2 pi)               (FP64)
//   taps             j = floor(g - W/2) + 1 + t, t = 0..W-1, wrapped mod K
//   weight           phi(g - j) = I0(beta sqrt(1 - (2(g-j)/W)^2)) / I0(beta)
//   deapodisation    I0(beta) / Phi(r/K),  Phi(nu) = W sinh(z)/z,
//                    z = sqrt(beta^2 - (pi W nu)^2),  r = i - n/2
//   beta             Beatty's rule pi sqrt((W/osf)^2 (osf - 1/2)^2 - 0.8)
// All tables are evaluated in FP64 on the device and rounded to FP32 once.
//
// Tiles: the last transformed axis (y in 2D, z in 3D) is kept whole in LDS;
// the other grid axes are cut into tiles of `tile` columns.  Every sample is
// listed once per tile its W x W footprint touches (at most 2 in 2D, 4 in
// 3D), grouped by tile with a counting sort, so that interpolation and
// spreading work tile by tile out of LDS.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include "common.hpp"
#include "fft_reg.hpp"

namespace pnp {

namespace {

__device__ double bessel_i0(double z) {
  // power series sum_k ((z/2)^2)^k / (k!)^2, converges for every z
  const double q = 0.25 * z * z;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 400; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

__global__ void k_twiddles(float2* tw, int K) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K) return;
  double s, c;
  sincospi(-2.0 * (double)t / (double)K, &s, &c);
  tw[t] = make_float2((float)c, (float)s);
}

// The roots the register passes take for their four-step split K = K1 K2,
// in two layouts after the K roots: [k1][t] = W^(t k1) (t < K2) and
// [r2][t] = W^(t r2) (t < K1), the same values as tw[t k1] and tw[t r2].
__global__ void k_twiddles_fs(float2* tw, int K, int K1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int K2 = K / K1;
  if (i >= 2 * K) return;
  const int j = i < K ? (i % K2) * (i / K2) : ((i - K) % K1) * ((i - K) / K1);
  double s, c;
  sincospi(-2.0 * (double)j / (double)K, &s, &c);
  tw[K + i] = make_float2((float)c, (float)s);
}

__global__ void k_deapod(float* dp, int n, int K, int W, double beta) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double nu = (double)(i - n / 2) / (double)K;
  const double a = M_PI * W * nu;
  const double z2 = beta * beta - a * a;
  double Phi;
  if (z2 > 0) {
    double z = sqrt(z2);
    Phi = W * sinh(z) / z;
  } else if (z2 < 0) {
    double z = sqrt(-z2);
    Phi = W * sin(z) / z;
  } else {
    Phi = W;
  }
  dp[i] = (float)(bessel_i0(beta) / Phi);
}

__device__ __forceinline__ int wrapi(long long j, int K) {
  long long r = j % K;
  return (int)(r < 0 ? r + K : r);
}

// Per sample: FP64 grid coordinates -> wrapped first tap, FP32 weights, and
// the tiles the footprint touches (counted with atomics).
__global__ void k_plan_samples(const float* __restrict__ traj, long long M, int ndim, int Kx, int Ky,
                               int Kz, int W, double beta, int tile, int ntx, int nty,
                               int4* __restrict__ j0, float* __restrict__ wts,
                               int* __restrict__ tile_count, int* __restrict__ sample_tiles,
                               int slots) {
  long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int Kd[3] = {Kx, Ky, Kz};
  int jj[3] = {0, 0, 0};
  const double inv_i0b = 1.0 / bessel_i0(beta);
  for (int a = 0; a < ndim; ++a) {
    const double g = (double)traj[m * ndim + a] * (double)Kd[a] / (2.0 * M_PI);
    const double f = floor(g - 0.5 * W) + 1.0;
    for (int t = 0; t < W; ++t) {
      const double u = g - (f + t);
      const double q = 2.0 * u / W;
      const double arg = fmax(1.0 - q * q, 0.0);
      wts[(m * ndim + a) * W + t] = (float)(bessel_i0(beta * sqrt(arg)) * inv_i0b);
    }
    jj[a] = wrapi((long long)f, Kd[a]);
  }
  j0[m] = make_int4(jj[0], jj[1], jj[2], 0);
  if (!tile_count) return;   // no strip tables (3D plans)
  // tiles along x (and y in 3D) touched by taps j0 .. j0 + W - 1 (mod K)
  int tx[2], ty[2];
  int nxs = 0, nys = 0;
  tx[nxs++] = jj[0] / tile;
  {
    int e = jj[0] + W - 1;
    if (e >= Kx) e -= Kx;
    int t1 = e / tile;
    if (t1 != tx[0]) tx[nxs++] = t1;
  }
  if (ndim == 3) {
    ty[nys++] = jj[1] / tile;
    int e = jj[1] + W - 1;
    if (e >= Ky) e -= Ky;
    int t1 = e / tile;
    if (t1 != ty[0]) ty[nys++] = t1;
  } else {
    ty[nys++] = 0;
  }
  int s = 0;
  for (int b = 0; b < nys; ++b)
    for (int a = 0; a < nxs; ++a) {
      const int tid = ty[b] * ntx + tx[a];
      sample_tiles[m * slots + s++] = tid;
      atomicAdd(&tile_count[tid], 1);
    }
  for (; s < slots; ++s) sample_tiles[m * slots + s] = -1;
}

__global__ void k_scan_tiles(const int* __restrict__ count, int ntiles, int* __restrict__ off,
                             int* __restrict__ cursor, int* __restrict__ maxc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int acc = 0, mx = 0;
  for (int t = 0; t < ntiles; ++t) {
    off[t] = acc;
    cursor[t] = 0;
    acc += count[t];
    mx = count[t] > mx ? count[t] : mx;
  }
  off[ntiles] = acc;
  *maxc = mx;
}

__global__ void k_scatter(long long M, int slots, const int* __restrict__ sample_tiles,
                          const int* __restrict__ off, int* __restrict__ cursor,
                          int* __restrict__ ent_sample, int* __restrict__ sample_ent) {
  long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  for (int s = 0; s < slots; ++s) {
    const int t = sample_tiles[m * slots + s];
    if (t < 0) {
      sample_ent[m * slots + s] = -1;
      continue;
    }
    const int pos = atomicAdd(&cursor[t], 1);
    const int e = off[t] + pos;
    ent_sample[e] = (int)m;
    sample_ent[m * slots + s] = e;
  }
}

__device__ __forceinline__ int tile_of_entry(const int* __restrict__ off, int ntiles, long long e) {
  int lo = 0, hi = ntiles;  // off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int row_of(const int4 j, int ra) { return ra == 1 ? j.y : j.z; }

// Within every tile, order the entries by the first tap along the axis kept
// whole in LDS (y in 2D, z in 3D) -- a counting sort into row buckets --
// and, inside a bucket, by sample index.  row_start[t][r] is the first
// entry of tile t whose first tap is row r (absolute entry index).
__global__ void k_row_hist(long long E, const int* __restrict__ off, int ntiles,
                           const int* __restrict__ ent, const int4* __restrict__ j0, int ra, int R,
                           int* __restrict__ rcnt) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int t = tile_of_entry(off, ntiles, e);
  atomicAdd(&rcnt[(long long)t * R + row_of(j0[ent[e]], ra)], 1);
}

__global__ void k_row_scan(const int* __restrict__ off, int ntiles, int R, const int* __restrict__ rcnt,
                           int* __restrict__ rstart, int* __restrict__ rcur) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int acc = off[t];
  for (int r = 0; r < R; ++r) {
    rstart[(long long)t * (R + 1) + r] = acc;
    rcur[(long long)t * R + r] = 0;
    acc += rcnt[(long long)t * R + r];
  }
  rstart[(long long)t * (R + 1) + R] = acc;
}

__global__ void k_row_scatter(long long E, const int* __restrict__ off, int ntiles,
                              const int* __restrict__ ent_in, const int4* __restrict__ j0, int ra, int R,
                              const int* __restrict__ rstart, int* __restrict__ rcur,
                              int* __restrict__ ent_out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int t = tile_of_entry(off, ntiles, e);
  const int m = ent_in[e];
  const int r = row_of(j0[m], ra);
  const int pos = rstart[(long long)t * (R + 1) + r] + atomicAdd(&rcur[(long long)t * R + r], 1);
  ent_out[pos] = m;
}

// insertion sort of each (tile, row) bucket by sample index (buckets are short)
__global__ void k_bucket_sort(int ntiles, int R, const int* __restrict__ rstart, int* __restrict__ ent) {
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (long long)ntiles * R) return;
  const long long t = b / R, r = b % R;
  const int s = rstart[t * (R + 1) + r], e = rstart[t * (R + 1) + r + 1];
  for (int i = s + 1; i < e; ++i) {
    const int v = ent[i];
    int j = i - 1;
    while (j >= s && ent[j] > v) {
      ent[j + 1] = ent[j];
      --j;
    }
    ent[j + 1] = v;
  }
}

__global__ void k_refresh_sample_ent(long long E, int slots, const int* __restrict__ ent_sample,
                                     const int* __restrict__ off, const int* __restrict__ sample_tiles,
                                     int ntiles, int* __restrict__ sample_ent) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int lo = tile_of_entry(off, ntiles, e);
  const int m = ent_sample[e];
  for (int s = 0; s < slots; ++s)
    if (sample_tiles[(long long)m * slots + s] == lo) sample_ent[(long long)m * slots + s] = (int)e;
}

// Packed per-entry records (2D): taps, sample and the 12 weights in tile order.
__global__ void k_build_records(long long E, const int* __restrict__ ent_sample,
                                const int4* __restrict__ j0, const float* __restrict__ wts,
                                EntryRec* __restrict__ rec) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int m = ent_sample[e];
  const int4 jj = j0[m];
  const float* w = wts + (long long)m * 12;
  EntryRec r;
  r.idx = make_int4(jj.x, jj.y, m, 0);
  r.w0 = make_float4(w[0], w[1], w[2], w[3]);
  r.w1 = make_float4(w[4], w[5], w[6], w[7]);
  r.w2 = make_float4(w[8], w[9], w[10], w[11]);
  rec[e] = r;
}

__global__ void k_check_finite(const float* __restrict__ v, long long n, int* __restrict__ bad) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(v[i])) atomicOr(bad, 1);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

bool fft_factor(int K, FFTDesc* d) {
  d->K = K;
  d->nrad = 0;
  int r = K;
  const int order[5] = {8, 4, 2, 5, 3};
  for (int oi = 0; oi < 5; ++oi) {
    const int R = order[oi];
    while (r % R == 0) {
      if (d->nrad >= kMaxRadices) return false;
      d->rad[d->nrad++] = R;
      r /= R;
    }
  }
  return r == 1;
}

int64_t image_size(const pnp_plan* p) {
  int64_t N = 1;
  for (int a = 0; a < p->ndim; ++a) N *= p->ax[a].n;
  return N;
}

static int choose_tile(int K) {
  const int pref[] = {8, 12, 10, 6, 16, 15, 9, 18, 20, 24, 25, 27, 30, 32};
  for (int t : pref)
    if (K % t == 0) return t;
  return 0;
}

__global__ void k_deapod_yz(const float* __restrict__ dy, const float* __restrict__ dz, int ny, int nz,
                            float* __restrict__ dyz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ny * nz) dyz[i] = dy[i % ny] * dz[i / ny];
}

// 3D plan: twiddles and deapodisation per axis, the combined y-z
// deapodisation of the (z, y) image rows, and per sample the wrapped first
// taps and kernel weights (the 3D operator spreads and interpolates from
// the full oversampled grid; no strip tables).
// 3D sort by first-tap cell: keys, cell bounds, tables in sorted order
__global__ void k3_cell_keys(long long M, const int4* __restrict__ j0, int Kx, int Ky, uint32_t* __restrict__ keys,
                             int32_t* __restrict__ vals) {
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int4 j = j0[m];
  keys[m] = ((uint32_t)j.z * (uint32_t)Ky + (uint32_t)j.y) * (uint32_t)Kx + (uint32_t)j.x;
  vals[m] = (int32_t)m;
}

// off[c] = first sorted index whose key is >= c, for c = 0..ncells
__global__ void k3_cell_bounds(long long ncells, const uint32_t* __restrict__ keys, long long M,
                               int32_t* __restrict__ off) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncells) return;
  long long lo = 0, hi = M;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if ((long long)keys[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  off[c] = (int32_t)lo;
}

__global__ void k3_sorted_tables(long long M, int W, const int32_t* __restrict__ sm, const int4* __restrict__ j0,
                                 const float* __restrict__ wts, int32_t* __restrict__ jx, float* __restrict__ sw) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int32_t m = sm[i];
  jx[i] = j0[m].x;
  for (int k = 0; k < 3 * W; ++k) sw[i * 3 * W + k] = wts[(long long)m * 3 * W + k];
}

static void sort_by_cell(pnp_plan* p, hipStream_t stream) {
  const long long M = p->M;
  const int Kx = p->ax[0].K, Ky = p->ax[1].K, Kz = p->ax[2].K;
  const long long ncells = (long long)Kx * Ky * Kz;
  if (M >= (1ll << 31) || ncells >= (1ll << 31)) fail(PNP_ERR_SHAPE, "3D plan too large for the sample sort");
  int bits = 1;
  while ((1ll << bits) < ncells) ++bits;
  void* blk = nullptr;
  auto release = [&] {
    if (blk) (void)hipFree(blk);
  };
  try {
    size_t tb = 0;
    PNP_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                               (const int32_t*)nullptr, (int32_t*)nullptr, (int)M, 0, bits, stream));
    const size_t kb = align256(sizeof(uint32_t) * M);
    PNP_HIP(hipMalloc(&blk, 3 * kb + align256(tb)));
    char* c = (char*)blk;
    uint32_t* keys = (uint32_t*)c;
    uint32_t* keys_s = (uint32_t*)(c + kb);
    int32_t* vals = (int32_t*)(c + 2 * kb);
    void* tmp = c + 3 * kb;
    const unsigned nb = (unsigned)((M + 255) / 256);
    k3_cell_keys<<<nb, 256, 0, stream>>>(M, p->j0, Kx, Ky, keys, vals);
    PNP_CHECK_LAUNCH();
    PNP_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys_s, vals, p->sorted_m, (int)M, 0, bits, stream));
    k3_cell_bounds<<<(unsigned)((ncells + 1 + 255) / 256), 256, 0, stream>>>(ncells, keys_s, M, p->cell_off);
    PNP_CHECK_LAUNCH();
    k3_sorted_tables<<<nb, 256, 0, stream>>>(M, p->W, p->sorted_m, p->j0, p->wts, p->sorted_jx, p->sorted_w);
    PNP_CHECK_LAUNCH();
    PNP_HIP(hipStreamSynchronize(stream));
  } catch (...) {
    release();
    throw;
  }
  release();
}

// Candidates of every 8^3 grid tile for the tiled 3D spread: the samples
// whose first-tap cell lies in [t0 - 5, t0 + 7] on each axis (mod K), read
// off the cell offsets as 13 x 13 row ranges.
__global__ void k3_tile_cands(const int32_t* __restrict__ cell_off, int Kx, int Ky, int Kz,
                              int32_t* __restrict__ cnt) {
  const int ntx = Kx / 8, nty = Ky / 8, ntz = Kz / 8;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntx * nty * ntz) return;
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int x0 = tx * 8 - 5;
  long long c = 0;
  for (int rz = 0; rz < 13; ++rz) {
    const int cz = (tz * 8 - 5 + rz + Kz) % Kz;
    for (int ry = 0; ry < 13; ++ry) {
      const int cy = (ty * 8 - 5 + ry + Ky) % Ky;
      const long long row = ((long long)cz * Ky + cy) * Kx;
      if (x0 >= 0) {
        c += cell_off[row + x0 + 13] - cell_off[row + x0];
      } else {
        c += cell_off[row + Kx] - cell_off[row + Kx + x0];
        c += cell_off[row + x0 + 13] - cell_off[row];
      }
    }
  }
  cnt[t] = (int32_t)c;
}

// Home samples of every 8^3 grid tile for the tiled 3D interpolation: the
// samples whose first-tap cell lies in the tile, 8 x 8 row ranges.
__global__ void k3_tile_home(const int32_t* __restrict__ cell_off, int Kx, int Ky, int Kz,
                             int32_t* __restrict__ cnt) {
  const int ntx = Kx / 8, nty = Ky / 8, ntz = Kz / 8;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntx * nty * ntz) return;
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  int c = 0;
  for (int rz = 0; rz < 8; ++rz)
    for (int ry = 0; ry < 8; ++ry) {
      const long long row = ((long long)(tz * 8 + rz) * Ky + ty * 8 + ry) * Kx + tx * 8;
      c += cell_off[row + 8] - cell_off[row];
    }
  cnt[t] = c;
}

// Work list of the tiled 3D spread: one item per tile, tiles with more than
// kSpreadChunk3 candidates split into several items with partial slots.
// Work list of the tiled 3D interpolation: tiles with home samples in tile
// order (neighbouring tiles, whose staged regions overlap, run together),
// split into items of at most kInterpChunk3 samples.
static constexpr int kSpreadChunk3 = 2048;
static constexpr int kInterpChunk3 = 512;

static void build_spread3(pnp_plan* p, hipStream_t stream) {
  const int Kx = p->ax[0].K, Ky = p->ax[1].K, Kz = p->ax[2].K;
  if (Kx % 8 || Ky % 8 || Kz % 8 || Kx < 16 || Ky < 16 || Kz < 16)
    fail(PNP_ERR_SHAPE, "3D spread tiles need grid sides divisible by 8");
  const int nt = (Kx / 8) * (Ky / 8) * (Kz / 8);
  int32_t* dcnt = nullptr;
  struct Free {
    int32_t*& q;
    ~Free() { if (q) (void)hipFree(q); }
  } fr{dcnt};
  PNP_HIP(hipMalloc((void**)&dcnt, 2 * sizeof(int32_t) * nt));
  k3_tile_cands<<<(nt + 255) / 256, 256, 0, stream>>>(p->cell_off, Kx, Ky, Kz, dcnt);
  PNP_CHECK_LAUNCH();
  k3_tile_home<<<(nt + 255) / 256, 256, 0, stream>>>(p->cell_off, Kx, Ky, Kz, dcnt + nt);
  PNP_CHECK_LAUNCH();
  std::vector<int32_t> cnt(nt), home(nt);
  PNP_HIP(hipMemcpyAsync(cnt.data(), dcnt, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, stream));
  PNP_HIP(hipMemcpyAsync(home.data(), dcnt + nt, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, stream));
  PNP_HIP(hipStreamSynchronize(stream));
  std::vector<int4> ipi;
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < home[t]; k += kInterpChunk3) ipi.push_back(make_int4(t, k, std::min(home[t], k + kInterpChunk3), 0));
  std::vector<int> order(nt);
  for (int t = 0; t < nt; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
  std::vector<int4> items, folds;
  items.reserve(nt + 64);
  int slots = 0;
  for (int t : order) {
    const int c = cnt[t];
    if (c <= kSpreadChunk3) {
      items.push_back(make_int4(t, 0, c, -1));
      continue;
    }
    const int nch = (c + kSpreadChunk3 - 1) / kSpreadChunk3;
    folds.push_back(make_int4(t, slots, nch, 0));
    for (int k = 0; k < nch; ++k)
      items.push_back(make_int4(t, k * kSpreadChunk3, std::min(c, (k + 1) * kSpreadChunk3), slots + k));
    slots += nch;
  }
  // the heavy chunks first (all chunks of a split tile hold kSpreadChunk3
  // candidates but the last)
  std::stable_sort(items.begin(), items.end(), [](const int4& a, const int4& b) { return a.z - a.y > b.z - b.y; });
  const size_t bi = align256(sizeof(int4) * items.size()), bf = align256(sizeof(int4) * std::max<size_t>(1, folds.size()));
  const size_t bp = align256(sizeof(int4) * std::max<size_t>(1, ipi.size()));
  PNP_HIP(hipMalloc(&p->block3, bi + bf + bp));
  p->sp_items = (int4*)p->block3;
  p->sp_folds = (int4*)((char*)p->block3 + bi);
  p->ip_items = (int4*)((char*)p->block3 + bi + bf);
  p->n_ip_items = (int)ipi.size();
  if (!ipi.empty())
    PNP_HIP(hipMemcpyAsync(p->ip_items, ipi.data(), sizeof(int4) * ipi.size(), hipMemcpyHostToDevice, stream));
  p->n_sp_items = (int)items.size();
  p->n_sp_folds = (int)folds.size();
  p->sp_slots = slots;
  PNP_HIP(hipMemcpyAsync(p->sp_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, stream));
  if (!folds.empty())
    PNP_HIP(hipMemcpyAsync(p->sp_folds, folds.data(), sizeof(int4) * folds.size(), hipMemcpyHostToDevice, stream));
  PNP_HIP(hipStreamSynchronize(stream));
}

static void plan_create_3d(pnp_plan* p, const float* traj, hipStream_t stream) {
  const int64_t M = p->M;
  p->tile = 8;                  // strip width of the column passes
  p->row_coils = 4;
  p->row_coils_fwd = 4;
  p->ntx = p->ax[0].K / 8;
  p->nty = 1;
  p->ntiles = 0;
  p->slots = 0;
  p->E = 0;
  p->max_tile_entries = 0;
  PNP_HIP(hipGetDevice(&p->device));
  {
    int* bad = nullptr;
    PNP_HIP(hipMalloc((void**)&bad, sizeof(int)));
    PNP_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
    const long long nv = M * 3;
    k_check_finite<<<(unsigned)((nv + 255) / 256), 256, 0, stream>>>(traj, nv, bad);
    PNP_CHECK_LAUNCH();
    int hbad = 0;
    PNP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    PNP_HIP(hipStreamSynchronize(stream));
    PNP_HIP(hipFree(bad));
    if (hbad) fail(PNP_ERR_NUMERIC, "trajectory holds non-finite coordinates");
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  size_t o_tw[3], o_dp[3];
  for (int a = 0; a < 3; ++a) {
    o_tw[a] = take(sizeof(float2) * 3 * p->ax[a].K);
    o_dp[a] = take(sizeof(float) * p->ax[a].n);
  }
  const size_t o_yz = take(sizeof(float) * p->ax[1].n * p->ax[2].n);
  const size_t o_j0 = take(sizeof(int4) * M);
  const size_t o_w = take(sizeof(float) * M * 3 * p->W);
  const size_t o_traj = take(sizeof(float) * M * 3);
  const long long ncells = (long long)p->ax[0].K * p->ax[1].K * p->ax[2].K;
  const size_t o_sm = take(sizeof(int32_t) * M);
  const size_t o_jx = take(sizeof(int32_t) * M);
  const size_t o_sw = take(sizeof(float) * M * 3 * p->W);
  const size_t o_co = take(sizeof(int32_t) * (ncells + 1));
  PNP_HIP(hipMalloc(&p->block, off));
  p->block_bytes = off;
  char* base = (char*)p->block;
  for (int a = 0; a < 3; ++a) {
    p->ax[a].fft.tw = (const float2*)(base + o_tw[a]);
    p->ax[a].deapod = (float*)(base + o_dp[a]);
  }
  p->deapod_yz = (float*)(base + o_yz);
  p->j0 = (int4*)(base + o_j0);
  p->wts = (float*)(base + o_w);
  p->traj = (float*)(base + o_traj);
  p->sorted_m = (int32_t*)(base + o_sm);
  p->sorted_jx = (int32_t*)(base + o_jx);
  p->sorted_w = (float*)(base + o_sw);
  p->cell_off = (int32_t*)(base + o_co);
  p->tile_off = nullptr;
  p->row_start = nullptr;
  p->tile_order = nullptr;
  p->ent_sample = nullptr;
  p->sample_ent = nullptr;
  p->rec = nullptr;
  PNP_HIP(hipMemcpyAsync(p->traj, traj, sizeof(float) * M * 3, hipMemcpyDeviceToDevice, stream));
  for (int a = 0; a < 3; ++a) {
    const int K = p->ax[a].K, n = p->ax[a].n;
    k_twiddles<<<(K + 255) / 256, 256, 0, stream>>>((float2*)p->ax[a].fft.tw, K);
    PNP_CHECK_LAUNCH();
    if (const int k1 = four_step_k1(K)) {
      k_twiddles_fs<<<(2 * K + 255) / 256, 256, 0, stream>>>((float2*)p->ax[a].fft.tw, K, k1);
      PNP_CHECK_LAUNCH();
    }
    k_deapod<<<(n + 255) / 256, 256, 0, stream>>>(p->ax[a].deapod, n, K, p->W, p->beta);
    PNP_CHECK_LAUNCH();
  }
  const int nyz = p->ax[1].n * p->ax[2].n;
  k_deapod_yz<<<(nyz + 255) / 256, 256, 0, stream>>>(p->ax[1].deapod, p->ax[2].deapod, p->ax[1].n, p->ax[2].n,
                                                     p->deapod_yz);
  PNP_CHECK_LAUNCH();
  k_plan_samples<<<(unsigned)((M + 255) / 256), 256, 0, stream>>>(traj, M, 3, p->ax[0].K, p->ax[1].K, p->ax[2].K,
                                                                   p->W, p->beta, 8, 1, 1, p->j0, p->wts, nullptr,
                                                                   nullptr, 0);
  PNP_CHECK_LAUNCH();
  sort_by_cell(p, stream);
  build_spread3(p, stream);
}

pnp_plan* plan_create(int ndim, const int32_t* shape, int64_t M, const float* traj,
                      hipStream_t stream) {
  if (ndim != 2 && ndim != 3) fail(PNP_ERR_SHAPE, "ndim must be 2 or 3 (got %d)", ndim);
  if (M < 1) fail(PNP_ERR_SHAPE, "M must be >= 1 (got %lld)", (long long)M);
  if (M > (int64_t)1 << 30) fail(PNP_ERR_SHAPE, "M too large (%lld)", (long long)M);
  pnp_plan* p = new pnp_plan();
  p->ndim = ndim;
  p->M = M;
  p->W = 6;
  const double osf = 2.0;
  p->beta = M_PI * std::sqrt((p->W / osf) * (p->W / osf) * (osf - 0.5) * (osf - 0.5) - 0.8);
  p->block = nullptr;
  try {
    for (int a = 0; a < 3; ++a) {
      p->ax[a].n = 1;
      p->ax[a].K = 1;
      p->ax[a].deapod = nullptr;
      p->ax[a].fft.tw = nullptr;
      p->ax[a].fft.nrad = 0;
    }
    for (int a = 0; a < ndim; ++a) {
      const int n = shape[ndim - 1 - a];
      if (n < 4 || n > 1024 || (n & 1))
        fail(PNP_ERR_SHAPE, "image size %d unsupported (even, 4..1024)", n);
      p->ax[a].n = n;
      p->ax[a].K = 2 * n;
      if (!fft_factor(2 * n, &p->ax[a].fft))
        fail(PNP_ERR_SHAPE, "grid size %d must have only prime factors 2, 3, 5", 2 * n);
    }
    if (ndim == 3) {
      plan_create_3d(p, traj, stream);
      return p;
    }
    p->tile = choose_tile(p->ax[0].K);
    p->row_coils = 4;
    p->row_coils_fwd = 4;
    if (ndim == 3 && choose_tile(p->ax[1].K) != p->tile)
      fail(PNP_ERR_SHAPE, "3D x and y grids need a common tile size");
    if (p->tile == 0) fail(PNP_ERR_SHAPE, "no tile size divides grid size %d", p->ax[0].K);
    p->ntx = p->ax[0].K / p->tile;
    p->nty = ndim == 3 ? p->ax[1].K / p->tile : 1;
    p->ntiles = p->ntx * p->nty;
    p->slots = ndim == 3 ? 4 : 2;
    nufft2d_check_plan(p);

    PNP_HIP(hipGetDevice(&p->device));

    // validate the trajectory on the device
    {
      int* bad = nullptr;
      PNP_HIP(hipMalloc((void**)&bad, sizeof(int)));
      PNP_HIP(hipMemsetAsync(bad, 0, sizeof(int), stream));
      const long long nv = M * ndim;
      k_check_finite<<<(unsigned)((nv + 255) / 256), 256, 0, stream>>>(traj, nv, bad);
      PNP_CHECK_LAUNCH();
      int hbad = 0;
      PNP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
      PNP_HIP(hipStreamSynchronize(stream));
      PNP_HIP(hipFree(bad));
      if (hbad) fail(PNP_ERR_NUMERIC, "trajectory holds non-finite coordinates");
    }

    // one allocation: tables + per-sample data + entries (E <= slots*M)
    const int64_t Emax = (int64_t)p->slots * M;
    const int ra = ndim - 1;                 // axis kept whole in LDS (y in 2D, z in 3D)
    const int R = p->ax[ra].K;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off += align256(bytes);
      return o;
    };
    size_t o_tw[3], o_dp[3];
    for (int a = 0; a < ndim; ++a) {
      o_tw[a] = take(sizeof(float2) * 3 * p->ax[a].K);
      o_dp[a] = take(sizeof(float) * p->ax[a].n);
    }
    const size_t o_j0 = take(sizeof(int4) * M);
    const size_t o_w = take(sizeof(float) * M * ndim * p->W);
    const size_t o_off = take(sizeof(int) * (p->ntiles + 1));
    const size_t o_rs = take(sizeof(int) * (size_t)p->ntiles * (R + 1));
    const size_t o_es = take(sizeof(int) * Emax);
    const size_t o_se = take(sizeof(int) * M * p->slots);
    const size_t o_rec = take(sizeof(EntryRec) * (ndim == 2 ? Emax : 1));
    const size_t o_traj = take(sizeof(float) * M * ndim);
    const size_t o_ord = take(sizeof(int) * p->ntiles);
    const size_t o_ai = take(sizeof(int4) * ((size_t)p->ntiles + kMaxAdjSlots));
    const size_t o_as = take(sizeof(int4) * kMaxAdjSlots);
    // set-up scratch (freed below)
    size_t soff = 0;
    const size_t s_cnt = soff; soff += align256(sizeof(int) * p->ntiles);
    const size_t s_cur = soff; soff += align256(sizeof(int) * p->ntiles);
    const size_t s_max = soff; soff += align256(sizeof(int));
    const size_t s_st = soff; soff += align256(sizeof(int) * M * p->slots);
    const size_t s_rc = soff; soff += align256(sizeof(int) * (size_t)p->ntiles * R);
    const size_t s_ru = soff; soff += align256(sizeof(int) * (size_t)p->ntiles * R);
    const size_t s_tmp = soff; soff += align256(sizeof(int) * Emax);

    PNP_HIP(hipMalloc(&p->block, off));
    p->block_bytes = off;
    char* base = (char*)p->block;
    for (int a = 0; a < ndim; ++a) {
      p->ax[a].fft.tw = (const float2*)(base + o_tw[a]);
      p->ax[a].deapod = (float*)(base + o_dp[a]);
    }
    p->j0 = (int4*)(base + o_j0);
    p->wts = (float*)(base + o_w);
    p->tile_off = (int32_t*)(base + o_off);
    p->row_start = (int32_t*)(base + o_rs);
    p->ent_sample = (int32_t*)(base + o_es);
    p->sample_ent = (int32_t*)(base + o_se);
    p->rec = (EntryRec*)(base + o_rec);
    p->traj = (float*)(base + o_traj);
    p->tile_order = (int32_t*)(base + o_ord);
    p->adj_items = (int4*)(base + o_ai);
    p->adj_splits = (int4*)(base + o_as);
    PNP_HIP(hipMemcpyAsync(p->traj, traj, sizeof(float) * M * ndim, hipMemcpyDeviceToDevice, stream));

    struct Scratch {
      char* ptr = nullptr;
      ~Scratch() { if (ptr) (void)hipFree(ptr); }
    } scratch;
    PNP_HIP(hipMalloc((void**)&scratch.ptr, soff));
    int* cnt = (int*)(scratch.ptr + s_cnt);
    int* cur = (int*)(scratch.ptr + s_cur);
    int* mx = (int*)(scratch.ptr + s_max);
    int* st = (int*)(scratch.ptr + s_st);
    int* rcnt = (int*)(scratch.ptr + s_rc);
    int* rcur = (int*)(scratch.ptr + s_ru);
    int* etmp = (int*)(scratch.ptr + s_tmp);

    for (int a = 0; a < ndim; ++a) {
      const int K = p->ax[a].K, n = p->ax[a].n;
      k_twiddles<<<(K + 255) / 256, 256, 0, stream>>>((float2*)p->ax[a].fft.tw, K);
      PNP_CHECK_LAUNCH();
      if (const int k1 = four_step_k1(K)) {
        k_twiddles_fs<<<(2 * K + 255) / 256, 256, 0, stream>>>((float2*)p->ax[a].fft.tw, K, k1);
        PNP_CHECK_LAUNCH();
      }
      k_deapod<<<(n + 255) / 256, 256, 0, stream>>>(p->ax[a].deapod, n, K, p->W, p->beta);
      PNP_CHECK_LAUNCH();
    }
    PNP_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * p->ntiles, stream));
    PNP_HIP(hipMemsetAsync(rcnt, 0, sizeof(int) * (size_t)p->ntiles * R, stream));
    const unsigned gM = (unsigned)((M + 255) / 256);
    k_plan_samples<<<gM, 256, 0, stream>>>(traj, M, ndim, p->ax[0].K, p->ax[1].K, p->ax[2].K, p->W,
                                           p->beta, p->tile, p->ntx, p->nty, p->j0, p->wts, cnt, st,
                                           p->slots);
    PNP_CHECK_LAUNCH();
    k_scan_tiles<<<1, 64, 0, stream>>>(cnt, p->ntiles, p->tile_off, cur, mx);
    PNP_CHECK_LAUNCH();
    // entries grouped by tile (arbitrary order) into etmp
    k_scatter<<<gM, 256, 0, stream>>>(M, p->slots, st, p->tile_off, cur, etmp, p->sample_ent);
    PNP_CHECK_LAUNCH();
    int hE = 0, hmax = 0;
    PNP_HIP(hipMemcpyAsync(&hE, p->tile_off + p->ntiles, sizeof(int), hipMemcpyDeviceToHost, stream));
    PNP_HIP(hipMemcpyAsync(&hmax, mx, sizeof(int), hipMemcpyDeviceToHost, stream));
    PNP_HIP(hipStreamSynchronize(stream));
    p->E = hE;
    p->max_tile_entries = hmax;
    const unsigned gE = (unsigned)std::max<int64_t>(1, (p->E + 255) / 256);
    // order each tile by (first row tap, sample): row buckets + bucket sort
    k_row_hist<<<gE, 256, 0, stream>>>(p->E, p->tile_off, p->ntiles, etmp, p->j0, ra, R, rcnt);
    PNP_CHECK_LAUNCH();
    k_row_scan<<<(p->ntiles + 63) / 64, 64, 0, stream>>>(p->tile_off, p->ntiles, R, rcnt, p->row_start,
                                                          rcur);
    PNP_CHECK_LAUNCH();
    k_row_scatter<<<gE, 256, 0, stream>>>(p->E, p->tile_off, p->ntiles, etmp, p->j0, ra, R, p->row_start,
                                          rcur, p->ent_sample);
    PNP_CHECK_LAUNCH();
    {
      const long long nb = (long long)p->ntiles * R;
      k_bucket_sort<<<(unsigned)((nb + 255) / 256), 256, 0, stream>>>(p->ntiles, R, p->row_start,
                                                                     p->ent_sample);
      PNP_CHECK_LAUNCH();
    }
    if (p->E > 0) {
      k_refresh_sample_ent<<<gE, 256, 0, stream>>>(p->E, p->slots, p->ent_sample, p->tile_off, st,
                                                   p->ntiles, p->sample_ent);
      PNP_CHECK_LAUNCH();
      if (ndim == 2) {
        k_build_records<<<gE, 256, 0, stream>>>(p->E, p->ent_sample, p->j0, p->wts, p->rec);
        PNP_CHECK_LAUNCH();
      }
    }
    // dispatch order of the 2D spread: the tiles with the most entries (the
    // k-space centre) first, so their long workgroups start at once
    {
      std::vector<int32_t> off(p->ntiles + 1), ord(p->ntiles);
      PNP_HIP(hipMemcpyAsync(off.data(), p->tile_off, sizeof(int32_t) * (p->ntiles + 1), hipMemcpyDeviceToHost,
                             stream));
      PNP_HIP(hipStreamSynchronize(stream));
      for (int t = 0; t < p->ntiles; ++t) ord[t] = t;
      std::stable_sort(ord.begin(), ord.end(),
                       [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
      PNP_HIP(hipMemcpyAsync(p->tile_order, ord.data(), sizeof(int32_t) * p->ntiles, hipMemcpyHostToDevice,
                             stream));
    }
    // work items of the 2D adjoint spread: the entries in the window of every
    // (strip, 8-row block), first row taps [8 rb - 5, 8 rb + 8) wrapped
    if (ndim == 2) {
      std::vector<int32_t> rs((size_t)p->ntiles * (R + 1));
      PNP_HIP(hipMemcpyAsync(rs.data(), p->row_start, sizeof(int32_t) * rs.size(), hipMemcpyDeviceToHost, stream));
      PNP_HIP(hipStreamSynchronize(stream));
      const int nrb = R / 8;
      p->adj_cost.assign((size_t)p->ntiles * nrb, 0);
      for (int t = 0; t < p->ntiles; ++t) {
        const int32_t* r = rs.data() + (size_t)t * (R + 1);
        for (int rb = 0; rb < nrb; ++rb) {
          const int lo = rb * 8 - 5, hi = rb * 8 + 8;
          p->adj_cost[(size_t)t * nrb + rb] = lo >= 0 ? r[hi] - r[lo] : (r[R] - r[R + lo]) + (r[hi] - r[0]);
        }
      }
      adj_build_items(p, 1, 128, stream);
    }
    PNP_HIP(hipStreamSynchronize(stream));
  } catch (...) {
    if (p->block) (void)hipFree(p->block);
    if (p->block3) (void)hipFree(p->block3);
    delete p;
    throw;
  }
  return p;
}

void plan_destroy(pnp_plan* p) {
  if (!p) return;
  if (p->block) (void)hipFree(p->block);
  if (p->block3) (void)hipFree(p->block3);
  delete p;
}

}  // namespace pnp
