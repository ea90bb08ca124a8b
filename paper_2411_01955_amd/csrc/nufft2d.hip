// Multicoil 2D non-Cartesian operator by Kaiser-Bessel gridding, with every
// step fused so that the oversampled grid never travels through HBM:
//
//   forward  A x   (Eq. 1, y_l = F_Omega S_l x)
//     rows_fwd        pre (x * S_l * deapod) + zero pad + row FFT (along x)
//                     -> mid[l][iy][Kx]       (only the ny image rows exist)
//     cols_fwd        strip of `tile` grid columns: column FFT (along y) in
//                     LDS, then type-2 interpolation of the entries (samples
//                     whose footprint touches the strip) -> per-entry partials
//     k_gather_entries  y_l[m] = N^{-1/2} * sum of the sample's partials
//   adjoint  A^H D_w y
//     cols_adj        strip: type-1 spread of w_m y_l[m] as a gather (each
//                     wave accumulates the row-sorted entries of its 16-row
//                     grid blocks as FP32 MFMA products of row weights and
//                     column-weighted values, no atomics) into the strip in
//                     LDS, column inverse FFT, keep the ny image rows
//                     -> mid[l][iy][Kx]
//     rows_adj        row inverse FFT, crop, deapod, conj(S_l), sum over the
//                     coils of the workgroup -> per-coil-group partial images
//     k_sum_groups    out = sum over coil groups
//
// Two implementations of the transforms: grid sizes with a register
// factorisation K = K1*K2 (fft_reg.hpp) use the four-step kernels (*_fs),
// all others the LDS Stockham kernels.  Pixel r = i - n/2 sits at grid index
// r mod K; grid index j is frequency j (mod K).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "fft_lds.hpp"
#include "fft_reg.hpp"
#include "fs_bodies.hpp"
#include "trace.hpp"

namespace pnp {

namespace {

constexpr int kThreads = 256;
constexpr int kRowCoils = 4;      // coils per workgroup in the generic row passes and the batch

// k-space input of the adjoint column pass: y[l][m], or -- inside the
// normal operator -- the sum of the sample's interpolation partials.
struct KIn {
  const float2* y;          // [L][M]; nullptr: use the partials
  const float2* ypart;      // [L][E]
  const int* sample_ent;    // [M][2]
  long long M, E;
};

__device__ __forceinline__ float2 k_at(const KIn& in, int l, int m) {
  if (in.y) return in.y[(long long)l * in.M + m];
  const int e0 = in.sample_ent[2 * (long long)m], e1 = in.sample_ent[2 * (long long)m + 1];
  float2 v = make_float2(0.f, 0.f);
  if (e0 >= 0) v = in.ypart[(long long)l * in.E + e0];
  if (e1 >= 0) v = cadd(v, in.ypart[(long long)l * in.E + e1]);
  return v;
}

struct Taps {
  int jx, jy, m;
  float wx[6], wy[6];
};

__device__ __forceinline__ Taps load_taps(const EntryRec* __restrict__ rec, int e) {
  const EntryRec r = rec[e];
  Taps t;
  t.jx = r.idx.x;
  t.jy = r.idx.y;
  t.m = r.idx.z;
  t.wx[0] = r.w0.x; t.wx[1] = r.w0.y; t.wx[2] = r.w0.z; t.wx[3] = r.w0.w;
  t.wx[4] = r.w1.x; t.wx[5] = r.w1.y;
  t.wy[0] = r.w1.z; t.wy[1] = r.w1.w;
  t.wy[2] = r.w2.x; t.wy[3] = r.w2.y; t.wy[4] = r.w2.z; t.wy[5] = r.w2.w;
  return t;
}

// type-2 interpolation of one entry from a strip held in LDS as columns
// g[c*GS + row], c < tile (grid columns c0 + c).  The entry's first tap
// column relative to the strip, d in [-5, 7], gives every tap's column by
// one add; rows that do not wrap (jy <= Ky - 6, all but the last rows) are
// read at constant offsets from the column's first tap row.
__device__ __forceinline__ float2 interp_entry(const Taps& t, const float2* __restrict__ g, int GS,
                                               int c0, int tile, int Kx, int Ky) {
  int d = t.jx - c0;
  if (d > 7) d -= Kx;
  if (d < -5) d += Kx;
  const bool nowrap = t.jy <= Ky - 6;
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int ta = 0; ta < 6; ++ta) {
    const int c = d + ta;
    if ((unsigned)c < (unsigned)tile) {
      float2 sum = make_float2(0.f, 0.f);
      const float2* gc = g + c * GS;
      if (nowrap) {
#pragma unroll
        for (int tb = 0; tb < 6; ++tb) sum = cfma(t.wy[tb], gc[t.jy + tb], sum);
      } else {
#pragma unroll
        for (int tb = 0; tb < 6; ++tb) {
          int row = t.jy + tb;
          if (row >= Ky) row -= Ky;
          sum = cfma(t.wy[tb], gc[row], sum);
        }
      }
      acc = cfma(t.wx[ta], sum, acc);
    }
  }
  return acc;
}

// type-1 spread of one entry into the LDS strip (LDS float atomics)
__device__ __forceinline__ void spread_entry(const Taps& t, float2 v, float2* g, int GS, int c0,
                                             int tile, int Kx, int Ky) {
#pragma unroll
  for (int ta = 0; ta < 6; ++ta) {
    int col = t.jx + ta;
    if (col >= Kx) col -= Kx;
    const int c = col - c0;
    if ((unsigned)c < (unsigned)tile) {
      const float2 vx = cscale(v, t.wx[ta]);
#pragma unroll
      for (int tb = 0; tb < 6; ++tb) {
        int row = t.jy + tb;
        if (row >= Ky) row -= Ky;
        float* dst = reinterpret_cast<float*>(&g[c * GS + row]);
        atomicAdd(dst, vx.x * t.wy[tb]);
        atomicAdd(dst + 1, vx.y * t.wy[tb]);
      }
    }
  }
}

// =====================================================================
// Generic path: LDS Stockham transforms (any 2,3,5-smooth K)
// =====================================================================
__global__ void __launch_bounds__(kThreads)
k_rows_fwd(ImgIn in, const float2* __restrict__ S, int L, int nx, int ny,
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
  const ImgScal bt = img_scal(in);
  for (int t = threadIdx.x; t < nl * Kx; t += blockDim.x) {
    const int li = t / Kx;
    const int j = t - li * Kx;
    const int ix = img_of_grid(j, nx, Kx);
    float2 v = make_float2(0.f, 0.f);
    if (ix >= 0) {
      const long long pix = (long long)iy * nx + ix;
      const float2 xv = img_at(in, (long long)iy * nx, ix, bt, li == 0 && blockIdx.y == 0);
      v = cscale(cmul(S[(long long)(l0 + li) * N + pix], xv), dax[ix] * sy);
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
                  int LS, const int* __restrict__ tile_off, const EntryRec* __restrict__ rec,
                  long long E, float2* __restrict__ ypart) {
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
    const Taps t = load_taps(rec, e);
    ypart[(long long)l * E + e] = interp_entry(t, g, LS, c0, tile, Kx, Ky);
  }
}

__global__ void __launch_bounds__(kThreads)
k_cols_adj_spread(const float2* __restrict__ yent, long long E,
                  int nx, int ny, int Kx, FFTDesc fd, int tile, int LS,
                  const int* __restrict__ tile_off, const EntryRec* __restrict__ rec,
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
    const Taps t = load_taps(rec, e);
    spread_entry(t, yent[(long long)l * E + e], a, LS, c0, tile, Kx, Ky);
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
           const float* __restrict__ dax, const float* __restrict__ day, FFTDesc fd,
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
  const float sy = day[iy];
  for (int ix = threadIdx.x; ix < nx; ix += blockDim.x) {
    const int jx = grid_of_img(ix, nx, Kx);
    const long long pix = (long long)iy * nx + ix;
    float2 acc = make_float2(0.f, 0.f);
    for (int li = 0; li < nl; ++li)
      acc = cadd(acc, cmulc(S[(long long)(l0 + li) * N + pix], r[li * Kx + jx]));
    part[(long long)g * N + pix] = cscale(acc, dax[ix] * sy);
  }
}

// =====================================================================
// Register path: four-step transforms, K = K1*K2
// =====================================================================
// RC coils per workgroup (static LDS: RC transpose blocks and one image
// row; RC = 8 only where it fits in 64 KB).  The 2D row kernels run on
// images of side K/2 (HALF), with 32-bit offsets (one coil group's mid and
// maps stay far below 4 GB).
template <int K1, int K2>
constexpr int fit_rc(int rc) {
  return ((size_t)rc * FS<K1, K2>::LA + FS<K1, K2>::K / 2) * sizeof(float2) <= 65536 ? rc : 4;
}

template <int K1, int K2, int RC>
__global__ void __launch_bounds__(RC * K1)
k_rows_fwd_fs(ImgIn in, const float2* __restrict__ S, int L, int nx, int ny,
              const float* __restrict__ dax, const float* __restrict__ day,
              const float2* __restrict__ tw, float2* __restrict__ mid) {
  __shared__ float2 A[RC * FS<K1, K2>::LA];
  __shared__ float2 X[FS<K1, K2>::K / 2];
  rows_fwd_body<K1, K2, RC, true, unsigned>(in, S, L, nx, ny, dax, day, tw, mid, blockIdx.x, blockIdx.y, A, X);
}

template <int K1, int K2>
__global__ void __launch_bounds__(8 * K1)
k_cols_fwd_fs(const float2* __restrict__ mid, int nx, int ny, int Kx, const float2* __restrict__ tw,
              int tile, const int* __restrict__ tile_off, const EntryRec* __restrict__ rec, long long E,
              float2* __restrict__ ypart) {
  using F = FS<K1, K2>;
  __shared__ float2 lds[8 * F::CSTR];
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  // (strip, coil) in XCD order, coil fastest: the coils of a strip run on one
  // XCD, so the strip's entry records come from that XCD's L2 after the first
  const int lin = xcd_order(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int s = lin / gridDim.y;
  const int l = lin % gridDim.y;
  const int c0 = s * tile;
  const bool colok = c < tile;
  // the zero-padded column transform (image rows ny = K/2), as in the Toeplitz pass
  float2 u[K2];
  col_fwd<K1, K2, true, unsigned>(mid + (long long)l * ny * Kx + c0, (unsigned)Kx, ny, colok, tw, lds, u);
  if (colok) {
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) lds[c * F::GS + t + K1 * k2] = u[k2];
  }
  __syncthreads();
  const int e0 = tile_off[s], e1 = tile_off[s + 1];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const Taps tp = load_taps(rec, e);
    ypart[(long long)l * E + e] = interp_entry(tp, lds, F::GS, c0, tile, Kx, F::K);
  }
}

// Image rows of an inverse column transform (grid rows j = t + K1 k2 of a
// zero-padded column, image side K/2: rows with P <= k2 < 3P, P = K2/4, are
// padding) stored into the strip whose column c of row i sits at
// strip[c + i * rs], as buffer stores at workgroup-uniform row offsets.
template <int K1, int K2>
__device__ __forceinline__ void store_image_rows(float2* __restrict__ strip, unsigned rs, int c, int t,
                                                 const float2 (&u)[K2]) {
  constexpr int P = K2 / 4;
  const auto rsrc = buf_rsrc(strip);
  const unsigned vo = ((unsigned)c + (unsigned)t * rs) * 8u;
#pragma unroll
  for (int k2 = 0; k2 < K2; ++k2) {
    if (k2 < P) buf_st2(rsrc, vo, (unsigned)(K1 * (k2 + P)) * rs * 8u, u[k2]);
    else if (k2 >= 3 * P) buf_st2(rsrc, vo, (unsigned)(K1 * (k2 - 3 * P)) * rs * 8u, u[k2]);
  }
}

constexpr int kAdjThreads = 256;    // = 8 * K1 for K1 = 32: every wave gathers and transforms
constexpr int kSpreadChunk = kAdjThreads;   // entries staged in LDS at a time, one per thread
constexpr int kAdjWaves = kAdjThreads / 64;
constexpr int kSpreadRB = 16;       // grid rows per spread block (the M side of one MFMA tile)
constexpr int kMaxDense = 4;        // dense row blocks per strip shared by all waves

typedef float f32x4 __attribute__((ext_vector_type(4)));

// LDS of the spread kernel: the grid strip, and -- while the entries are
// gathered -- the staged chunk (its MFMA operands), then the dense blocks'
// per-wave partial tiles; the three uses follow each other in time.
template <int K1, int K2>
struct AdjLds {
  static constexpr int STRIP = 8 * FS<K1, K2>::CSTR * 8;
  static constexpr int STAGE = kSpreadChunk * (16 + 8 + 1) * 4;   // B rows, row weights, first rows
  static constexpr int DENSE = kMaxDense * kAdjWaves * 256 * 4;
  static constexpr int M1 = STRIP > STAGE ? STRIP : STAGE;
  static constexpr int BYTES = M1 > DENSE ? M1 : DENSE;
};

// Type-1 spread by gathering, as dense products on the matrix cores.  A work
// item is a strip of 8 grid columns -- the whole strip, or part p of P of a
// heavy strip (the k-space centre), which takes every P-th staged chunk of
// the strip's entries starting at chunk p; the parts run as separate
// workgroups, write partial grid strips to their slots of `spart`, and
// k_cols_adj_fin_fs adds them in part order and transforms the strip.
//
// The kernel's weight factors over the two axes, so the contribution of a
// set of entries to a block of 16 grid rows of the strip is a product
//   G[r][c] += sum_e  wy_e(r - jy_e) * (w_e y_e) wx_e(c - jx_e)
// of a 16 x E matrix of row weights and an E x 8 complex matrix of weighted
// values times column weights (stored as 16 real columns, re then im): one
// v_mfma_f32_16x16x4_f32 takes four entries.  Staging a chunk computes each
// entry's B row once (its 16 values for this strip) and its row weights;
// the MFMA loop only places the row weights (lane row i of the block gets
// wy_e(16 rb + i - jy_e), or 0 outside the window).  Wave w of the four owns
// the row blocks rb = w, w + 4, ... and keeps their 16 x 16 tiles in registers,
// taking every entry whose first row tap lies within 5 rows above the block
// (entries are sorted by first row tap, row_start indexes them).  Up to
// kMaxDense blocks whose window holds dense_min or more entries (the most
// such blocks first: the densely sampled k-space centre) are shared by all
// waves instead: each wave takes a fixed slice of every staged chunk of the
// block's entries, and the four partial tiles are added in wave order.
// Each grid point is written once: no atomics, a fixed summation order.
template <int K1, int K2>
__global__ void __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(K1 * K2 >= 1024 ? 2 : 3)))
k_cols_adj_fs(KIn kin, const float* __restrict__ dcf, float scale,
              int nx, int ny, int Kx, const float2* __restrict__ tw, int tile,
              const int* __restrict__ tile_off, const int* __restrict__ row_start,
              const int4* __restrict__ items, int dense_min, const EntryRec* __restrict__ rec,
              float2* __restrict__ mid, float2* __restrict__ spart, int nslots) {
  using F = FS<K1, K2>;
  constexpr int NRB = F::K / kSpreadRB;                          // row blocks per strip
  constexpr int RBW = (NRB + kAdjWaves - 1) / kAdjWaves;         // row blocks per wave
  static_assert(F::K % kSpreadRB == 0, "row blocks tile the column");
  static_assert(kMaxDense <= kAdjWaves && 8 * K1 <= kAdjThreads, "one wave per dense block; FFT threads");
  __shared__ f32x4 U[AdjLds<K1, K2>::BYTES / 16];
  __shared__ int srs[F::K + 1];
  __shared__ int sdense[kMaxDense + 1];                          // count, then row blocks
  float2* lds = reinterpret_cast<float2*>(U);                    // the grid strip (after the gather)
  float* ldsf = reinterpret_cast<float*>(U);
  float* Bs = reinterpret_cast<float*>(U);                       // [chunk][16] B rows
  float* Wy = Bs + kSpreadChunk * 16;                            // [chunk][8] row weights
  int* Jy = reinterpret_cast<int*>(Wy + kSpreadChunk * 8);       // [chunk] first row tap
  f32x4* dpart = U;                                              // [dense][wave][lane] partial tiles
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;           // FFT threads: t < K1
  const int4 item = items[blockIdx.y];     // (strip, part, parts, first slot); heaviest first, coils adjacent
  const int s = item.x;
  const int l = blockIdx.x;
  const int c0 = s * tile;
  const bool colok = c < tile && t < K1;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;   // MFMA: A row / B column i16, K index k4
  const int e0 = tile_off[s], e1 = tile_off[s + 1];
  int cb = e0 + item.y * kSpreadChunk;
  // this thread's entry of the next chunk to stage, loaded ahead: first
  // taps, column and row weights, and the weighted k-space value
  // scale * w_m * y_l[m] of its sample m (y given, or the sum of the
  // sample's interpolation partials inside the normal operator)
  struct Staged {
    int jx, jy;
    float wx[6], wy[6];
    float2 v;
  } nx_e;
  auto fetch = [&](int cs) {
    const int e = cs + (int)threadIdx.x;
    if (cs < e1 && e < e1) {
      const EntryRec r = rec[e];
      nx_e.jx = r.idx.x;
      nx_e.jy = r.idx.y;
      nx_e.wx[0] = r.w0.x; nx_e.wx[1] = r.w0.y; nx_e.wx[2] = r.w0.z; nx_e.wx[3] = r.w0.w;
      nx_e.wx[4] = r.w1.x; nx_e.wx[5] = r.w1.y;
      nx_e.wy[0] = r.w1.z; nx_e.wy[1] = r.w1.w;
      nx_e.wy[2] = r.w2.x; nx_e.wy[3] = r.w2.y; nx_e.wy[4] = r.w2.z; nx_e.wy[5] = r.w2.w;
      const int m = r.idx.z;
      nx_e.v = cscale(k_at(kin, l, m), dcf ? dcf[m] * scale : scale);
    }
  };
  fetch(cb);
  for (int i = threadIdx.x; i <= F::K; i += blockDim.x) srs[i] = row_start[(long long)s * (F::K + 1) + i];
  __syncthreads();
  // entry range(s) of the window of row block rb: first row taps in
  // [16 rb - 5, 16 rb + 16), wrapped
  auto window = [&](int rb, int& ra0, int& rb0, int& ra1, int& rb1) {
    const int lo = rb * kSpreadRB - 5, hi = rb * kSpreadRB + kSpreadRB;
    if (lo >= 0) {
      ra0 = srs[lo]; rb0 = srs[hi]; ra1 = 0; rb1 = 0;
    } else {
      ra0 = srs[F::K + lo]; rb0 = srs[F::K]; ra1 = srs[0]; rb1 = srs[hi];
    }
  };
  static_assert(NRB <= 64, "one lane per row block");
  if (wave == 0) {
    // the kMaxDense fullest windows holding dense_min or more entries (ties:
    // lower block first), in that order; lane rb scores block rb
    int key = -1;
    if (lane < NRB) {
      int ra0, rb0, ra1, rb1;
      window(lane, ra0, rb0, ra1, rb1);
      const int n = (rb0 - ra0) + (rb1 - ra1);
      if (n >= dense_min) key = min(n, 1 << 24) * 64 + (63 - lane);
    }
    int nd = 0;
    for (int d = 0; d < kMaxDense; ++d) {
      int best = key;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) best = max(best, __shfl_xor(best, off));
      if (best < 0) break;
      if (lane == 0) sdense[1 + d] = 63 - (best & 63);
      if (key == best) key = -1;
      ++nd;
    }
    if (lane == 0) sdense[0] = nd;
  }
  f32x4 acc[RBW], accd[kMaxDense];
#pragma unroll
  for (int k = 0; k < RBW; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d < kMaxDense; ++d) accd[d] = f32x4{0.f, 0.f, 0.f, 0.f};
  // entries [ea, eb) of the staged chunk starting at cb into the 16-row block
  // starting at row0, four entries per MFMA and two MFMAs per step (all LDS
  // reads of a step issued first); lanes past eb get weight 0 and read a
  // valid slot.  ea and eb are wave-uniform.
  auto gather = [&](int ea, int eb, int row0, f32x4& a) {
    ea = __builtin_amdgcn_readfirstlane(ea);
    eb = __builtin_amdgcn_readfirstlane(eb);
    const int row = row0 + i16;
    for (int e = ea; e < eb; e += 8) {
      int ii[2], jy[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        ii[u] = min(e + 4 * u + k4, eb - 1) - cb;
        jy[u] = Jy[ii[u]];
      }
      float av[2], bv[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        int dy = row - jy[u];
        dy += dy < 0 ? F::K : 0;
        const bool ok = e + 4 * u + k4 < eb && dy < 6;
        av[u] = Wy[ii[u] * 8 + (ok ? dy : 0)];
        av[u] = ok ? av[u] : 0.f;
        bv[u] = Bs[ii[u] * 16 + i16];
      }
      a = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], bv[0], a, 0, 0, 0);
      a = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], bv[1], a, 0, 0, 0);
    }
  };
  for (; cb < e1; cb += item.z * kSpreadChunk) {
    const int n = min(kSpreadChunk, e1 - cb);
    __syncthreads();  // previous chunk consumed (and the dense list written)
    // staging: each thread forms its entry's B row (re and im of the 8 strip
    // columns) and stores its row weights, then loads its entry of the next
    // chunk, which arrives while this one is gathered
    if ((int)threadIdx.x < n) {
      const int i = threadIdx.x;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int gc = c0 + q;
        if (gc >= Kx) gc -= Kx;
        int dx = gc - nx_e.jx;
        dx += dx < 0 ? Kx : 0;
        float w = 0.f;
#pragma unroll
        for (int a = 0; a < 6; ++a) w = dx == a ? nx_e.wx[a] : w;
        Bs[i * 16 + q] = nx_e.v.x * w;
        Bs[i * 16 + 8 + q] = nx_e.v.y * w;
      }
      Jy[i] = nx_e.jy;
      *reinterpret_cast<float4*>(Wy + i * 8) = make_float4(nx_e.wy[0], nx_e.wy[1], nx_e.wy[2], nx_e.wy[3]);
      *reinterpret_cast<float2*>(Wy + i * 8 + 4) = make_float2(nx_e.wy[4], nx_e.wy[5]);
    }
    fetch(cb + item.z * kSpreadChunk);
    __syncthreads();
    const int ce = cb + n;
    const int nd = sdense[0];
#pragma unroll
    for (int k = 0; k < RBW; ++k) {
      const int rb = wave + k * kAdjWaves;
      bool shared = false;
#pragma unroll
      for (int d = 0; d < kMaxDense; ++d) shared |= d < nd && sdense[1 + d] == rb;
      if (rb < NRB && !shared) {
        int ra0, rb0, ra1, rb1;
        window(rb, ra0, rb0, ra1, rb1);
        gather(max(ra0, cb), min(rb0, ce), rb * kSpreadRB, acc[k]);
        gather(max(ra1, cb), min(rb1, ce), rb * kSpreadRB, acc[k]);
      }
    }
#pragma unroll
    for (int d = 0; d < kMaxDense; ++d) {
      if (d < nd) {
        const int rb = sdense[1 + d];
        int ra[2], rz[2];
        window(rb, ra[0], rz[0], ra[1], rz[1]);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
          const int ea = max(ra[part], cb), eb = min(rz[part], ce);
          if (ea < eb) {
            const long long len = eb - ea;
            gather(ea + (int)(len * wave / kAdjWaves), ea + (int)(len * (wave + 1) / kAdjWaves),
                   rb * kSpreadRB, accd[d]);
          }
        }
      }
    }
  }
  __syncthreads();                         // gather done: the staging area is free
  const int nd = sdense[0];
  f32x4 dsum = f32x4{0.f, 0.f, 0.f, 0.f};
  if (nd > 0) {                            // (uniform) dense partial tiles, added in wave order
#pragma unroll
    for (int d = 0; d < kMaxDense; ++d)
      if (d < nd) dpart[(d * kAdjWaves + wave) * 64 + lane] = accd[d];
    __syncthreads();
    if (wave < nd) {                       // wave d adds dense block d's tiles
      for (int w = 0; w < kAdjWaves; ++w) dsum += dpart[(wave * kAdjWaves + w) * 64 + lane];
    }
    __syncthreads();                       // tiles read: the strip may overwrite them
  }
  // tile element (4 k4 + j, i16) -> strip column i16 % 8 (re / im: i16 / 8)
  auto put = [&](int rb, const f32x4& a) {
    const int cc = i16 & 7, ri = i16 >> 3;
    if (cc < tile) {
#pragma unroll
      for (int j = 0; j < 4; ++j) ldsf[2 * (cc * F::GS + rb * kSpreadRB + 4 * k4 + j) + ri] = a[j];
    }
  };
#pragma unroll
  for (int k = 0; k < RBW; ++k) {
    const int rb = wave + k * kAdjWaves;
    bool shared = false;
#pragma unroll
    for (int d = 0; d < kMaxDense; ++d) shared |= d < nd && sdense[1 + d] == rb;
    if (rb < NRB && !shared) put(rb, acc[k]);
  }
  if (wave < nd) put(sdense[1 + wave], dsum);
  __syncthreads();
  if (item.w >= 0) {
    // a part: its partial grid strip to slot item.w + part (row-major, 8 columns)
    float2* sp = spart + ((long long)l * nslots + item.w + item.y) * F::K * 8;
    for (int i = threadIdx.x; i < F::K * 8; i += blockDim.x) sp[i] = lds[(i & 7) * F::GS + (i >> 3)];
    return;
  }
  float2 v[K1];
  if (colok && t < K2) {
#pragma unroll
    for (int n1 = 0; n1 < K1; ++n1) v[n1] = lds[c * F::GS + n1 * K2 + t];
  }
  __syncthreads();
  if (colok && t < K2) {
    reg::dft<K1, true>(v);
    fs_twiddle<K1, K2, true>(v, t, tw);
#pragma unroll
    for (int k1 = 0; k1 < K1; ++k1) lds[c * F::CS + k1 * F::AS + t] = v[k1];
  }
  __syncthreads();
  if (colok) {
    float2 u[K2];
#pragma unroll
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = lds[c * F::CS + t * F::AS + n2];
    reg::dft<K2, true>(u);
    store_image_rows<K1, K2>(mid + (long long)l * ny * Kx + c0, (unsigned)Kx, c, t, u);
  }
}

// grid strips of split items: the parts' partial strips added in part order,
// then the column inverse FFT and the image rows.  Every part's values of a
// thread's elements are loaded before any is added (all in flight at once);
// parts past the strip's count read as zero and are added last.
constexpr int kFinThreads = 1024;
constexpr int kMaxParts = 8;
template <int K1, int K2>
__global__ void __launch_bounds__(kFinThreads)
k_cols_adj_fin_fs(const float2* __restrict__ spart, int nslots, const int4* __restrict__ splits, int ny, int Kx,
                  const float2* __restrict__ tw, int tile, float2* __restrict__ mid) {
  using F = FS<K1, K2>;
  constexpr int NE = F::K * 8;                                   // elements of a strip
  constexpr int PER = (NE + kFinThreads - 1) / kFinThreads;      // per thread
  constexpr int R = PER <= 5 ? PER : (PER + 1) / 2;              // per round of loads
  __shared__ float2 lds[8 * F::CSTR];
  const int l = blockIdx.x;
  const int4 sp = splits[blockIdx.y];      // (strip, first slot, parts <= kMaxParts, 0)
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  const int c0 = sp.x * tile;
  const bool colok = c < tile && t < K1;
  const float2* src = spart + ((long long)l * nslots + sp.y) * NE;
  for (int j0 = 0; j0 < PER; j0 += R) {
    float2 b[kMaxParts][R];
#pragma unroll
    for (int q = 0; q < kMaxParts; ++q) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int i = (int)threadIdx.x + (j0 + j) * kFinThreads;
        b[q][j] = q < sp.z && i < NE ? src[(long long)q * NE + i] : make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int i = (int)threadIdx.x + (j0 + j) * kFinThreads;
      float2 a = b[0][j];
#pragma unroll
      for (int q = 1; q < kMaxParts; ++q) a = cadd(a, b[q][j]);
      if (i < NE) lds[(i & 7) * F::GS + (i >> 3)] = a;
    }
  }
  __syncthreads();
  float2 v[K1];
  if (colok && t < K2) {
#pragma unroll
    for (int n1 = 0; n1 < K1; ++n1) v[n1] = lds[c * F::GS + n1 * K2 + t];
  }
  __syncthreads();
  if (colok && t < K2) {
    reg::dft<K1, true>(v);
    fs_twiddle<K1, K2, true>(v, t, tw);
#pragma unroll
    for (int k1 = 0; k1 < K1; ++k1) lds[c * F::CS + k1 * F::AS + t] = v[k1];
  }
  __syncthreads();
  if (colok) {
    float2 u[K2];
#pragma unroll
    for (int n2 = 0; n2 < K2; ++n2) u[n2] = lds[c * F::CS + t * F::AS + n2];
    reg::dft<K2, true>(u);
    store_image_rows<K1, K2>(mid + (long long)l * ny * Kx + c0, (unsigned)Kx, c, t, u);
  }
}

template <int K1, int K2, int RC>
__global__ void __launch_bounds__(RC * K1)
k_rows_adj_fs(const float2* __restrict__ mid, const float2* __restrict__ S, int L, int nx, int ny,
              const float* __restrict__ dax, const float* __restrict__ day,
              const float2* __restrict__ tw, float2* __restrict__ part, FusedDots fd) {
  __shared__ float2 A[RC * FS<K1, K2>::LA];
  rows_adj_body<K1, K2, RC, true, unsigned>(mid, S, L, nx, ny, dax, day, tw, part, blockIdx.x, blockIdx.y, A, fd);
}

template <int K1, int K2>
__global__ void __launch_bounds__(8 * K1)
k_cols_toep_fs(float2* __restrict__ mid, int ny, int Kx, const float2* __restrict__ tw, int tile,
               const float* __restrict__ T) {
  __shared__ float2 lds[8 * FS<K1, K2>::CS];
  // (strip, coil) in XCD order, coil fastest: each XCD sweeps a contiguous
  // range of strips through all coils, so a strip's slice of T stays in its
  // L2 across the coils and neighbouring strips share cache lines there
  const int lin = xcd_order(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  cols_toep_body<K1, K2>(mid, ny, Kx, tw, tile, T, (lin / gridDim.y) * tile, lin % gridDim.y, lds);
}

// =====================================================================
// yent[l][e] = scale * w_m * y_l[m] for the sample m of entry e (y given, or
// the sum of the sample's interpolation partials inside the normal operator)
__global__ void k_entry_values(KIn kin, const EntryRec* __restrict__ rec, const float* __restrict__ dcf,
                               float scale, int L, float2* __restrict__ yent) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)L * kin.E) return;
  const int l = (int)(t / kin.E);
  const long long e = t - (long long)l * kin.E;
  const int m = rec[e].idx.z;
  yent[t] = cscale(k_at(kin, l, m), dcf ? dcf[m] * scale : scale);
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

// =====================================================================
// Batched Toeplitz normal operator: for each stage and each grid size, one
// launch runs the work items of all slices of that size, one workgroup per
// item: (slice, row, coil group) for the row passes, (slice, strip, coil)
// for the column pass.  Items are read in XCD order (xcd_order), so each
// XCD works through a contiguous range of the table, where the items that
// share data sit together -- the coil groups of one image row, the coils of
// one strip and its slice of T.  Two alternatives were measured and
// rejected on gfx950: a switch over sizes inside one kernel, and a
// persistent loop over items; both raise the register allocation (186-286
// VGPRs against 113-143 for one item per workgroup) and cost occupancy.
template <int K1, int K2>
__global__ void __launch_bounds__(kRowCoils * K1)
k_batch_rows_fwd(const BatchSlice* __restrict__ sl, const NormalIn* __restrict__ ins,
                 const int4* __restrict__ items, int n_items) {
  __shared__ float2 A[kRowCoils * FS<K1, K2>::LA];
  __shared__ float2 X[FS<K1, K2>::K / 2];
  const int4 w = items[xcd_order(blockIdx.x, n_items)];
  const BatchSlice& b = sl[w.x];
  const ImgIn in{ins[w.x].x, ins[w.x].cg};
  rows_fwd_body<K1, K2, kRowCoils, true, unsigned>(in, b.S, b.L, b.nx, b.ny, nullptr, nullptr, b.tw, b.mid, w.y, w.z,
                                                   A, X);
}

template <int K1, int K2>
__global__ void __launch_bounds__(8 * K1)
k_batch_cols_toep(const BatchSlice* __restrict__ sl, const int4* __restrict__ items, int n_items) {
  __shared__ float2 lds[8 * FS<K1, K2>::CS];
  const int4 w = items[xcd_order(blockIdx.x, n_items)];
  const BatchSlice& b = sl[w.x];
  cols_toep_body<K1, K2>(b.mid, b.ny, b.K, b.tw, 8, b.T, 8 * w.y, w.z, lds);
}

template <int K1, int K2>
__global__ void __launch_bounds__(kRowCoils * K1)
k_batch_rows_adj(const BatchSlice* __restrict__ sl, const int4* __restrict__ items, int n_items) {
  __shared__ float2 A[kRowCoils * FS<K1, K2>::LA];
  const int4 w = items[xcd_order(blockIdx.x, n_items)];
  const BatchSlice& b = sl[w.x];
  rows_adj_body<K1, K2, kRowCoils, true, unsigned>(b.mid, b.S, b.L, b.nx, b.ny, nullptr, nullptr, b.tw, b.part, w.y,
                                                   w.z, A, FusedDots{});
}

template <int K1, int K2>
struct BatchLaunch {
  static void rows_fwd(const BatchSlice* sl, const NormalIn* ins, const int4* items, int n, hipStream_t s) {
    PNP_LAUNCH((k_batch_rows_fwd<K1, K2>), dim3(n), dim3(kRowCoils * K1), 0, s, sl, ins, items, n);
  }
  static void cols_toep(const BatchSlice* sl, const int4* items, int n, hipStream_t s) {
    PNP_LAUNCH((k_batch_cols_toep<K1, K2>), dim3(n), dim3(8 * K1), 0, s, sl, items, n);
  }
  static void rows_adj(const BatchSlice* sl, const int4* items, int n, hipStream_t s) {
    PNP_LAUNCH((k_batch_rows_adj<K1, K2>), dim3(n), dim3(kRowCoils * K1), 0, s, sl, items, n);
  }
};

// ------------------------------------------------- register-path launchers
template <int K1, int K2>
struct FSLaunch {
  // the plan's coils per workgroup, as instantiated for this grid size
  // (adjoint and forward row passes)
  static int rc_of(const pnp_plan* p) {
    return p->row_coils == 2 ? 2 : (p->row_coils == 8 ? fit_rc<K1, K2>(8) : 4);
  }
  static int rc_fwd_of(const pnp_plan* p) {
    return p->row_coils_fwd == 2 ? 2 : (p->row_coils_fwd == 8 ? fit_rc<K1, K2>(8) : 4);
  }
  template <int RC>
  static void rows_fwd_rc(const pnp_plan* p, const ImgIn& in, const float2* S, int L, const float* dax,
                          const float* day, float2* mid, hipStream_t s) {
    PNP_LAUNCH((k_rows_fwd_fs<K1, K2, RC>), dim3(p->ax[1].n, (L + RC - 1) / RC), dim3(RC * K1), 0, s, in, S, L,
               p->ax[0].n, p->ax[1].n, dax, day, p->ax[0].fft.tw, mid);
  }
  template <int RC>
  static void rows_adj_rc(const pnp_plan* p, int L, const float2* mid, const float2* S, const float* dax,
                          const float* day, float2* part, const FusedDots& fd, hipStream_t s) {
    PNP_LAUNCH((k_rows_adj_fs<K1, K2, RC>), dim3(p->ax[1].n, (L + RC - 1) / RC), dim3(RC * K1), 0, s, mid, S, L,
               p->ax[0].n, p->ax[1].n, dax, day, p->ax[0].fft.tw, part, fd);
  }
  static void rows_fwd_any(const pnp_plan* p, const ImgIn& in, const float2* S, int L, const float* dax,
                           const float* day, float2* mid, hipStream_t s) {
    switch (rc_fwd_of(p)) {
      case 2: rows_fwd_rc<2>(p, in, S, L, dax, day, mid, s); break;
      case 8: rows_fwd_rc<fit_rc<K1, K2>(8)>(p, in, S, L, dax, day, mid, s); break;
      default: rows_fwd_rc<4>(p, in, S, L, dax, day, mid, s); break;
    }
  }
  static void rows_adj_any(const pnp_plan* p, int L, const float2* mid, const float2* S, const float* dax,
                           const float* day, float2* part, const FusedDots& fd, hipStream_t s) {
    switch (rc_of(p)) {
      case 2: rows_adj_rc<2>(p, L, mid, S, dax, day, part, fd, s); break;
      case 8: rows_adj_rc<fit_rc<K1, K2>(8)>(p, L, mid, S, dax, day, part, fd, s); break;
      default: rows_adj_rc<4>(p, L, mid, S, dax, day, part, fd, s); break;
    }
  }
  static void rows_fwd(const pnp_plan* p, const ImgIn& in, const float2* S, int L, float2* mid,
                       hipStream_t s) {
    rows_fwd_any(p, in, S, L, p->ax[0].deapod, p->ax[1].deapod, mid, s);
  }
  static void rows_coils(const pnp_plan* p, int* rc) { *rc = rc_of(p); }
  static void cols_fwd(const pnp_plan* p, int L, const float2* mid, float2* ypart, hipStream_t s) {
    PNP_LAUNCH((k_cols_fwd_fs<K1, K2>), dim3(p->ntx, L), dim3(8 * K1), 0, s, mid, p->ax[0].n,
               p->ax[1].n, p->ax[0].K, p->ax[1].fft.tw, p->tile, p->tile_off, p->rec,
               (long long)p->E, ypart);
  }
  static void cols_adj(const pnp_plan* p, int L, const KIn& kin, const float* dcf, float scale, float2* mid,
                       float2* spart, hipStream_t s) {
    PNP_LAUNCH((k_cols_adj_fs<K1, K2>), dim3(L, p->n_adj_items), dim3(kAdjThreads), 0, s, kin, dcf, scale,
               p->ax[0].n, p->ax[1].n, p->ax[0].K, p->ax[1].fft.tw, p->tile, p->tile_off,
               p->row_start, p->adj_items, p->adj_dense_min, p->rec, mid, spart, kMaxAdjSlots);
    if (p->n_adj_splits > 0)
      PNP_LAUNCH((k_cols_adj_fin_fs<K1, K2>), dim3(L, p->n_adj_splits), dim3(kFinThreads), 0, s, spart, kMaxAdjSlots,
                 p->adj_splits, p->ax[1].n, p->ax[0].K, p->ax[1].fft.tw, p->tile, mid);
  }
  static void rows_adj(const pnp_plan* p, int L, const float2* mid, const float2* S, float2* part,
                       hipStream_t s) {
    rows_adj_any(p, L, mid, S, p->ax[0].deapod, p->ax[1].deapod, part, FusedDots{}, s);
  }
  // Toeplitz variants: no deapodisation, column pass = FFT * T * IFFT
  static void rows_fwd_toep(const pnp_plan* p, const ImgIn& in, const float2* S, int L, float2* mid,
                            hipStream_t s) {
    rows_fwd_any(p, in, S, L, nullptr, nullptr, mid, s);
  }
  static void cols_toep(const pnp_plan* p, int L, const float* T, float2* mid, hipStream_t s) {
    PNP_LAUNCH((k_cols_toep_fs<K1, K2>), dim3(p->ntx, L), dim3(8 * K1), 0, s, mid, p->ax[1].n, p->ax[0].K,
               p->ax[1].fft.tw, p->tile, T);
  }
  static void rows_adj_toep(const pnp_plan* p, int L, const float2* mid, const float2* S, float2* part,
                            const FusedDots& fd, hipStream_t s) {
    rows_adj_any(p, L, mid, S, nullptr, nullptr, part, fd, s);
  }
};

// Calls FSLaunch<K1,K2>::fn(args...) for the register factorisation of K.
#define PNP_FS_DISPATCH(K, fn, ...)                                     \
  [&]() -> bool {                                                       \
    switch (K) {                                                        \
      case 128: FSLaunch<16, 8>::fn(__VA_ARGS__); return true;          \
      case 192: FSLaunch<16, 12>::fn(__VA_ARGS__); return true;         \
      case 256: FSLaunch<16, 16>::fn(__VA_ARGS__); return true;         \
      case 512: FSLaunch<32, 16>::fn(__VA_ARGS__); return true;         \
      case 640: FSLaunch<32, 20>::fn(__VA_ARGS__); return true;         \
      case 768: FSLaunch<32, 24>::fn(__VA_ARGS__); return true;         \
      case 1024: FSLaunch<32, 32>::fn(__VA_ARGS__); return true;        \
      default: return false;                                            \
    }                                                                   \
  }()

bool fs_ok(const pnp_plan* p) {
  return p->tile <= 8 && four_step_k1(p->ax[0].K) && four_step_k1(p->ax[1].K);
}

}  // namespace

bool toep_fused_dots(const pnp_toeplitz* tp) { return tp && tp->plan->ndim == 2 && fs_ok(tp->plan); }

int op_groups(const pnp_plan* p, int L) {
  if (p->ndim == 3) return op3_groups(L);
  int rc = kRowCoils;
  if (fs_ok(p)) {
    rc = 4;
    PNP_FS_DISPATCH(p->ax[0].K, rows_coils, p, &rc);
  }
  return (L + rc - 1) / rc;
}
int op_groups_max(int L) { return (L + 1) / 2; }
int batch_groups(int L) { return (L + kRowCoils - 1) / kRowCoils; }

size_t op_workspace_bytes(const pnp_plan* p, int L) {
  if (p->ndim == 3) return op3_workspace_bytes(p, L);
  const int Kx = p->ax[0].K;
  const int64_t N = image_size(p);
  const int G = std::max(op_groups_max(L), op_groups(p, L));
  size_t b = 0;
  b += al(sizeof(float2) * (size_t)L * p->ax[1].n * Kx);   // mid
  b += al(sizeof(float2) * (size_t)L * (size_t)std::max<int64_t>(p->E, 1));  // ypart
  b += al(sizeof(float2) * (size_t)L * p->M);             // ytmp
  b += al(sizeof(float2) * (size_t)L * (size_t)std::max<int64_t>(p->E, 1));  // yent
  b += al(sizeof(float2) * (size_t)G * N);                 // part
  b += al(sizeof(float2) * (size_t)L * kMaxAdjSlots * p->ax[1].K * 8);   // split strips of the spread
  return b;
}

OpWorkspace op_workspace(const pnp_plan* p, int L, void* ws) {
  if (p->ndim == 3) return op3_workspace(p, L, ws);
  OpWorkspace w{};
  const int Kx = p->ax[0].K;
  const int64_t N = image_size(p);
  const int G = std::max(op_groups_max(L), op_groups(p, L));
  char* c = (char*)ws;
  w.mid = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * p->ax[1].n * Kx);
  w.ypart = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * (size_t)std::max<int64_t>(p->E, 1));
  w.ytmp = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * p->M);
  w.yent = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * (size_t)std::max<int64_t>(p->E, 1));
  w.part = (float2*)c;
  c += al(sizeof(float2) * (size_t)G * N);
  w.spart = (float2*)c;
  c += al(sizeof(float2) * (size_t)L * kMaxAdjSlots * p->ax[1].K * 8);
  w.bytes = (size_t)(c - (char*)ws);
  return w;
}

void adj_build_items(pnp_plan* p, int split, int dense_min, hipStream_t s) {
  const int ns = p->ntiles, nrb = p->ax[1].K / 8;
  if (split < 0 || split > 3) fail(PNP_ERR_ARG, "spread split level %d outside 0..3", split);
  if (dense_min < 1) fail(PNP_ERR_ARG, "dense-block threshold %d must be >= 1", dense_min);
  // a strip's work: the entries of every row block's window
  std::vector<long long> cost(ns);
  for (int t = 0; t < ns; ++t) {
    long long c = 0;
    for (int rb = 0; rb < nrb; ++rb) c += p->adj_cost[(size_t)t * nrb + rb];
    cost[t] = c;
  }
  std::vector<long long> sorted(cost);
  std::sort(sorted.begin(), sorted.end());
  const long long median = std::max<long long>(1, sorted[ns / 2]);
  const long long target = split == 0 ? (1ll << 62) : median * (split == 1 ? 4 : split == 2 ? 2 : 1);
  std::vector<int> order(ns);
  for (int t = 0; t < ns; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  struct It { int4 v; long long c; };
  std::vector<It> items;
  std::vector<int4> splits;
  int slots = 0;
  for (int t : order) {
    int parts = (int)std::min<long long>(kMaxParts, (cost[t] + target - 1) / target);
    parts = std::min(parts, kMaxAdjSlots - slots);
    if (parts <= 1) {
      items.push_back({make_int4(t, 0, 1, -1), cost[t]});
      continue;
    }
    splits.push_back(make_int4(t, slots, parts, 0));
    for (int k = 0; k < parts; ++k) items.push_back({make_int4(t, k, parts, slots), cost[t] / parts});
    slots += parts;
  }
  std::stable_sort(items.begin(), items.end(), [](const It& a, const It& b) { return a.c > b.c; });
  std::vector<int4> v(items.size());
  for (size_t i = 0; i < items.size(); ++i) v[i] = items[i].v;
  PNP_HIP(hipMemcpyAsync(p->adj_items, v.data(), sizeof(int4) * v.size(), hipMemcpyHostToDevice, s));
  if (!splits.empty())
    PNP_HIP(hipMemcpyAsync(p->adj_splits, splits.data(), sizeof(int4) * splits.size(), hipMemcpyHostToDevice, s));
  PNP_HIP(hipStreamSynchronize(s));
  p->n_adj_items = (int)v.size();
  p->n_adj_splits = (int)splits.size();
  p->adj_split = split;
  p->adj_dense_min = dense_min;
}

// A 2D plan whose grid is served by the general passes must fit their LDS
// (the register-FFT sizes always do).
void nufft2d_check_plan(const pnp_plan* p) {
  if (fs_ok(p)) return;
  const size_t need = std::max(rows_lds(p->ax[0].K), cols_lds(p));
  if (need > 160 * 1024)
    fail(PNP_ERR_UNSUPPORTED, "grid %dx%d needs %zu bytes of LDS per workgroup (160 KB available)", p->ax[1].K,
         p->ax[0].K, need);
}

static void check_lds(const pnp_plan* p) { nufft2d_check_plan(p); }

// image -> per-entry interpolation partials in w.ypart
static void forward_to_partials(const pnp_plan* p, const ImgIn& in, const float2* smaps, int L,
                                const OpWorkspace& w, hipStream_t s) {
  const int nx = p->ax[0].n, ny = p->ax[1].n, Kx = p->ax[0].K;
  if (fs_ok(p)) {
    PNP_FS_DISPATCH(Kx, rows_fwd, p, in, smaps, L, w.mid, s);
    PNP_FS_DISPATCH(p->ax[1].K, cols_fwd, p, L, w.mid, w.ypart, s);
    return;
  }
  const int G = op_groups(p, L);
  check_lds(p);
  {
    const size_t lds = rows_lds(Kx);
    set_lds_limit((const void*)k_rows_fwd, lds);
    PNP_LAUNCH(k_rows_fwd, dim3(ny, G), dim3(kThreads), lds, s, in, smaps, L, nx, ny, p->ax[0].deapod,
               p->ax[1].deapod, p->ax[0].fft, w.mid);
  }
  {
    const size_t lds = cols_lds(p);
    set_lds_limit((const void*)k_cols_fwd_interp, lds);
    PNP_LAUNCH(k_cols_fwd_interp, dim3(p->ntx, L), dim3(kThreads), lds, s, w.mid, nx, ny, Kx,
               p->ax[1].fft, p->tile, col_stride(p->ax[1].K), p->tile_off, p->rec, (long long)p->E,
               w.ypart);
  }
}

// k-space (y or partials) -> per-coil-group partial images in `dst` [G][N]
static void adjoint_to_groups(const pnp_plan* p, const KIn& kin, const float2* smaps, int L,
                              const float* dcf, float scale, float2* dst, const OpWorkspace& w,
                              hipStream_t s) {
  const int nx = p->ax[0].n, ny = p->ax[1].n, Kx = p->ax[0].K;
  const int G = op_groups(p, L);
  if (fs_ok(p)) {   // the spread weights the k-space values as it stages them
    PNP_FS_DISPATCH(p->ax[1].K, cols_adj, p, L, kin, dcf, scale, w.mid, w.spart, s);
    PNP_FS_DISPATCH(Kx, rows_adj, p, L, w.mid, smaps, dst, s);
    return;
  }
  // weighted k-space values in entry order
  {
    const long long tot = (long long)L * p->E;
    if (tot > 0)
      PNP_LAUNCH(k_entry_values, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, kin, p->rec, dcf,
                 scale, L, w.yent);
  }
  check_lds(p);
  {
    const size_t lds = cols_lds(p);
    set_lds_limit((const void*)k_cols_adj_spread, lds);
    PNP_LAUNCH(k_cols_adj_spread, dim3(p->ntx, L), dim3(kThreads), lds, s, w.yent, (long long)p->E, nx,
               ny, Kx, p->ax[1].fft, p->tile, col_stride(p->ax[1].K), p->tile_off, p->rec, w.mid);
  }
  {
    const size_t lds = rows_lds(Kx);
    set_lds_limit((const void*)k_rows_adj, lds);
    PNP_LAUNCH(k_rows_adj, dim3(ny, G), dim3(kThreads), lds, s, w.mid, smaps, L, nx, ny,
               p->ax[0].deapod, p->ax[1].deapod, p->ax[0].fft, dst);
  }
}

void op_forward(const pnp_plan* p, const float2* x, const float2* smaps, int L, float2* y,
                const OpWorkspace& w, hipStream_t s) {
  if (p->ndim == 3) return op3_forward(p, x, smaps, L, y, w, s);
  forward_to_partials(p, ImgIn{x, CGUpdate{}}, smaps, L, w, s);
  const long long tot = p->M * L;
  const float scale = (float)(1.0 / std::sqrt((double)image_size(p)));
  PNP_LAUNCH(k_gather_entries, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, w.ypart,
             p->sample_ent, (long long)p->M, (long long)p->E, L, scale, y);
}

void op_adjoint(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf,
                float2* x, const OpWorkspace& w, hipStream_t s) {
  if (p->ndim == 3) return op3_adjoint(p, y, smaps, L, dcf, x, w, s);
  const int G = op_groups(p, L);
  const int64_t N = image_size(p);
  const float scale = (float)(1.0 / std::sqrt((double)N));
  float2* dst = G == 1 ? x : w.part;
  adjoint_to_groups(p, KIn{y, nullptr, nullptr, (long long)p->M, (long long)p->E}, smaps, L, dcf,
                    scale, dst, w, s);
  if (G > 1)
    PNP_LAUNCH(k_sum_groups, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w.part, G,
               (long long)N, x);
}

void op_adjoint_coils(const pnp_plan* p, const float2* y, int L, const float* dcf, const float2* ones,
                      float2* out, const OpWorkspace& w, hipStream_t s) {
  const int64_t N = image_size(p);
  if (p->ndim == 3) {
    for (int l = 0; l < L; ++l) op3_adjoint(p, y + (long long)l * p->M, ones, 1, dcf, out + l * N, w, s);
    return;
  }
  const int nx = p->ax[0].n, ny = p->ax[1].n, Kx = p->ax[0].K;
  const float scale = (float)(1.0 / std::sqrt((double)N));
  const KIn kin{y, nullptr, nullptr, (long long)p->M, (long long)p->E};
  const long long mstride = (long long)ny * Kx;               // one coil's half-transformed grid
  if (fs_ok(p)) {
    PNP_FS_DISPATCH(p->ax[1].K, cols_adj, p, L, kin, dcf, scale, w.mid, w.spart, s);
    for (int l = 0; l < L; ++l) PNP_FS_DISPATCH(Kx, rows_adj, p, 1, w.mid + l * mstride, ones, out + l * N, s);
    return;
  }
  const long long tot = (long long)L * p->E;
  if (tot > 0)
    PNP_LAUNCH(k_entry_values, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, kin, p->rec, dcf, scale, L,
               w.yent);
  check_lds(p);
  {
    const size_t lds = cols_lds(p);
    set_lds_limit((const void*)k_cols_adj_spread, lds);
    PNP_LAUNCH(k_cols_adj_spread, dim3(p->ntx, L), dim3(kThreads), lds, s, w.yent, (long long)p->E, nx,
               ny, Kx, p->ax[1].fft, p->tile, col_stride(p->ax[1].K), p->tile_off, p->rec, w.mid);
  }
  const size_t lds = rows_lds(Kx);
  set_lds_limit((const void*)k_rows_adj, lds);
  for (int l = 0; l < L; ++l)
    PNP_LAUNCH(k_rows_adj, dim3(ny, 1), dim3(kThreads), lds, s, w.mid + l * mstride, ones, 1, nx, ny,
               p->ax[0].deapod, p->ax[1].deapod, p->ax[0].fft, out + l * N);
}

void op_normal_parts(const pnp_plan* p, const NormalIn& in, const float2* smaps, int L,
                     const float* dcf, const OpWorkspace& w, hipStream_t s) {
  if (p->ndim == 3) return op3_normal_parts(p, in, smaps, L, dcf, w, s);
  forward_to_partials(p, ImgIn{in.x, in.cg}, smaps, L, w, s);
  const float scale = (float)(1.0 / (double)image_size(p));   // both N^{-1/2} factors
  adjoint_to_groups(p, KIn{nullptr, w.ypart, p->sample_ent, (long long)p->M, (long long)p->E}, smaps,
                    L, dcf, scale, w.part, w, s);
}

bool toeplitz_supported(const pnp_plan* p) { return p->ndim == 3 ? plan3_supported(p) : fs_ok(p); }

bool batch_grid_supported(int K) {
  return K == 128 || K == 192 || K == 256 || K == 512 || K == 640 || K == 768 || K == 1024;
}

#define PNP_BATCH_DISPATCH(K, fn, ...)                                   \
  do {                                                                  \
    switch (K) {                                                        \
      case 128: BatchLaunch<16, 8>::fn(__VA_ARGS__); break;             \
      case 192: BatchLaunch<16, 12>::fn(__VA_ARGS__); break;            \
      case 256: BatchLaunch<16, 16>::fn(__VA_ARGS__); break;            \
      case 512: BatchLaunch<32, 16>::fn(__VA_ARGS__); break;            \
      case 640: BatchLaunch<32, 20>::fn(__VA_ARGS__); break;            \
      case 768: BatchLaunch<32, 24>::fn(__VA_ARGS__); break;            \
      case 1024: BatchLaunch<32, 32>::fn(__VA_ARGS__); break;           \
      default: fail(PNP_ERR_UNSUPPORTED, "batched grid size %d", K);    \
    }                                                                   \
  } while (0)

void batch_rows_fwd(int K, const BatchSlice* sl, const NormalIn* ins, const int4* items, int n_items,
                    hipStream_t s) {
  if (n_items > 0) PNP_BATCH_DISPATCH(K, rows_fwd, sl, ins, items, n_items, s);
}

void batch_cols_toep(int K, const BatchSlice* sl, const int4* items, int n_items, hipStream_t s) {
  if (n_items > 0) PNP_BATCH_DISPATCH(K, cols_toep, sl, items, n_items, s);
}

void batch_rows_adj(int K, const BatchSlice* sl, const int4* items, int n_items, hipStream_t s) {
  if (n_items > 0) PNP_BATCH_DISPATCH(K, rows_adj, sl, items, n_items, s);
}

void op_normal_toep_parts(const pnp_toeplitz* tp, const NormalIn& in, const float2* smaps, int L,
                          const OpWorkspace& w, hipStream_t s) {
  const pnp_plan* p = tp->plan;
  if (p->ndim == 3) return op3_normal_toep_parts(tp, in, smaps, L, w, s);
  const ImgIn im{in.x, in.cg};
  PNP_FS_DISPATCH(p->ax[0].K, rows_fwd_toep, p, im, smaps, L, w.mid, s);
  PNP_FS_DISPATCH(p->ax[1].K, cols_toep, p, L, tp->T, w.mid, s);
  PNP_FS_DISPATCH(p->ax[0].K, rows_adj_toep, p, L, w.mid, smaps, w.part, in.fd, s);
}

void op_normal_toep(const pnp_toeplitz* tp, const float2* x, const float2* smaps, int L, float2* out,
                    const OpWorkspace& w, hipStream_t s) {
  op_normal_toep_parts(tp, plain_input(x), smaps, L, w, s);
  const int G = op_groups(tp->plan, L);
  const int64_t N = image_size(tp->plan);
  PNP_LAUNCH(k_sum_groups, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w.part, G,
             (long long)N, out);
}

void op_normal(const pnp_plan* p, const float2* x, const float2* smaps, int L, const float* dcf,
               float2* out, const OpWorkspace& w, hipStream_t s) {
  op_normal_parts(p, plain_input(x), smaps, L, dcf, w, s);
  const int G = op_groups(p, L);
  const int64_t N = image_size(p);
  PNP_LAUNCH(k_sum_groups, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w.part, G,
             (long long)N, out);
}

}  // namespace pnp
