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
//   adjoint:       type-1 spread into LDS-resident 8^3 grid tiles (no
//                  atomics), then the inverse z / y / x passes with crops,
//                  deapodisation, conj(S_l) and the coil-group sums
//   Toeplitz normal operator: x pass -> y pass -> z pass in place on g2
//                  (zero-padded FFT along z, times T, inverse, crop) ->
//                  inverse y pass -> inverse x pass with the coil sums; the
//                  full grid is never formed.
// The transfer function T is the DFT of the point-spread function
// psf[d] = N^{-1} sum_m w_m exp(i <k_m, d>), |d_a| < n_a, formed exactly in
// FP64 from per-axis Dirichlet tables (toeplitz.hip).
#include <algorithm>
#include <cstddef>
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
  rows_adj_body<K1, K2, kRowCoils3, HALF, OFF>(mid, S, L, nx, nrows, dax, dyz, tw, part, blockIdx.x, blockIdx.y, A,
                                               FusedDots{});
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
  // (set, strip) in XCD order, strip fastest: neighbouring strips -- the two
  // halves of each 128-byte line of a row -- run back to back on one XCD
  const int lin = xcd_order(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int set = lin / gridDim.x;
  const int a = set / cs.nb, b = set % cs.nb;
  const int c0 = (lin % gridDim.x) * 8;
  const float2* src = in + a * cs.in_sa + b * cs.in_sb + c0;
  float2* dst = out + a * cs.out_sa + b * cs.out_sb + c0;
  float2 u[K2];
  col_fwd<K1, K2, HALF, OFF>(src, (OFF)cs.rs_in, nimg, true, tw, lds, u);
  const OFF rb = (OFF)cs.rs_out * 8u, cb = (OFF)c * 8u + (OFF)t * rb;
  if constexpr (sizeof(OFF) == 4) {   // buffer stores: row offsets are workgroup-uniform
    const auto rsrc = buf_rsrc(dst);
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) buf_st2(rsrc, cb, (unsigned)(K1 * k2) * rb, u[k2]);
  } else {
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) st_off(dst, cb + (OFF)(K1 * k2) * rb, u[k2]);
  }
}

// inverse: all K rows -> image rows (nimg), cropped
template <int K1, int K2, bool HALF, typename OFF>
__global__ void __launch_bounds__(8 * K1)
k3_cols_inv(const float2* __restrict__ in, float2* __restrict__ out, ColSets cs, int nimg,
            const float2* __restrict__ tw) {
  __shared__ float2 lds[8 * FS<K1, K2>::CS];
  const int c = threadIdx.x % 8, t = threadIdx.x / 8;
  // (set, strip) in XCD order, strip fastest: neighbouring strips -- the two
  // halves of each 128-byte line of a row -- run back to back on one XCD
  const int lin = xcd_order(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int set = lin / gridDim.x;
  const int a = set / cs.nb, b = set % cs.nb;
  const int c0 = (lin % gridDim.x) * 8;
  const float2* src = in + a * cs.in_sa + b * cs.in_sb + c0;
  float2* dst = out + a * cs.out_sa + b * cs.out_sb + c0;
  float2 u[K2];
  const OFF rb = (OFF)cs.rs_in * 8u, cb = (OFF)c * 8u + (OFF)t * rb;
  if constexpr (sizeof(OFF) == 4) {
    const auto rsrc = buf_rsrc(src);
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = buf_ld2(rsrc, cb, (unsigned)(K1 * k2) * rb);
  } else {
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = ld_off(src, cb + (OFF)(K1 * k2) * rb);
  }
  col_inv<K1, K2, HALF, OFF>(dst, (OFF)cs.rs_out, nimg, true, tw, lds, u);
}

// z pass of the Toeplitz operator, in place on g2: sets (coil l, row ky),
// visited in XCD order with the coil fastest (T slices shared in L2; an
// order with neighbouring strips back to back measured 2% slower)
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
  if constexpr (sizeof(OFF) == 4) {
    const auto rsrc = buf_rsrc(Ts);
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = cscale(u[k2], buf_ld1(rsrc, cb, (unsigned)(K1 * k2) * tb));
  } else {
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = cscale(u[k2], ld_off(Ts, cb + (OFF)(K1 * k2) * tb));
  }
  col_inv<K1, K2, true, OFF>(strip, (OFF)plane, nz, true, tw, lds, u);
}

// type-2 interpolation from grid regions staged in LDS:
// y[l][m] = scale * (sum of the 6^3 taps of grid[l] around sample m).  A
// work item is a chunk of one 8^3 tile's home samples (first-tap cell in
// [t0, t0 + 8)^3), whose taps all lie in the 13^3 region [t0, t0 + 13)^3
// (mod K).  The workgroup stages that region for 2 coils in LDS
// ([z][y][x][coil], 35 KB; each point read once from the grid instead of
// once per tap), then lane (s, c) sums sample s's taps for coil c from LDS
// in the order of a direct gather: x fastest, then y, then z.  Two coils a
// workgroup keep four workgroups per CU staging at once (128^3 x 32 coils:
// 1, 2 and 4 coils per workgroup measured 6.40, 6.12 and 6.93 ms per
// forward operator).
constexpr int kI3C = 2;                  // coils per workgroup
constexpr int kI3R = 13;                 // staged region side: tile + kernel width - 1
constexpr int kI3Lds = kI3R * kI3R * kI3R * kI3C * (int)sizeof(float2);

__global__ void __launch_bounds__(256)
k3_interp_tiles(const float2* __restrict__ grid, int L, int Kx, int Ky, int Kz, long long M,
                const int32_t* __restrict__ cell_off, const int32_t* __restrict__ sorted_m,
                const int32_t* __restrict__ sjx, const float* __restrict__ sw, const int4* __restrict__ items,
                int nitems, float scale, float2* __restrict__ y) {
  extern __shared__ float4 lds_raw[];
  float2* const R = reinterpret_cast<float2*>(lds_raw);
  __shared__ int rbeg[64], rpre[64];
  // one workgroup per (item, coil group); each XCD takes a contiguous range
  // of items of one coil group, whose staged regions overlap in its L2
  const int lin = xcd_order(blockIdx.x, gridDim.x);
  const int4 it = items[lin % nitems];
  const int l0 = (lin / nitems) * kI3C;
  const int ntx = Kx / 8, nty = Ky / 8;
  const int t0x = (it.x % ntx) * 8, t0y = ((it.x / ntx) % nty) * 8, t0z = (it.x / (ntx * nty)) * 8;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {  // wave 0: the tile's 64 (z, y) rows, their sorted ranges and inclusive counts
    const long long row = ((long long)(t0z + (tid >> 3)) * Ky + t0y + (tid & 7)) * Kx + t0x;
    const int b = cell_off[row];
    int v = cell_off[row + 8] - b;
    rbeg[tid] = b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    rpre[tid] = v;
  }
  // stage the region: lane x (13 of 16 used) of region row (z, y, coil)
  // loads one point, in batches of 11 rows whose loads are all issued
  // before their stores; coordinates wrap mod K
  const long long vol = (long long)Kz * Ky * Kx;
  {
    constexpr int kRows = kI3R * kI3R * kI3C, kB = 11, kIt = (kRows + 16 * kB - 1) / (16 * kB);
    const int x = tid & 15;
    int gx = t0x + x;
    if (gx >= Kx) gx -= Kx;
#pragma unroll 1
    for (int b = 0; b < kIt; ++b) {
      float2 v[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int r = (tid >> 4) + 16 * (b * kB + u);
        const int c = r % kI3C, yz = r / kI3C, yy = yz % kI3R, zz = yz / kI3R;
        v[u] = make_float2(0.f, 0.f);
        if (x < kI3R && r < kRows && l0 + c < L) {
          int gy = t0y + yy, gz = t0z + zz;
          if (gy >= Ky) gy -= Ky;
          if (gz >= Kz) gz -= Kz;
          v[u] = grid[(long long)(l0 + c) * vol + ((long long)gz * Ky + gy) * Kx + gx];
        }
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const int r = (tid >> 4) + 16 * (b * kB + u);
        const int c = r % kI3C, yz = r / kI3C, yy = yz % kI3R, zz = yz / kI3R;
        if (x < kI3R && r < kRows) R[((zz * kI3R + yy) * kI3R + x) * kI3C + c] = v[u];
      }
    }
  }
  __syncthreads();
  const int c = tid % kI3C;
  for (int k = it.y + tid / kI3C; k < it.z; k += 256 / kI3C) {
    int lo = 0, hi = 63;                   // the row with rpre[r - 1] <= k < rpre[r]
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rpre[mid] > k) hi = mid;
      else lo = mid + 1;
    }
    const int i = rbeg[lo] + k - (lo > 0 ? rpre[lo - 1] : 0);
    const int dz = lo >> 3, dy = lo & 7, dx = sjx[i] - t0x;
    float w[3][6];
    const float2* wp = reinterpret_cast<const float2*>(sw + (long long)i * 18);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const float2 q = wp[e];
      w[(2 * e) / 6][(2 * e) % 6] = q.x;
      w[(2 * e + 1) / 6][(2 * e + 1) % 6] = q.y;
    }
    const float2* base = R + ((dz * kI3R + dy) * kI3R + dx) * kI3C + c;
    float2 acc = make_float2(0.f, 0.f);
    for (int tz = 0; tz < 6; ++tz) {
      float2 az = make_float2(0.f, 0.f);
#pragma unroll
      for (int ty = 0; ty < 6; ++ty) {
        const float2* row = base + (tz * kI3R + ty) * kI3R * kI3C;
        float2 ay = make_float2(0.f, 0.f);
#pragma unroll
        for (int tx = 0; tx < 6; ++tx) ay = cfma(w[0][tx], row[tx * kI3C], ay);
        az = cfma(w[1][ty], ay, az);
      }
      acc = cfma(w[2][tz], az, acc);
    }
    if (l0 + c < L) y[(long long)(l0 + c) * M + sorted_m[i]] = cscale(acc, scale);
  }
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

// type-1 spread into grid tiles on the matrix cores.  The grid is cut into
// 8^3 tiles; tile [t0, t0 + 8)^3 receives from the samples whose first-tap
// cell lies in [t0 - 5, t0 + 7] on every axis (mod K): 13 x 13 rows of 13
// cells, each row a contiguous range of the cell-sorted samples (two where x
// wraps).  One workgroup accumulates one work item -- a tile, or a chunk of
// a heavy tile's candidates -- for 16 coils.  The kernel's weight factors
// over the axes, so a block of 16 tile points (two rows of 8 at one z)
// receives
//   G[p][c] += sum_s  wz_s(z - dz_s) wy_s(y_p - dy_s) wx_s(x_p - dx_s) v_s[c]
// a 16 x S matrix of weight products (0 outside a sample's window) times an
// S x 16 matrix of the coil values (8 coils as re, im columns): one
// v_mfma_f32_16x16x4_f32 per four candidates and coil half.  The 32 blocks
// of the tile are dealt to the four waves diagonally (wave w owns, at each
// z, the row pair (w - z) mod 4), so the blocks a group of four neighbouring
// candidates touches spread over all waves; a wave skips, uniformly, the
// blocks outside the group's window.  Every tile point is summed by one
// lane in candidate order: no atomics, a fixed summation order.
// Candidates are staged kT3S at a time (weights, first-tap offsets relative
// to the tile, the 16 coil values).  The tile goes to the grid in 64-byte row
// segments, or to its partial slot (heavy tiles), which k3_fold_tiles adds up
// in slot order.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kT3C = 16;                 // coils per workgroup
constexpr int kT3S = 32;                 // staged candidates (a multiple of 32)
constexpr int kT3F = kT3S / 32;          // candidates per staging group of 8 threads
constexpr int kT3Rows = 13 * 13;         // candidate rows per tile
struct alignas(16) Spread3Lds {
  int rb0[kT3Rows], rc0[kT3Rows], rb1[kT3Rows];   // row: first range start / size, second range start
  int pre[256];                          // inclusive candidate counts up to each row (scan)
  alignas(16) float w[kT3S][20];         // x, y, z weights of the staged candidates (rows padded to 16 B)
  alignas(16) int d[kT3S][4];            // first tap relative to the tile (x, y, z), sorted index or -1
  float2 v[kT3S][kT3C];
  float out[4][16][33];                  // per wave: one finished block, [point][coil column]
};

// Four waves per SIMD: the accumulators then live in VGPRs (107, no spills)
// instead of 78 VGPRs + 64 AGPRs at three waves (128^3 x 32-coil adjoint
// 6.84 -> 6.42 ms, bit-identical).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k3_spread_tiles(const float2* __restrict__ ys, int L, const int32_t* __restrict__ cell_off,
                const int32_t* __restrict__ sjx, const float* __restrict__ sw, const int4* __restrict__ items,
                int Kx, int Ky, int Kz, float2* __restrict__ grid, float2* __restrict__ partial) {
  extern __shared__ float4 lds_raw[];
  Spread3Lds& S = *reinterpret_cast<Spread3Lds*>(lds_raw);
  static_assert(offsetof(Spread3Lds, d) % 16 == 0, "int4 reads of the staged offsets");
  const int4 it = items[blockIdx.x];
  const int l0 = blockIdx.y * kT3C;
  const int ntx = Kx / 8, nty = Ky / 8;
  const int t0x = (it.x % ntx) * 8, t0y = ((it.x / ntx) % nty) * 8, t0z = (it.x / (ntx * nty)) * 8;
  const int tid = threadIdx.x;
  // candidate rows (dz, dy) = (r / 13 - 5, r % 13 - 5), their sorted ranges
  // and the inclusive scan of their sizes (Hillis-Steele over 256 entries)
  int cnt = 0;
  if (tid < kT3Rows) {
    const int cz = (t0z - 5 + tid / 13 + Kz) % Kz, cy = (t0y - 5 + tid % 13 + Ky) % Ky;
    const long long row = ((long long)cz * Ky + cy) * Kx;
    const int x0 = t0x - 5;
    if (x0 >= 0) {
      const int b = cell_off[row + x0];
      S.rb0[tid] = b;
      S.rc0[tid] = cell_off[row + x0 + 13] - b;
      S.rb1[tid] = 0;
      cnt = S.rc0[tid];
    } else {
      const int b0 = cell_off[row + Kx + x0], b1 = cell_off[row];
      S.rb0[tid] = b0;
      S.rc0[tid] = cell_off[row + Kx] - b0;
      S.rb1[tid] = b1;
      cnt = S.rc0[tid] + cell_off[row + x0 + 13] - b1;
    }
  }
  S.pre[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int add = tid >= off ? S.pre[tid - off] : 0;
    __syncthreads();
    S.pre[tid] += add;
    __syncthreads();
  }

  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i16 = lane & 15, k4 = lane >> 4;   // MFMA: A row / B column i16, candidate k4 of a group
  const int px = i16 & 7, py = i16 >> 3;       // A row i16 = point (row pair + py, px) of a block
  // Staging of a round of kT3S candidates: candidate s = tid / 8 + 32 f is
  // located by the 8 threads (s mod 32, j) (the row with pre[r - 1] <= k <
  // pre[r], binary search), which load its 9 weight pairs and 16 coil values
  // (item j + 8 m of 25) into registers; the registers of the next round are
  // loaded while the current round is accumulated, and stored to LDS
  // between the two barriers that end it.  Slots past the item's end hold
  // zero weights and values.
  const int ss = tid >> 3, sj = tid & 7;
  int4 nd[kT3F];
  float2 nv[kT3F][4];
  auto fetch = [&](int kb) {
#pragma unroll
    for (int f = 0; f < kT3F; ++f) {
      const int k = kb + ss + 32 * f;
      nd[f] = make_int4(0, 0, 0, -1);
      if (k < it.z) {
        int lo = 0, hi = kT3Rows - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (S.pre[mid] > k) hi = mid;
          else lo = mid + 1;
        }
        const int o = k - (lo > 0 ? S.pre[lo - 1] : 0);
        const int i = o < S.rc0[lo] ? S.rb0[lo] + o : S.rb1[lo] + (o - S.rc0[lo]);
        nd[f] = make_int4(0, lo % 13 - 5, lo / 13 - 5, i);
        if (sj == 0) {
          int ddx = sjx[i] - t0x;
          if (ddx > 7) ddx -= Kx;
          nd[f].x = ddx;
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int e = sj + 8 * m;
        float2 val = make_float2(0.f, 0.f);
        if (nd[f].w >= 0 && e < 25) {
          if (e < 9) val = reinterpret_cast<const float2*>(sw + (long long)nd[f].w * 18)[e];
          else if (l0 + e - 9 < L) val = ys[(long long)nd[f].w * L + l0 + e - 9];
        }
        nv[f][m] = val;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int f = 0; f < kT3F; ++f) {
      const int slot = ss + 32 * f;
      if (sj == 0) *reinterpret_cast<int4*>(S.d[slot]) = nd[f];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int e = sj + 8 * m;
        if (e < 9) reinterpret_cast<float2*>(S.w[slot])[e] = nv[f][m];
        else if (e < 25) S.v[slot][e - 9] = nv[f][m];
      }
    }
  };
  // acc[z][h]: the wave's block at plane z, coils 8h .. 8h + 7
  f32x4 acc[8][2];
#pragma unroll
  for (int z = 0; z < 8; ++z) acc[z][0] = acc[z][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (it.y < it.z) {
    fetch(it.y);
    store();
  }
  __syncthreads();
  for (int k0 = it.y; k0 < it.z; k0 += kT3S) {
    const bool more = k0 + kT3S < it.z;
    if (more) fetch(k0 + kT3S);
    const int ns = min(kT3S, it.z - k0);
    for (int g = 0; g < ns; g += 4) {
      const int s = g + k4;
      const int4 dd = *reinterpret_cast<const int4*>(S.d[s]);
      // the group's window on z and y, clipped to the tile (wave-uniform)
      const int z0 = __builtin_amdgcn_readlane(dd.z, 0), z1 = __builtin_amdgcn_readlane(dd.z, 16);
      const int z2 = __builtin_amdgcn_readlane(dd.z, 32), z3 = __builtin_amdgcn_readlane(dd.z, 48);
      const int y0 = __builtin_amdgcn_readlane(dd.y, 0), y1 = __builtin_amdgcn_readlane(dd.y, 16);
      const int y2 = __builtin_amdgcn_readlane(dd.y, 32), y3 = __builtin_amdgcn_readlane(dd.y, 48);
      const int zlo = min(min(z0, z1), min(z2, z3)), zhi = max(max(z0, z1), max(z2, z3)) + 6;
      const int ylo = min(min(y0, y1), min(y2, y3)), yhi = max(max(y0, y1), max(y2, y3)) + 6;
      const float* ws = S.w[s];
      const int tx = px - dd.x;
      const float wx = ws[(unsigned)tx < 6u ? tx : 0];
      const float wxv = (unsigned)tx < 6u ? wx : 0.f;
      const float* vs = reinterpret_cast<const float*>(S.v[s]);
      const float b0 = vs[i16], b1 = vs[16 + i16];
#pragma unroll
      for (int z = 0; z < 8; ++z) {
        const int yp = (wv - z) & 3;
        if (z < zlo || z >= zhi || 2 * yp + 1 < ylo || 2 * yp >= yhi) continue;
        const int tz = z - dd.z, ty = 2 * yp + py - dd.y;
        const float wz = ws[12 + ((unsigned)tz < 6u ? tz : 0)];
        const float wy = ws[6 + ((unsigned)ty < 6u ? ty : 0)];
        const float a = ((unsigned)tz < 6u && (unsigned)ty < 6u) ? wz * wy * wxv : 0.f;
        acc[z][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b0, acc[z][0], 0, 0, 0);
        acc[z][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b1, acc[z][1], 0, 0, 0);
      }
    }
    __syncthreads();
    if (more) store();
    __syncthreads();
  }
  // write the tile block by block: the wave's block goes through its LDS
  // slot (tile element (4 k4 + r, i16) = point 4 k4 + r, coil column i16 of
  // half h), then each lane writes 4 points (32 B) of one coil row, a pair
  // of lanes one 64-byte row segment
  const long long plane = (long long)Ky * Kx, vol = plane * Kz;
  const int cc = lane >> 2, yy = (lane >> 1) & 1, xh = (lane & 1) * 4;
  const int col = (cc >> 3) * 16 + (cc & 7) * 2;
  float (*ob)[33] = S.out[wv];
#pragma unroll
  for (int z = 0; z < 8; ++z) {
    const int yp = (wv - z) & 3;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) ob[4 * k4 + r][16 * h + i16] = acc[z][h][r];
    __syncthreads();
    if (l0 + cc < L) {
      float4 q[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int pa = yy * 8 + xh + 2 * u;
        q[u] = make_float4(ob[pa][col], ob[pa][col + 1], ob[pa + 1][col], ob[pa + 1][col + 1]);
      }
      const int y = 2 * yp + yy;
      float4* dst = it.w < 0
          ? reinterpret_cast<float4*>(grid + (long long)(l0 + cc) * vol + (long long)(t0z + z) * plane +
                                      (long long)(t0y + y) * Kx + t0x + xh)
          : reinterpret_cast<float4*>(partial + ((long long)it.w * L + l0 + cc) * 512 + z * 64 + y * 8 + xh);
      dst[0] = q[0];
      dst[1] = q[1];
    }
    __syncthreads();
  }
}

// grid tile of a split tile = the sum of its partial slots, in slot order
// (workgroup: one fold, one coil)
__global__ void __launch_bounds__(256)
k3_fold_tiles(const float2* __restrict__ partial, const int4* __restrict__ folds, int L, int Kx, int Ky, int Kz,
              float2* __restrict__ grid) {
  const int4 f = folds[blockIdx.x];
  const int l = blockIdx.y;
  const int ntx = Kx / 8, nty = Ky / 8;
  const int t0x = (f.x % ntx) * 8, t0y = ((f.x / ntx) % nty) * 8, t0z = (f.x / (ntx * nty)) * 8;
  const long long plane = (long long)Ky * Kx, vol = plane * Kz;
  for (int pt = threadIdx.x; pt < 512; pt += 256) {
    float2 a = partial[((long long)f.y * L + l) * 512 + pt];
    for (int k = 1; k < f.z; ++k) a = cadd(a, partial[((long long)(f.y + k) * L + l) * 512 + pt]);
    const int x = pt & 7, y = (pt >> 3) & 7, zz = pt >> 6;
    grid[(long long)l * vol + (long long)(t0z + zz) * plane + (long long)(t0y + y) * Kx + t0x + x] = a;
  }
}

__global__ void k3_sum_groups(const float2* __restrict__ part, int G, long long N, float2* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float2 v = part[i];
  for (int g = 1; g < G; ++g) v = cadd(v, part[(long long)g * N + i]);
  out[i] = v;
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
  b += al3(sizeof(float2) * (size_t)std::max(p->sp_slots, 1) * L * 512);   // spread partial tiles
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
  c += al3(sizeof(float2) * (size_t)L * p->M);
  w.spart = (float2*)c;
  w.bytes = op3_workspace_bytes(p, L);
  return w;
}

// the oversampled coil grids -> k-space (every sample is the home sample of one tile item)
static void interp3(const pnp_plan* p, const Dims& d, int L, const float2* grid, float scale, float2* y,
                    hipStream_t s) {
  if (p->n_ip_items == 0) return;
  PNP_HIP(hipFuncSetAttribute((const void*)k3_interp_tiles, hipFuncAttributeMaxDynamicSharedMemorySize, kI3Lds));
  const long long nb = (long long)p->n_ip_items * ((L + kI3C - 1) / kI3C);
  if (nb >= (1ll << 31)) fail(PNP_ERR_SHAPE, "3D interpolation work list too long");
  PNP_LAUNCH(k3_interp_tiles, dim3((unsigned)nb), dim3(256), kI3Lds, s, grid, L, d.Kx, d.Ky, d.Kz, (long long)p->M,
             p->cell_off, p->sorted_m, p->sorted_jx, p->sorted_w, p->ip_items, p->n_ip_items, scale, y);
}

void op3_forward(const pnp_plan* p, const float2* x, const float2* smaps, int L, float2* y, const OpWorkspace& w,
                 hipStream_t s) {
  need3(p);
  const Dims d = dims_of(p);
  passes_fwd(p, d, ImgIn{x, CGUpdate{}}, smaps, L, p->ax[0].deapod, p->deapod_yz, w.mid, w.g2, w.grid, s);
  interp3(p, d, L, w.grid, (float)(1.0 / std::sqrt((double)d.N)), y, s);
}

// k-space y (or w.ytmp) -> coil-group partials in `dst`
static void adjoint_parts3(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf,
                           float scale, float2* dst, const OpWorkspace& w, hipStream_t s) {
  const Dims d = dims_of(p);
  const long long ML = p->M * L;
  PNP_LAUNCH(k3_sort_y, dim3((unsigned)((ML + 255) / 256)), dim3(256), 0, s, (long long)p->M, L, y, dcf,
             p->sorted_m, scale, w.ysort);
  PNP_HIP(hipFuncSetAttribute((const void*)k3_spread_tiles, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(Spread3Lds)));
  const unsigned cchunks = (unsigned)((L + kT3C - 1) / kT3C);
  PNP_LAUNCH(k3_spread_tiles, dim3((unsigned)p->n_sp_items, cchunks), dim3(256), sizeof(Spread3Lds), s, w.ysort, L,
             p->cell_off, p->sorted_jx, p->sorted_w, p->sp_items, d.Kx, d.Ky, d.Kz, w.grid, w.spart);
  if (p->n_sp_folds > 0)
    PNP_LAUNCH(k3_fold_tiles, dim3((unsigned)p->n_sp_folds, (unsigned)L), dim3(256), 0, s, w.spart, p->sp_folds, L,
               d.Kx, d.Ky, d.Kz, w.grid);
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
  interp3(p, d, L, w.grid, 1.0f, w.ytmp, s);
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


}  // namespace pnp
