// BF16 MFMA contractions of the UNet denoiser (forward and backward).
//
// Every convolution-like step is one GEMM C[M][N] = sum_k A(m,k) B(k,n)
// computed by k_mfma_gemm<View>: a 64x64 output tile per 256-thread
// workgroup (four waves, each a 32x32 quarter made of 2x2 16x16 MFMA
// blocks), K consumed 32 at a time with v_mfma_f32_16x16x32_bf16 (FP32
// accumulation), operands staged through LDS with the next K-step's global
// loads issued before the current step's MFMAs.
//
// A `View` describes one contraction:
//   AK / BK        false: loadA(m, k) / loadB(k, n) return 8 consecutive-k
//                  BF16 values of one row m / column n (operand contiguous in k)
//                  true:  loadA(k, m) / loadB(k, n) return 8 consecutive-m / -n
//                  values at one k (operand contiguous in m / n)
//   k_lo(z), k_hi(z)  the K range handled by grid slice z (split-K)
//   pre(m, n)      the epilogue's operand of element (m, n) read from memory
//                  (bias, ReLU-derivative mask as 1/0; 0 where none): the
//                  kernels read all of them before the first store, so the
//                  loads are not serialised behind stores that might alias
//   store(m, n, v, e) the epilogue (bias, ReLU, ReLU-derivative mask, BF16 or
//                  FP32 output, FP32 atomics for split-K weight gradients)
// Activations are NHWC BF16 with a per-tensor channel stride and offset, so
// the concatenated skip connections are channel slices, never copies.
// Channel counts, strides and offsets are multiples of 8 (16-byte loads).
#pragma once

#include <type_traits>

#include <cstring>

#include "common.hpp"

namespace pnp {
namespace unet {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// FP32 -> BF16, round to nearest even (NaN stays NaN, quieted); written as
// a select so that epilogues do not branch per element
__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const uint32_t quiet = (u >> 16) | 0x40u;
  return (uint16_t)((u & 0x7fffffffu) > 0x7f800000u ? quiet : rounded);
}
__host__ __device__ __forceinline__ float bf2f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
// a BF16 value is > 0 (ReLU derivative of a stored ReLU output)
__device__ __forceinline__ bool bf_pos(uint16_t h) { return h != 0 && !(h & 0x8000u); }

// An activation slice: NHWC, `cs` channels per pixel in memory, the slice
// starts at channel `co` and has `c` channels.
struct Act {
  uint16_t* p;
  int cs, co, c;
};

struct Geo {
  int B, H, W;   // batch and spatial size of the pixel space
  __device__ int P() const { return B * H * W; }
};

__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
// 16 zero bytes: the load address of lanes whose operand element is outside
// the tensor (a zero padding tap, a row past the end)
static __device__ __attribute__((aligned(16))) const uint32_t kZeroRow[4] = {0u, 0u, 0u, 0u};
// 16-byte load through the global address space (a pointer chosen between
// a tensor and kZeroRow would otherwise become a flat load, which the
// hardware counts together with the LDS accesses)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld16g(const uint16_t* p) {
  const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)(p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

// Waits once for every outstanding vector-memory load (vmcnt 0, the other
// counters left at their maximum): the epilogue operands have arrived, and
// the per-element stores that follow need no wait of their own.
__device__ __forceinline__ void epilogue_operands_ready() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ------------------------------------------------------------ the GEMM
template <class View>
__global__ void __launch_bounds__(256) k_mfma_gemm(View v) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64][40];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64][40];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  // loader coordinates: k-contiguous operands load row r = tid/4, k offset
  // 8*(tid%4); m/n-contiguous operands load k = tid/8, rows 8*(tid%8)..+7
  const int rr = tid >> 2, rk = (tid & 3) * 8;
  const int tk = tid >> 3, tr = (tid & 7) * 8;
  const int klo = v.k_lo(blockIdx.z), khi = v.k_hi(blockIdx.z);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto fetch = [&](int k0, uint4& a, uint4& b) {
    if constexpr (View::AK) a = v.loadA(k0 + tk, m0 + tr);
    else a = v.loadA(m0 + rr, k0 + rk);
    if constexpr (View::BK) b = v.loadB(k0 + tk, n0 + tr);
    else b = v.loadB(k0 + rk, n0 + rr);
  };
  auto put = [&](uint16_t (*S)[40], const uint4& val, bool kmajor) {
    if (!kmajor) {
      *reinterpret_cast<uint4*>(&S[rr][rk]) = val;
    } else {
      const uint32_t w[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        S[tr + 2 * i][tk] = (uint16_t)(w[i] & 0xffffu);
        S[tr + 2 * i + 1][tk] = (uint16_t)(w[i] >> 16);
      }
    }
  };

  uint4 na = zero4(), nb = zero4();
  if (klo < khi) fetch(klo, na, nb);
  for (int k0 = klo; k0 < khi; k0 += 32) {
    put(As, na, View::AK);
    put(Bs, nb, View::BK);
    __syncthreads();
    if (k0 + 32 < khi) fetch(k0 + 32, na, nb);
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // output block layout: lane holds rows 4*(lane/16) + q (q < 4) of column lane%16
  float e[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        e[i][j][q] = v.pre(m0 + wm + 16 * i + 4 * (lane >> 4) + q, n0 + wn + 16 * j + (lane & 15));
  epilogue_operands_ready();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        v.store(m0 + wm + 16 * i + 4 * (lane >> 4) + q, n0 + wn + 16 * j + (lane & 15), acc[i][j][q], e[i][j][q]);
}

// Offsets of the 3x3 taps (t = 3*(dy+1) + (dx+1)); a 1x1 convolution has one
// tap at offset 0.
__device__ __forceinline__ int tap_dy(int taps, int t) { return taps == 9 ? t / 3 - 1 : 0; }
__device__ __forceinline__ int tap_dx(int taps, int t) { return taps == 9 ? t % 3 - 1 : 0; }

// ReLU-derivative mask of a backward epilogue: channel n < mc of pixel m is
// kept only where the forward ReLU output (mask slice) is positive.
struct Mask {
  const uint16_t* p;   // nullptr: no mask
  int cs, co, mc;
  __device__ bool keep(int m, int n) const {
    return !p || n >= mc || bf_pos(p[(long long)m * cs + co + n]);
  }
  // keep() of element (m, n) when it lies in [0, P) x [0, nmax), else false;
  // the load is issued for every lane (clamped to element (0, 0))
  __device__ float keep_or_zero(int m, int n, int P, int nmax) const {
    const bool in = m < P && n < nmax;
    const bool chk = p && in && n < mc;
    const uint16_t* q = p ? p : reinterpret_cast<const uint16_t*>(kZeroRow);
    const uint16_t h = q[chk ? (long long)m * cs + co + n : 0ll];
    return in && (!chk || bf_pos(h)) ? 1.f : 0.f;
  }
};

// ------------------------------------------------------------ views
// Convolution ('same' zero padding, 3x3 or 1x1), forward:
//   out[p][n] = bias[n] + sum_{t, c} in[p + off(t)][c] W[n][t][c]
//   m = pixel, k = t*Cp + c, n = output channel.
struct ConvFwd {
  static constexpr bool AK = false, BK = false;
  static constexpr int TAP_SIGN = 1;      // k_gemm_tiled: input pixel = output pixel + tap offset
  Act in;
  const uint16_t* W;      // [Cout][taps][Cp] BF16
  const float* bias;      // [Cout] FP32
  Act out;                // BF16 output slice (unused when out_f32 is set)
  float* out_f32;         // [P][Cout] FP32 output, or nullptr
  Geo g;
  int taps, Cp, Cout, relu;
  int chunks;             // K chunks summed in order (k_gemm_tiled; 1 elsewhere)
  Act pool;               // k_conv3_halo: also the 2x2 max-pool of the output (pool.p == nullptr: none)
  // k_conv3_halo, a 32-channel output: also the network's 1 x 1 output layer
  // and residual (head_w == nullptr: none): head_o[p] = head_b + head_w . out[p]
  // (FP32, channels in order) and head_dst[p] = head_u[p] + head_o[p] when set
  const uint16_t* head_w;  // BF16 [2][32]
  const float* head_b;     // FP32 [2]
  const float2* head_u;
  float2* head_o;
  float2* head_dst;
  __device__ int k_lo(int) const { return 0; }
  __device__ int k_hi(int) const { return taps * Cp; }
  // start of output channel n's weights (k_gemm_tiled)
  __device__ const uint16_t* wrow(int n) const { return W + (long long)n * taps * Cp; }
  __device__ uint4 loadA(int m, int k) const {
    if (m >= g.P() || k >= taps * Cp) return zero4();
    const int t = k / Cp, c = k - t * Cp;
    const int x = m % g.W + tap_dx(taps, t), y = (m / g.W) % g.H + tap_dy(taps, t);
    if ((unsigned)y >= (unsigned)g.H || (unsigned)x >= (unsigned)g.W) return zero4();
    const long long pix = ((long long)(m / (g.W * g.H)) * g.H + y) * g.W + x;
    return ld16(in.p + pix * in.cs + in.co + c);
  }
  __device__ uint4 loadB(int k, int n) const {
    if (n >= Cout || k >= taps * Cp) return zero4();
    return ld16(W + (long long)n * taps * Cp + k);
  }
  __device__ float pre(int, int n) const {     // unconditional load (a clamped index)
    const float b = bias[n < Cout ? n : 0];
    return n < Cout ? b : 0.f;
  }
  // output pixels of rows m .. m+3 (k_gemm_tiled)
  __device__ void pix4(int m, long long (&o)[4]) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = m + q;
  }
  __device__ void store_px(int m, long long px, int n, float val, float b) const {
    if (m >= g.P() || n >= Cout) return;
    val += b;
    if (relu) val = fmaxf(val, 0.f);
    if (out_f32)
      out_f32[px * Cout + n] = val;
    else
      out.p[px * out.cs + out.co + n] = f2bf(val);
  }
  __device__ void store(int m, int n, float val, float b) const { store_px(m, m, n, val, b); }
  // coalesced BF16 epilogue of k_gemm_tiled: value of an element, output pixel
  __device__ bool vec_store() const { return out_f32 == nullptr; }
  __device__ float act(float val, float b) const {
    val += b;
    return relu ? fmaxf(val, 0.f) : val;
  }
  __device__ long long pix(int m) const { return m; }
  __device__ uint4 finish8(int, int, uint4 v8) const { return v8; }
};

// Forward convolution (view ConvFwd) and transposed convolution (UpFwd, one
// tap, grid z = the output sub-pixel) with larger output tiles (inference
// and training forward passes): a TM x TN tile per group of four waves, the waves
// arranged WM x (4/WM), each a (16 BI) x 32 block of BI x 2 MFMA tiles, LDS
// stages double-buffered (one barrier per step).  The K loop walks the taps
// and 32-channel chunks of the input (Cp a multiple of 32) in the order of
// k_mfma_gemm.  The layer's K steps form v.chunks equal chunks: each chunk
// is accumulated from zero and the chunk sums are added in order, so the
// result depends on the layer and the image size only; G = 1 runs the
// chunks one after the other, G = v.chunks runs them on G wave groups of
// one workgroup (256 G threads) combined in order through LDS -- the deep
// layers of one image launch a few tens of tiles, whose long K loops would
// otherwise run one wave per SIMD with nothing to hide their latency.
// CH = false instantiations serve single-chunk layers only (one set of
// accumulators).  A step's tap and chunk are tracked by counters (no
// division), each thread's pixel offset is formed once, and the global
// loads run D steps ahead of the MFMAs in a register ring.  TN = 32 serves
// the 32-channel layers without the half-empty tiles of the 64 x 64 kernel.
template <class V, int TM, int TN, int WM, int D, int G, bool CH>
__global__ void __launch_bounds__(256 * G) k_gemm_tiled(V v) {
  constexpr int WN = 4 / WM;
  constexpr int BI = TM / WM / 16, BJ = TN / WN / 16;
  static_assert((BI == 4 || BI == 2) && BJ == 2, "(16 BI) x 32 per wave");
  static_assert(D >= 1 && D <= 6, "prefetch depth");
  static_assert(CH || G == 1, "wave groups need chunk sums");
  constexpr int RA = TM / 64;                  // A rows per thread
  constexpr int STAGE = 2 * (TM + TN) * 40;    // BF16 elements of one group's A and B stages
  static_assert(G == 1 || (G - 1) * TM * TN * 2 <= G * STAGE, "LDS reduction fits in the stages");
  __shared__ __attribute__((aligned(16))) uint16_t lds[G * STAGE];
  const int grp = G == 1 ? 0 : (int)(threadIdx.x >> 8);
  const int tid = threadIdx.x & 255;
  uint16_t (*As)[TM][40] = reinterpret_cast<uint16_t (*)[TM][40]>(lds + grp * STAGE);
  uint16_t (*Bs)[TN][40] = reinterpret_cast<uint16_t (*)[TN][40]>(lds + grp * STAGE + 2 * TM * 40);
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int wm = (wave / WN) * (TM / WM), wn = (wave % WN) * (TN / WN);
  const int rr = tid >> 2, kq = (tid & 3) * 8;
  const int H = v.g.H, W = v.g.W;
  const int P = v.g.P();
  // this thread's A rows: pixel coordinates and element offset of the
  // centre tap (channel kq of the slice)
  int px[RA], py[RA];
  long long pa[RA];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int m = m0 + rr + 64 * i;
    px[i] = m % W;
    py[i] = m < P ? (m / W) % H : -(1 << 20);     // out-of-range rows fail the bounds test
    pa[i] = (long long)m * v.in.cs + v.in.co + kq;
  }
  // steps of this group and of one chunk (multiples of D, checked by the
  // launcher)
  const int cpc = v.Cp / 32;
  const int nsteps = v.taps * cpc;
  const int csteps = nsteps / v.chunks;
  const int sbeg = grp * (nsteps / G), send = sbeg + nsteps / G;
  const bool bload = tid < TN * 4;
  const int bn = n0 + (tid >> 2);
  const bool bok = bload && bn < v.Cout;
  // every load is issued unconditionally: out-of-range lanes read a row of
  // zeros in device memory, so no value needs a select after its load and
  // the loads stay in flight across the steps
  const uint16_t* const zrow = reinterpret_cast<const uint16_t*>(kZeroRow);
  const uint16_t* bp = bok ? v.wrow(bn) + kq : zrow;
  const int bstep = bok ? 32 : 0;
  // tap and channel offset of the next fetch, and of the group's last step
  int ft = sbeg / cpc, fc = (sbeg - ft * cpc) * 32;
  const int lt = (send - 1) / cpc, lc = (send - 1 - lt * cpc) * 32;
  auto fetch = [&](int step, uint4 (&a)[RA], uint4& b) {
    const int dy = V::TAP_SIGN * tap_dy(v.taps, ft), dx = V::TAP_SIGN * tap_dx(v.taps, ft);
    const long long toff = (long long)(dy * W + dx) * v.in.cs + fc;
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      const int y = py[i] + dy, x = px[i] + dx;
      const bool ok = (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
      a[i] = ld16g(ok ? v.in.p + pa[i] + toff : zrow);
    }
    b = ld16g(bp + (long long)step * bstep);
  };
  auto advance = [&]() {
    fc += 32;
    if (fc == v.Cp) {
      fc = 0;
      ++ft;
    }
  };
  f32x4 acc[BI][BJ], tot[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = tot[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 na[D][RA], nb[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    fetch(sbeg + d, na[d], nb[d]);
    advance();
  }
  int left = csteps;                           // steps left in the current chunk
  for (int s0 = sbeg; s0 < send; s0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int step = s0 + d;
      const int buf = step & 1;
#pragma unroll
      for (int i = 0; i < RA; ++i) *reinterpret_cast<uint4*>(&As[buf][rr + 64 * i][kq]) = na[d][i];
      if (bload) *reinterpret_cast<uint4*>(&Bs[buf][tid >> 2][kq]) = nb[d];
      __syncthreads();
      // the last D steps fetch the group's final step again (a valid
      // address; the values are never used)
      const bool more = step + D < send;
      if (!more) {
        ft = lt;
        fc = lc;
      }
      fetch(more ? step + D : send - 1, na[d], nb[d]);
      if (more) advance();
      bf16x8 a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < BJ; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if constexpr (CH) left -= D;
    if (CH && left == 0) {                     // end of a chunk: add its sum in order
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
          tot[i][j] += acc[i][j];
          acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      left = csteps;
    }
  }
  if constexpr (!CH) {
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) tot[i][j] = acc[i][j];
  }
  if constexpr (G > 1) {
    // groups 1..G-1 hand their chunk sums to group 0, which adds them in
    // chunk order (the stages are free once every group has left the loop)
    float* red = reinterpret_cast<float*>(lds);
    __syncthreads();
    if (grp > 0) {
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            red[((grp - 1) * TM + wm + 16 * i + 4 * (lane >> 4) + q) * TN + wn + 16 * j + (lane & 15)] =
                tot[i][j][q];
    }
    __syncthreads();
    if (grp > 0) return;
#pragma unroll
    for (int g = 1; g < G; ++g)
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            tot[i][j][q] += red[((g - 1) * TM + wm + 16 * i + 4 * (lane >> 4) + q) * TN + wn + 16 * j + (lane & 15)];
  }
  float e[BJ];                                   // the epilogue operand of this lane's columns (bias)
#pragma unroll
  for (int j = 0; j < BJ; ++j) e[j] = v.pre(0, n0 + wn + 16 * j + (lane & 15));
  epilogue_operands_ready();
  if (v.vec_store()) {
    // BF16 results of this wave's (16 BI) x 32 block staged in LDS, then
    // written 8 channels (16 bytes) per lane: whole 16-byte pieces of a
    // pixel's channel vector instead of 2-byte stores.  The staging area
    // lies past the wave-group partial sums; each wave uses its own part.
    constexpr int SROW = 32 + 8;                 // staged row, BF16 elements (80 bytes)
    constexpr int SOFF = G == 1 ? 0 : (G - 1) * TM * TN * 2;
    static_assert(SOFF + 4 * 16 * BI * SROW <= G * STAGE, "epilogue staging fits");
    if constexpr (G == 1) __syncthreads();     // the last K step's operands are consumed
    uint16_t* st = lds + SOFF + wave * (16 * BI * SROW);
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          st[(16 * i + 4 * (lane >> 4) + q) * SROW + 16 * j + (lane & 15)] = f2bf(v.act(tot[i][j][q], e[j]));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int it = lane; it < 16 * BI * 4; it += 64) {
      const int r = it >> 2, g8 = it & 3;
      const int m = m0 + wm + r;
      if (m < P) {
        const uint4 val = v.finish8(m, n0 + wn + 8 * g8, *reinterpret_cast<const uint4*>(&st[r * SROW + 8 * g8]));
        *reinterpret_cast<uint4*>(v.out.p + v.pix(m) * v.out.cs + v.out.co + n0 + wn + 8 * g8) = val;
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < BI; ++i) {
    const int mr = m0 + wm + 16 * i + 4 * (lane >> 4);
    long long px[4];
    v.pix4(mr, px);
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) v.store_px(mr + q, px[q], n0 + wn + 16 * j + (lane & 15), tot[i][j][q], e[j]);
  }
}

// First convolution of the network (3x3, Cp = 8 input channels -- Re, Im,
// sigma, zero padding -- and 32 outputs): K = 72 fits one LDS stage as 12
// tap slots of 8 channels (slots 9..11 zero), consumed in three 32-wide MFMA
// steps in the order of k_mfma_gemm (k = tap * 8 + channel), so the results
// are those of the generic kernel.  128 pixels per 256-thread workgroup;
// thread t stages slots 6 (t & 1) .. + 5 of pixel t / 2 (one coordinate
// decomposition each); wave w computes rows 32 w .. 32 w + 31, all columns.
// With fi.u, the input slots are formed here from the complex image and the
// noise level (Re, Im, sigma, zeros: as the packing pass forms them) instead
// of read, and the pixel's own slot is also stored to fi.x0 (the packed input
// the weight gradient of this layer reads).
struct FirstIn {
  const float2* u;     // [B][H][W]; nullptr: read the packed input v.in
  const float* sig;    // [B], or nullptr: sig_c for every image
  float sig_c;
  uint16_t* x0;        // [B H W][8] packed input written alongside
};
__global__ void __launch_bounds__(256) k_conv_first(ConvFwd v, FirstIn fi) {
  constexpr int TM = 128, LDA = 12 * 8 + 8;     // row stride in BF16 elements (padded)
  __shared__ __attribute__((aligned(16))) uint16_t As[TM][LDA];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[32][LDA];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * TM;
  const int H = v.g.H, W = v.g.W, P = v.g.P();
  const uint16_t* const zrow = reinterpret_cast<const uint16_t*>(kZeroRow);
  {
    const int r = tid >> 1, j0 = (tid & 1) * 6;
    const int m = m0 + r;
    const int px = m % W, py = m < P ? (m / W) % H : -(1 << 20);
    const long long pa = (long long)m * v.in.cs + v.in.co;
    const float sg = fi.u ? (fi.sig ? fi.sig[m < P ? m / (H * W) : 0] : fi.sig_c) : 0.f;
    const uint32_t sbf = f2bf(sg);
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
      const int j = j0 + jj;
      const int dy = j < 9 ? j / 3 - 1 : 0, dx = j < 9 ? j % 3 - 1 : 0;
      const int y = py + dy, x = px + dx;
      const bool ok = j < 9 && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
      uint4 slot;
      if (fi.u) {   // (uniform)
        const float2 uv = ok ? fi.u[(long long)m + dy * W + dx] : make_float2(0.f, 0.f);
        slot = ok ? make_uint4((uint32_t)f2bf(uv.x) | ((uint32_t)f2bf(uv.y) << 16), sbf, 0u, 0u)
                  : make_uint4(0u, 0u, 0u, 0u);
        if (j == 4 && m < P) *reinterpret_cast<uint4*>(fi.x0 + (long long)m * 8) = slot;
      } else {
        slot = ld16g(ok ? v.in.p + pa + (long long)(dy * W + dx) * v.in.cs : zrow);
      }
      *reinterpret_cast<uint4*>(&As[r][8 * j]) = slot;
    }
  }
  {
    const int n = tid >> 3;
    for (int j = tid & 7; j < 12; j += 8) {
      const bool ok = j < 9 && n < v.Cout;
      *reinterpret_cast<uint4*>(&Bs[n][8 * j]) = ld16g(ok ? v.W + (long long)n * 72 + 8 * j : zrow);
    }
  }
  __syncthreads();
  const int wm = 32 * wave;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + (lane & 15)][32 * ks + 8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(&Bs[16 * j + (lane & 15)][32 * ks + 8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  float e[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) e[j] = v.pre(0, 16 * j + (lane & 15));
  epilogue_operands_ready();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        v.store_px(m, m, 16 * j + (lane & 15), acc[i][j][q], e[j]);
      }
}

// Convolution, gradient of the input:
//   dIn[q][c] = sum_{t, o} dZ[q - off(t)][o] W[o][t][c]
//   m = pixel q, k = t*Coutp + o, n = c; B read from WT[Cin][taps][Coutp].
struct ConvDX {
  static constexpr bool AK = false, BK = false;
  Act dz;                 // gradient at the conv output (ReLU mask applied), c <= Coutp
  const uint16_t* WT;     // [Cin][taps][Coutp] BF16
  Act dx;                 // BF16 output slice
  Mask mask;              // ReLU mask of the input's producer
  Geo g;
  int taps, Coutp, Cin;
  __device__ int k_lo(int) const { return 0; }
  __device__ int k_hi(int) const { return taps * Coutp; }
  __device__ uint4 loadA(int m, int k) const {
    if (m >= g.P() || k >= taps * Coutp) return zero4();
    const int t = k / Coutp, c = k - t * Coutp;
    const int x = m % g.W - tap_dx(taps, t), y = (m / g.W) % g.H - tap_dy(taps, t);
    if ((unsigned)y >= (unsigned)g.H || (unsigned)x >= (unsigned)g.W) return zero4();
    const long long pix = ((long long)(m / (g.W * g.H)) * g.H + y) * g.W + x;
    return ld16(dz.p + pix * dz.cs + dz.co + c);
  }
  __device__ uint4 loadB(int k, int n) const {
    if (n >= Cin || k >= taps * Coutp) return zero4();
    return ld16(WT + (long long)n * taps * Coutp + k);
  }
  __device__ float pre(int m, int n) const { return mask.keep_or_zero(m, n, g.P(), Cin); }
  __device__ void store(int m, int n, float val, float keep) const {
    if (m >= g.P() || n >= Cin) return;
    if (keep == 0.f) val = 0.f;
    dx.p[(long long)m * dx.cs + dx.co + n] = f2bf(val);
  }
};

// The input gradient in the form k_gemm_tiled reads: in = dz, W = WT
// [Cin][taps][Coutp], out = dx, Cp = Coutp, Cout = Cin, taps mirrored.  The
// producer's ReLU mask is applied to each 16-byte output piece in the
// coalesced epilogue (a dropped element is BF16 zero, as in ConvDX::store).
struct ConvDXT {
  static constexpr int TAP_SIGN = -1;
  Act in;
  const uint16_t* W;
  Act out;
  Mask mask;
  Geo g;
  int taps, Cp, Cout, chunks;
  __device__ const uint16_t* wrow(int n) const { return W + (long long)n * taps * Cp; }
  __device__ float pre(int, int) const { return 0.f; }
  __device__ bool vec_store() const { return true; }
  __device__ float act(float val, float) const { return val; }
  __device__ long long pix(int m) const { return m; }
  // channels n .. n+7 of pixel m (mask.mc is a multiple of 8)
  __device__ uint4 finish8(int m, int n, uint4 v8) const {
    if (!mask.p || n >= mask.mc) return v8;
    const uint4 h = ld16(mask.p + (long long)m * mask.cs + mask.co + n);
    const uint32_t hw[4] = {h.x, h.y, h.z, h.w};
    uint32_t vw[4] = {v8.x, v8.y, v8.z, v8.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t lo = bf_pos((uint16_t)(hw[k] & 0xffffu)) ? 0x0000ffffu : 0u;
      const uint32_t hi = bf_pos((uint16_t)(hw[k] >> 16)) ? 0xffff0000u : 0u;
      vw[k] &= lo | hi;
    }
    return make_uint4(vw[0], vw[1], vw[2], vw[3]);
  }
  __device__ void pix4(int m, long long (&o)[4]) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = m + q;
  }
  __device__ void store_px(int, long long, int, float, float) const {}   // (vec_store is always true)
};

// Output pixel of the 2x2 stride-2 transposed convolution for input pixel m
// (geometry g) and tap t = 2a + b.
__device__ __forceinline__ long long up_pix(const Geo& g, int m, int t) {
  const int j = m % g.W, i = (m / g.W) % g.H, b = m / (g.W * g.H);
  return ((long long)b * 2 * g.H + 2 * i + (t >> 1)) * (2 * g.W) + 2 * j + (t & 1);
}

// 2x2 stride-2 transposed convolution, forward; grid slice z = tap t:
//   out[2i+a][2j+b][n] = bias[n] + sum_c in[i][j][c] W[n][t][c]
//   m = input pixel, k = c, n = output channel.
struct UpFwd {
  static constexpr bool AK = false, BK = false;
  static constexpr int TAP_SIGN = 1;
  Act in;
  const uint16_t* W;      // [Cout][4][Cin] BF16
  const float* bias;
  Act out;                // BF16 slice at twice the resolution
  Geo g;                  // input geometry
  int Cin, Cout;
  int taps, Cp, chunks;   // k_gemm_tiled: 1 tap, Cp = Cin, 1 chunk
  __device__ int k_lo(int) const { return 0; }
  __device__ int k_hi(int) const { return Cin; }
  __device__ const uint16_t* wrow(int n) const { return W + ((long long)n * 4 + blockIdx.z) * Cin; }
  __device__ uint4 loadA(int m, int k) const {
    if (m >= g.P() || k >= Cin) return zero4();
    return ld16(in.p + (long long)m * in.cs + in.co + k);
  }
  __device__ uint4 loadB(int k, int n) const {
    if (n >= Cout || k >= Cin) return zero4();
    return ld16(W + ((long long)n * 4 + blockIdx.z) * Cin + k);
  }
  __device__ float pre(int, int n) const {
    const float b = bias[n < Cout ? n : 0];
    return n < Cout ? b : 0.f;
  }
  // output pixels of input rows m .. m+3 for this grid slice's sub-pixel,
  // one division pair for the four (k_gemm_tiled)
  __device__ void pix4(int m, long long (&o)[4]) const {
    const int t = blockIdx.z;
    if (g.W >= 4) {
      int r = m / g.W;
      int j = m - r * g.W;
      int b = r / g.H;
      int i = r - b * g.H;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        o[q] = ((long long)b * 2 * g.H + 2 * i + (t >> 1)) * (2 * g.W) + 2 * j + (t & 1);
        if (++j == g.W) {
          j = 0;
          if (++i == g.H) {
            i = 0;
            ++b;
          }
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = up_pix(g, m + q, t);
    }
  }
  __device__ void store_px(int m, long long px, int n, float val, float b) const {
    if (m >= g.P() || n >= Cout) return;
    out.p[px * out.cs + out.co + n] = f2bf(val + b);
  }
  __device__ void store(int m, int n, float val, float b) const { store_px(m, up_pix(g, m, blockIdx.z), n, val, b); }
  __device__ bool vec_store() const { return true; }
  __device__ float act(float val, float b) const { return val + b; }
  __device__ long long pix(int m) const { return up_pix(g, m, blockIdx.z); }
  __device__ uint4 finish8(int, int, uint4 v8) const { return v8; }
};

// Transposed convolution, gradient of the input:
//   dIn[i][j][c] = sum_{t, o} dOut[2i+a][2j+b][o] W[o][t][c]
//   m = input pixel, k = t*Cout + o, n = c; B read from WT[Cin][4][Cout].
struct UpDX {
  static constexpr bool AK = false, BK = false;
  Act dout;               // slice at twice the resolution
  const uint16_t* WT;
  Act dx;
  Mask mask;
  Geo g;                  // input geometry
  int Cin, Cout;
  __device__ int k_lo(int) const { return 0; }
  __device__ int k_hi(int) const { return 4 * Cout; }
  __device__ uint4 loadA(int m, int k) const {
    if (m >= g.P() || k >= 4 * Cout) return zero4();
    const int t = k / Cout, o = k - t * Cout;
    return ld16(dout.p + up_pix(g, m, t) * dout.cs + dout.co + o);
  }
  __device__ uint4 loadB(int k, int n) const {
    if (n >= Cin || k >= 4 * Cout) return zero4();
    return ld16(WT + (long long)n * 4 * Cout + k);
  }
  __device__ float pre(int m, int n) const { return mask.keep_or_zero(m, n, g.P(), Cin); }
  __device__ void store(int m, int n, float val, float keep) const {
    if (m >= g.P() || n >= Cin) return;
    if (keep == 0.f) val = 0.f;
    dx.p[(long long)m * dx.cs + dx.co + n] = f2bf(val);
  }
};

// ------------------------------------------------ 3x3 convolution from an LDS halo tile
// 3x3 convolution for layers with CP (32, 64, 128 or 256) padded input channels
// -- the forward pass (view ConvFwd) or the input gradient (ConvDXT: input
// dZ, the transposed weights, mirrored taps, the producer's ReLU mask on the
// output) -- : a workgroup computes an 8 x 16-pixel output patch for TN (32
// or 64) output channels.  It stages the 10 x 18-pixel input patch (the 3x3
// halo, zeros outside the image) once in LDS; the K loop -- taps in order,
// 32 channels a step, as in k_gemm_tiled -- then reads every A fragment
// from LDS at a compile-time offset (16 pixels of one patch row, 8 channels
// a lane: one 16-byte read) and the B fragments straight from the BF16
// weights in global memory, already in the MFMA lane layout, RING steps
// ahead.  No barrier inside the K loop.  In a group of four waves the waves
// split the output channels (16 each: every weight is loaded by one wave
// only) and, for TN = 32, the patch rows in two halves.  Layers whose K
// range k_gemm_tiled sums in G chunks run G such groups, one per chunk,
// each from zero; group 0 adds the other groups' sums in chunk order.  The
// output goes through LDS and leaves as 16-byte pieces (8 channels of a
// pixel).  Per element, the sum order is k_gemm_tiled's (the same MFMA
// operands step by step, the same chunk sums), so results are bit-identical.
constexpr int kHaloPY = 8, kHaloPX = 16;    // output patch
template <int CP, int TN, int G>
struct Halo {
  static constexpr int PS = CP + 8;                      // BF16 per staged pixel (16-byte pad: no bank conflicts)
  static constexpr int HY = kHaloPY + 2, HX = kHaloPX + 2;
  static constexpr int ELEMS = HY * HX * PS;             // staged input (BF16)
  static constexpr int PIX = kHaloPY * kHaloPX;
  static constexpr int RED = (G - 1) * PIX * TN * 2;     // chunk sums of groups 1..G-1 (FP32, in BF16 units)
  static constexpr int OS = TN + 8;                      // output staging row (BF16 per pixel)
  static constexpr int OUT = RED + PIX * OS;
  static constexpr int LDS = ELEMS > OUT ? ELEMS : OUT;
  static constexpr int WN = TN / 16, WM = 4 / WN, BI = kHaloPY / WM;   // waves along N, along M; rows a wave
};

template <class V, int CP, int TN, int G>
__global__ void __launch_bounds__(256 * G) k_conv3_halo(V v) {
  constexpr bool FWD = std::is_same<V, ConvFwd>::value;
  using Hl = Halo<CP, TN, G>;
  constexpr int NSTEPS = 9 * (CP / 32);
  static_assert(NSTEPS % G == 0, "whole chunks");
  constexpr int CST = NSTEPS / G;                        // steps of one chunk
  constexpr int RING = CST < 8 ? CST : 8;
  constexpr int CHUNKS = Hl::HY * Hl::HX * (CP / 8);     // 16-byte pieces of the halo patch
  constexpr int CPT = (CHUNKS + 256 * G - 1) / (256 * G);
  constexpr int BI = Hl::BI;
  extern __shared__ __attribute__((aligned(16))) uint16_t L[];   // Hl::LDS elements (dynamic: CP = 256 needs 95 KB)
  const int tid = threadIdx.x, grp = tid >> 8, lane = tid & 63, wave = (tid & 255) >> 6;
  const int wn = wave % Hl::WN, wm = wave / Hl::WN;
  const int H = v.g.H, W = v.g.W;
  const int npx = (W + kHaloPX - 1) / kHaloPX, npy = (H + kHaloPY - 1) / kHaloPY;
  const int pb = blockIdx.x;
  const int bx = pb % npx, by = (pb / npx) % npy, b = pb / (npx * npy);
  const int x0 = bx * kHaloPX, y0 = by * kHaloPY;
  const int n0 = blockIdx.y * TN;
  const uint16_t* zrow = reinterpret_cast<const uint16_t*>(kZeroRow);
  // the halo patch first (the critical path): piece q = (pixel, 8-channel group), pixel = hy*HX + hx
  // (in batches of at most HB pieces a thread, the last batch held across the weight loads)
  constexpr int HB = CPT < 12 ? CPT : 12;
  uint4 h[HB];
  auto hload = [&](int u0) {
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      const int q = tid + 256 * G * (u0 + u);
      const int pix = q / (CP / 8), c8 = q - pix * (CP / 8);
      const int hy = pix / Hl::HX, hx = pix - hy * Hl::HX;
      const int y = y0 + hy - 1, x = x0 + hx - 1;
      const bool ok = u0 + u < CPT && q < CHUNKS && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
      const long long gp = ((long long)b * H + y) * W + x;
      h[u] = ld16g(ok ? v.in.p + gp * v.in.cs + v.in.co + 8 * c8 : zrow);
    }
  };
  auto hstore = [&](int u0) {
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      const int q = tid + 256 * G * (u0 + u);
      if (u0 + u < CPT && q < CHUNKS) {
        const int pix = q / (CP / 8), c8 = q - pix * (CP / 8);
        *reinterpret_cast<uint4*>(&L[pix * Hl::PS + 8 * c8]) = h[u];
      }
    }
  };
#pragma unroll
  for (int u0 = 0; u0 + HB < CPT; u0 += HB) {
    hload(u0);
    hstore(u0);
  }
  constexpr int HLAST = (CPT - 1) / HB * HB;
  hload(HLAST);
  // B fragments of this wave's 16 output channels for its group's chunk: lane (column lane%16,
  // k group lane/16), step s = tap*(CP/32) + cb at element offset 32 s of the channel's weights
  const int nb = n0 + 16 * wn + (lane & 15);
  const int s0 = grp * CST;
  const uint16_t* wb = nb < v.Cout ? v.W + (long long)nb * 9 * CP + 8 * (lane >> 4) + 32 * s0 : zrow;
  const int wstep = nb < v.Cout ? 32 : 0;
  uint4 rb[RING];
#pragma unroll
  for (int s = 0; s < RING; ++s) rb[s] = ld16g(wb + s * wstep);
  hstore(HLAST);
  __syncthreads();
  f32x4 acc[BI];
#pragma unroll
  for (int i = 0; i < BI; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  // A fragment base: patch row BI*wm + i, pixel lane%16, channels 8*(lane/16)
  const uint16_t* abase = L + ((BI * wm) * Hl::HX + (lane & 15)) * Hl::PS + 8 * (lane >> 4);
#pragma unroll
  for (int sl = 0; sl < CST; ++sl) {
    // step s = s0 + sl: tap t, channel block cb (runtime for G > 1: one offset add)
    const int s = s0 + sl;
    const int t = s / (CP / 32), cb = s % (CP / 32);
    // halo offsets of tap t: input = output + (t/3 - 1, t%3 - 1), mirrored for the input gradient
    const int dy = V::TAP_SIGN > 0 ? t / 3 : 2 - t / 3, dx = V::TAP_SIGN > 0 ? t % 3 : 2 - t % 3;
    const uint16_t* ap = abase + (dy * Hl::HX + dx) * Hl::PS + 32 * cb;
    const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&rb[sl % RING]);
    if (sl + RING < CST) rb[sl % RING] = ld16g(wb + (sl + RING) * wstep);
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      const bf16x8 fa = *reinterpret_cast<const bf16x8*>(ap + i * Hl::HX * Hl::PS);
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[i], 0, 0, 0);
    }
    // keep each step's LDS reads within the step (hoisting them across the
    // unrolled loop costs more registers than it hides latency)
    if constexpr (BI > 4) __builtin_amdgcn_sched_barrier(0);
  }
  const float bias = v.pre(0, nb);
  __syncthreads();                                     // every wave is done with the halo
  float* red = reinterpret_cast<float*>(L);
  uint16_t* ost = L + Hl::RED;
  if constexpr (G > 1) {
    // chunk sums: groups 1..G-1 through LDS, group 0 adds them in chunk order
    if (grp > 0) {
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pix = (BI * wm + i) * kHaloPX + 4 * (lane >> 4) + q;
          red[((grp - 1) * Hl::PIX + pix) * TN + 16 * wn + (lane & 15)] = acc[i][q];
        }
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int i = 0; i < BI; ++i) {
        f32x4 tot = f32x4{0.f, 0.f, 0.f, 0.f};
        tot += acc[i];
#pragma unroll
        for (int g = 1; g < G; ++g)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int pix = (BI * wm + i) * kHaloPX + 4 * (lane >> 4) + q;
            tot[q] += red[((g - 1) * Hl::PIX + pix) * TN + 16 * wn + (lane & 15)];
          }
        acc[i] = tot;
      }
    }
  }
  // epilogue: bias, ReLU, BF16 into LDS as [pixel][channel], then 16-byte stores
  if (grp == 0) {
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int pix = (BI * wm + i) * kHaloPX + 4 * (lane >> 4) + q;
        ost[pix * Hl::OS + 16 * wn + (lane & 15)] = f2bf(v.act(acc[i][q], bias));
      }
  }
  __syncthreads();
  constexpr int PIECES = Hl::PIX * (TN / 8);
#pragma unroll
  for (int u = 0; u < (PIECES + 256 * G - 1) / (256 * G); ++u) {
    const int q = tid + 256 * G * u;
    const int pix = q / (TN / 8), c8 = q % (TN / 8);
    const int y = y0 + pix / kHaloPX, x = x0 + pix % kHaloPX;
    const int n = n0 + 8 * c8;
    if (q < PIECES && y < H && x < W && n < v.Cout) {
      const long long gp = ((long long)b * H + y) * W + x;
      *reinterpret_cast<uint4*>(v.out.p + gp * v.out.cs + v.out.co + n) =
          v.finish8((int)gp, n, *reinterpret_cast<const uint4*>(&ost[pix * Hl::OS + 8 * c8]));
    }
  }
  // fused output layer: one thread per pixel, the dot products in channel
  // order as k_unet_head (TN = 32 = all channels in this workgroup)
  if constexpr (FWD && TN == 32) {
    if (v.head_w && tid < Hl::PIX) {
      const int y = y0 + tid / kHaloPX, x = x0 + tid % kHaloPX;
      if (y < H && x < W) {
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int c = 0; c < 32; ++c) {
          const float f = bf2f(ost[tid * Hl::OS + c]);
          a0 = fmaf(f, bf2f(v.head_w[c]), a0);
          a1 = fmaf(f, bf2f(v.head_w[32 + c]), a1);
        }
        const long long gp = ((long long)b * H + y) * W + x;
        const float2 r = make_float2(a0 + v.head_b[0], a1 + v.head_b[1]);
        v.head_o[gp] = r;
        if (v.head_dst) {
          const float2 uu = v.head_u[gp];
          v.head_dst[gp] = make_float2(uu.x + r.x, uu.y + r.y);
        }
      }
    }
  }
  // fused 2x2 max-pool (H, W even; the patch covers whole windows): the
  // first maximum in window order (0,0), (0,1), (1,0), (1,1), as k_unet_pool
  if constexpr (FWD) {
  if (v.pool.p) {
    constexpr int PP = (kHaloPY / 2) * (kHaloPX / 2) * (TN / 8);
#pragma unroll
    for (int u = 0; u < (PP + 256 * G - 1) / (256 * G); ++u) {
      const int q = tid + 256 * G * u;
      const int pp = q / (TN / 8), c8 = q % (TN / 8);
      const int py = pp / (kHaloPX / 2), px = pp % (kHaloPX / 2);
      const int y = (y0 >> 1) + py, x = (x0 >> 1) + px;
      const int n = n0 + 8 * c8;
      if (q < PP && 2 * y < H && 2 * x < W && n < v.Cout) {
        uint16_t best[8];
        float bv[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int pix = (2 * py + (k >> 1)) * kHaloPX + 2 * px + (k & 1);
          const uint4 w4 = *reinterpret_cast<const uint4*>(&ost[pix * Hl::OS + 8 * c8]);
          const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const uint16_t hv = (uint16_t)((w[c >> 1] >> (16 * (c & 1))) & 0xffffu);
            const float f = bf2f(hv);
            if (k == 0 || f > bv[c]) {
              bv[c] = f;
              best[c] = hv;
            }
          }
        }
        const long long gp = ((long long)b * (H >> 1) + y) * (W >> 1) + x;
        *reinterpret_cast<uint4*>(v.pool.p + gp * v.pool.cs + v.pool.co + n) =
            make_uint4(best[0] | ((uint32_t)best[1] << 16), best[2] | ((uint32_t)best[3] << 16),
                       best[4] | ((uint32_t)best[5] << 16), best[6] | ((uint32_t)best[7] << 16));
      }
    }
  }
  }
}

// ------------------------------------------------ weight gradients
// dW[m][n] = sum_p dZ[p][m] B[p][n] over the pixels p of a slice, with dZ
// the output gradient (m = output channel) and B the im2col row of the
// layer input (n = t*Cin + c; n = taps*Cin is the bias column of ones), so
// that the bias gradient is the last column.  For the 2x2 stride-2
// transposed convolutions p runs over input pixels and each tap t is a GEMM
// of its own: A(p, m) = dOut[output pixel of (p, t)][m], B(p, n) = in[p][n],
// N = Cin + 1.  Both operands are pixel-major in memory, 8 channels per
// 16-byte load; MFMA wants them channel-major (8 consecutive pixels of one
// channel per lane).  A thread owns a "slot" (8 channels x 8 consecutive
// pixels of one operand), loads it with 8 16-byte loads and transposes it
// in registers into 8 LDS rows of 16 bytes.  The 16-byte chunks of a row
// are XOR-swizzled so that both the transposing stores and the MFMA reads
// spread over the banks.  The next 128-pixel stage's loads are held in
// registers during the current stage's MFMAs.
//
// Pixel slice z owns pixels [z*kchunk, (z+1)*kchunk) and stores its partial
// tile with plain stores into part[t][z][M][N]; k_dw_reduce adds the slices
// up in a fixed order (deterministic, no atomics).  The grid is 1D over
// splits x tiles, splits a multiple of 8: the hardware deals workgroups to
// the 8 XCDs round-robin, so workgroup w runs slice (w mod 8) + 8*(w / 8 /
// tiles) -- every tile of a slice on one XCD, whose L2 then fetches the
// slice's operands once.
struct DWArgs {
  const uint16_t* dz;   // pixel p, channel m at dz[p*dzs + m] (output pixels for the transposed convolution)
  const uint16_t* in;   // pixel p, channel c at in[p*ins + c]
  float* part;          // [taps of the transposed convolution or 1][splits][M][N]
  int dzs, ins;
  int H, W, P;          // pixel space of the sum
  int taps, Cin, M, N;  // convolution: N = taps*Cin + 1; transposed convolution: taps = 1, N = Cin + 1
  int up;               // 1: transposed convolution (tile index = tap, N tile, M tile)
  int kchunk;           // a multiple of the 128-pixel stage
  int sx, sy;           // a step of 128 pixels: x += sx, y += sy, carry x into y, y mod H
  int mt, mn, tiles;    // M tiles; M x N tiles; all tiles (x 4 taps for the transposed convolution)
  int splits;
};

static __device__ __attribute__((aligned(16))) const uint32_t kOneRow[4] = {0x3f80u, 0u, 0u, 0u};

// LDS element offset of row r, 16-byte chunk c (16 chunks of 8 BF16 per row)
__device__ __forceinline__ int dw_lds(int r, int c) { return r * 128 + 8 * (c ^ ((r ^ (r >> 3)) & 7)); }

// ALIGNED: W % 8 == 0, so that the 8 pixels of a slot lie in one image row
// (and P, a multiple of 8, ends no slot part-way)
template <int TM, int TN, bool ALIGNED>
__global__ void __launch_bounds__(256) k_dw_gemm(DWArgs a) {
  static_assert((TM / 32) * (TN / 32) == 4, "four 32 x 32 wave blocks");
  constexpr int SA = 2 * TM, SB = 2 * TN;          // slots: (TM/8 channel groups) x (16 pixel chunks)
  constexpr int NS = (SA + SB + 255) / 256;         // slots per thread
  static_assert(SA % 64 == 0, "a wave's slots are all of one operand");
  __shared__ __attribute__((aligned(16))) uint16_t L[(TM + TN) * 128];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = blockIdx.x >> 3, zl = j / a.tiles, tile = j - zl * a.tiles;
  const int z = (blockIdx.x & 7) + 8 * zl;
  const int tap = tile / a.mn, mnt = tile - tap * a.mn;
  const int m0 = (mnt % a.mt) * TM, n0 = (mnt / a.mt) * TN;
  const int wm = (wave / (TN / 32)) * 32, wn = (wave % (TN / 32)) * 32;
  const int klo = min(z * a.kchunk, a.P), khi = min(klo + a.kchunk, a.P);
  const uint16_t* zrow = reinterpret_cast<const uint16_t*>(kZeroRow);

  // slot set-up: source address of pixel 0 (tap offset included), address
  // steps per pixel index and per image column, tap offset, LDS row, pixel
  // chunk, image position of the chunk's first pixel
  const uint16_t* src[NS];
  int stride[NS], xstride[NS], dx[NS], dy[NS], row[NS], chunk[NS], px[NS], py[NS];
  bool live[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int sl = tid + 256 * u;
    live[u] = sl < SA + SB;
    dx[u] = dy[u] = 0;
    xstride[u] = 0;
    if (sl < SA) {
      const int g = sl % (TM / 8), m = m0 + 8 * g;
      chunk[u] = sl / (TM / 8);
      row[u] = 8 * g;
      src[u] = m < a.M ? a.dz + m : zrow;
      stride[u] = m < a.M ? a.dzs : 0;
      if (a.up && m < a.M) {
        // output pixel of input pixel p = (b*H + y)*W + x, tap (ty, tx):
        // (b*2H + 2y + ty)*2W + 2x + tx = 4p - 2x + 2W*ty + tx
        src[u] += (long long)(2 * a.W * (tap >> 1) + (tap & 1)) * a.dzs;
        stride[u] = 4 * a.dzs;
        xstride[u] = -2 * a.dzs;
      }
    } else {
      const int s2 = min(sl, SA + SB - 1) - SA, g = s2 % (TN / 8), n = n0 + 8 * g;
      chunk[u] = s2 / (TN / 8);
      row[u] = TM + 8 * g;
      if (n < a.taps * a.Cin) {
        const int t = n / a.Cin, c = n - t * a.Cin;
        dy[u] = tap_dy(a.taps, t);
        dx[u] = tap_dx(a.taps, t);
        src[u] = a.in + c + (long long)(dy[u] * a.W + dx[u]) * a.ins;
        stride[u] = a.ins;
      } else {
        src[u] = n == a.taps * a.Cin ? reinterpret_cast<const uint16_t*>(kOneRow) : zrow;
        stride[u] = 0;
      }
    }
    const int p = klo + 8 * chunk[u];
    px[u] = p % a.W;
    py[u] = (p / a.W) % a.H;
  }
  uint4 r[NS][8];
  // loads of the stage at k0 (called for consecutive stages); then advances
  // the slot positions by one stage
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int p0 = k0 + 8 * chunk[u];
      const uint16_t* s0 = src[u] + (long long)p0 * stride[u] + (long long)px[u] * xstride[u];
      if constexpr (ALIGNED) {
        const bool rowok = live[u] && p0 < khi && (unsigned)(py[u] + dy[u]) < (unsigned)a.H;
        const bool lok = !(dx[u] < 0 && px[u] == 0), rok = !(dx[u] > 0 && px[u] + 8 == a.W);
        const int step = stride[u] + xstride[u];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = rowok && (e > 0 || lok) && (e < 7 || rok);
          r[u][e] = ld16g(ok ? s0 + e * step : zrow);
        }
      } else {
        int x = px[u], y = py[u];
        const uint16_t* s = s0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = live[u] && p0 + e < khi && (unsigned)(x + dx[u]) < (unsigned)a.W &&
                          (unsigned)(y + dy[u]) < (unsigned)a.H;
          r[u][e] = ld16g(ok ? s : zrow);
          s += stride[u] + xstride[u];
          if (++x == a.W) {
            x = 0;
            y = y + 1 == a.H ? 0 : y + 1;
            s -= (long long)a.W * xstride[u];
          }
        }
      }
      px[u] += a.sx;
      py[u] += a.sy;
      if (px[u] >= a.W) { px[u] -= a.W; ++py[u]; }
      if (py[u] >= a.H) py[u] -= a.H;
    }
  };
  // channel i of the 8 pixels -> one 16-byte row chunk
  auto put = [&]() {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      if (!live[u]) continue;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t sel = (i & 1) ? 0x07060302u : 0x05040100u;
        uint32_t w[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint4& v = r[u][e];
          w[e] = (i >> 1) == 0 ? v.x : (i >> 1) == 1 ? v.y : (i >> 1) == 2 ? v.z : v.w;
        }
        const uint4 o = make_uint4(__builtin_amdgcn_perm(w[1], w[0], sel), __builtin_amdgcn_perm(w[3], w[2], sel),
                                   __builtin_amdgcn_perm(w[5], w[4], sel), __builtin_amdgcn_perm(w[7], w[6], sel));
        *reinterpret_cast<uint4*>(&L[dw_lds(row[u] + i, chunk[u])]) = o;
      }
    }
  };

  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = f32x4{0.f, 0.f, 0.f, 0.f};
  if (klo < khi) fetch(klo);
  for (int k0 = klo; k0 < khi; k0 += 128) {
    put();
    __syncthreads();
    if (k0 + 128 < khi) fetch(k0 + 128);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      bf16x8 fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        fa[i] = *reinterpret_cast<const bf16x8*>(&L[dw_lds(wm + 16 * i + (lane & 15), 4 * ks + (lane >> 4))]);
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
        fb[jj] = *reinterpret_cast<const bf16x8*>(&L[dw_lds(TM + wn + 16 * jj + (lane & 15), 4 * ks + (lane >> 4))]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[jj], acc[i][jj], 0, 0, 0);
    }
    __syncthreads();
  }
  // partial tile: lane holds rows 4*(lane/16) + q of column lane%16 of each block
  float* out = a.part + ((long long)tap * a.splits + z) * a.M * a.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q, n = n0 + wn + 16 * jj + (lane & 15);
        if (m < a.M && n < a.N) out[(long long)m * a.N + n] = acc[i][jj][q];
      }
}

// The reductions of every layer's partial tiles, one launch.  Job j owns
// blocks [first[j], first[j+1]); a block of 256 threads takes E = 256/G
// consecutive gradient entries, thread (e, g) adds the slices
// [S'*g/G, S'*(g+1)/G) of entry e in order, and thread (e, 0) then adds the G
// sums in order: a fixed order for a given shape.
//   convolution, entry (m, n), S' = S: sum_z part[z][m][n]; n < N-1 -> dW[m][n], n = N-1 -> db[m]
//   transposed convolution, entry (m, t*Cin + c), S' = S: sum_z part[t][z][m][c] -> dW[m][t][c];
//   entry (m, 4*Cin), S' = 4S: sum over the 4 taps' slices of part[.][.][m][Cin] -> db[m]
struct DWJob {
  const float* part;
  float *dW, *db;
  int S, M, N, up, Cin, G;
  unsigned first;
};
constexpr int kMaxDWJobs = 18;
struct DWJobs {
  DWJob j[kMaxDWJobs];
  int n;
};

__global__ void __launch_bounds__(256) k_dw_reduce(DWJobs jobs) {
  __shared__ float red[256];
  int ji = 0;
  for (int k = 1; k < jobs.n; ++k)
    if (blockIdx.x >= jobs.j[k].first) ji = k;
  const DWJob& J = jobs.j[ji];
  const int E = 256 / J.G, e = threadIdx.x % E, g = threadIdx.x / E;
  const int per_row = J.up ? 4 * J.Cin + 1 : J.N;   // gradient entries of one output channel
  const long long cnt = (long long)J.M * per_row;
  const long long idx = (long long)(blockIdx.x - J.first) * E + e;
  const bool ok = idx < cnt;
  const int m = ok ? (int)(idx / per_row) : 0, n = ok ? (int)(idx - (long long)m * per_row) : 0;
  const bool bias = n == per_row - 1;
  // slices of this entry: address of slice k = base + k * step
  const long long MN = (long long)J.M * J.N;
  long long base, step = MN;
  int S2 = J.S;
  if (!J.up) {
    base = (long long)m * J.N + n;
  } else if (!bias) {
    const int t = n / J.Cin, c = n - t * J.Cin;
    base = (long long)t * J.S * MN + (long long)m * J.N + c;
  } else {
    base = (long long)m * J.N + J.Cin;
    S2 = 4 * J.S;
  }
  const int z0 = (int)((long long)S2 * g / J.G), z1 = (int)((long long)S2 * (g + 1) / J.G);
  float acc = 0.f;
  if (ok) {
#pragma unroll 4
    for (int k = z0; k < z1; ++k) acc += J.part[base + k * step];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (g != 0 || !ok) return;
  for (int h = 1; h < J.G; ++h) acc += red[h * E + e];
  if (bias)
    J.db[m] = acc;
  else
    J.dW[(long long)m * (per_row - 1) + n] = acc;
}

}  // namespace unet
}  // namespace pnp
