// The learned prior D_sigma(u): a four-scale UNet on the image's real and
// imaginary parts plus a constant noise-level channel (the denoiser is
// conditioned on sigma and acts on complex images as two real channels,
// Sec. 2.3 and Sec. 4.2), trained with an l1 loss and Adam (Sec. 4.2).
//
// Architecture (widths 32/64/128/256):
//   enc: [conv3x3+ReLU] x2 per scale, 2x2 max-pool between scales
//   dec: 2x2 stride-2 transposed conv, concat [skip, up], [conv3x3+ReLU] x2
//   out: 1x1 conv to 2 channels;  D_sigma(u) = u + out   (FP32 residual)
// BF16 weights and activations, FP32 accumulation (MFMA), FP32 master
// weights and Adam moments.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "trace.hpp"
#include "unet_kernels.hpp"

namespace pnp {

using unet::Act;
using unet::Geo;
using unet::Mask;
using unet::bf2f;
using unet::f2bf;

namespace {

enum LayerKind { kConv3 = 0, kConv1 = 1, kUp = 2 };

struct LayerInfo {
  int kind, cin, cp, cout, coutp, taps;
  long long w_off, b_off, wt_off;   // floats into the master / grad / moment buffers; WT elements
};

constexpr int kLayers = 18;
// e1a e1b | e2a e2b | e3a e3b | ba bb | up3 d3a d3b | up2 d2a d2b | up1 d1a d1b | out
constexpr int kDef[kLayers][3] = {
    {kConv3, 3, 32},    {kConv3, 32, 32},   {kConv3, 32, 64},   {kConv3, 64, 64},
    {kConv3, 64, 128},  {kConv3, 128, 128}, {kConv3, 128, 256}, {kConv3, 256, 256},
    {kUp, 256, 128},    {kConv3, 256, 128}, {kConv3, 128, 128},
    {kUp, 128, 64},     {kConv3, 128, 64},  {kConv3, 64, 64},
    {kUp, 64, 32},      {kConv3, 64, 32},   {kConv3, 32, 32},
    {kConv1, 32, 2}};
// resolution level (halvings of H and W) of the pixels each layer's weight
// gradient sums over: a convolution's own, a transposed convolution's input
constexpr int kDWLevel[kLayers] = {0, 0, 1, 1, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0};

struct NetLayout {
  LayerInfo L[kLayers];
  long long n_params;   // flat FP32 count (includes the zero input-channel padding)
  long long n_wt;       // transposed BF16 weight elements
  long long n_real;     // parameters without padding
};

const NetLayout& layout() {
  static const NetLayout lay = [] {
    NetLayout t{};
    long long off = 0, wt = 0, real = 0;
    for (int i = 0; i < kLayers; ++i) {
      LayerInfo& l = t.L[i];
      l.kind = kDef[i][0];
      l.cin = kDef[i][1];
      l.cout = kDef[i][2];
      l.cp = (l.cin + 7) / 8 * 8;
      l.coutp = (l.cout + 7) / 8 * 8;
      l.taps = l.kind == kConv3 ? 9 : (l.kind == kConv1 ? 1 : 4);
      l.w_off = off;
      l.b_off = off + (long long)l.cout * l.taps * l.cp;
      off = l.b_off + l.cout;
      l.wt_off = wt;
      if (i > 0) wt += (long long)l.cin * l.taps * l.coutp;   // the input layer needs no dX
      real += (long long)l.cout * l.taps * l.cin + l.cout;
    }
    t.n_params = off;
    t.n_wt = wt;
    t.n_real = real;
    return t;
  }();
  return lay;
}

constexpr int kThreads = 256;

inline unsigned blocks_for(long long n, int per = kThreads) { return (unsigned)((n + per - 1) / per); }

// ------------------------------------------------------------ kernels
// x0[p] = (bf(Re u), bf(Im u), bf(sigma_b), 0, ..., 0)
// grid (pixel blocks, image): the image index comes from the grid, not from
// a division per pixel
__global__ void k_unet_pack(const float2* __restrict__ u, const float* __restrict__ sig, float sig_c,
                            long long HW, uint16_t* __restrict__ x0) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= HW) return;
  const long long p = (long long)blockIdx.y * HW + i;
  const float2 v = u[p];
  const float s = sig ? sig[blockIdx.y] : sig_c;
  uint4 o;
  o.x = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
  o.y = (uint32_t)f2bf(s);
  o.z = 0u;
  o.w = 0u;
  *reinterpret_cast<uint4*>(x0 + p * 8) = o;
}

// 2x2 max-pool; go = output geometry, C channels (multiple of 8)
__global__ void k_unet_pool(Act in, Act out, Geo go, int C) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int chunks = C / 8;
  const long long P = (long long)go.B * go.H * go.W;
  if (idx >= P * chunks) return;
  const long long p = idx / chunks;
  const int c8 = (int)(idx - p * chunks) * 8;
  const int x = (int)(p % go.W), y = (int)((p / go.W) % go.H);
  const long long b = p / ((long long)go.W * go.H);
  const int Wi = 2 * go.W, Hi = 2 * go.H;
  uint16_t best[8];
  float bv[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long ip = (b * Hi + 2 * y + (q >> 1)) * Wi + 2 * x + (q & 1);
    const uint4 v = *reinterpret_cast<const uint4*>(in.p + ip * in.cs + in.co + c8);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint16_t h = (uint16_t)((w[c >> 1] >> (16 * (c & 1))) & 0xffffu);
      const float f = bf2f(h);
      if (q == 0 || f > bv[c]) {
        bv[c] = f;
        best[c] = h;
      }
    }
  }
  uint4 o;
  o.x = best[0] | ((uint32_t)best[1] << 16);
  o.y = best[2] | ((uint32_t)best[3] << 16);
  o.z = best[4] | ((uint32_t)best[5] << 16);
  o.w = best[6] | ((uint32_t)best[7] << 16);
  *reinterpret_cast<uint4*>(out.p + p * out.cs + out.co + c8) = o;
}

// Max-pool backward fused with the ReLU derivative of the pooled tensor:
// gin[argmax] += gout where fin[argmax] > 0 (argmax: first maximum in the
// order (0,0), (0,1), (1,0), (1,1)).  Each input pixel belongs to exactly
// one window, so the read-modify-write is race free.
__global__ void k_unet_pool_bwd(Act fin, Act gout, Act gin, Geo go, int C) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long P = (long long)go.B * go.H * go.W;
  if (idx >= P * C) return;
  const long long p = idx / C;
  const int c = (int)(idx - p * C);
  const int x = (int)(p % go.W), y = (int)((p / go.W) % go.H);
  const long long b = p / ((long long)go.W * go.H);
  const int Wi = 2 * go.W, Hi = 2 * go.H;
  long long arg = 0;
  float bv = 0.f;
  uint16_t bh = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long ip = (b * Hi + 2 * y + (q >> 1)) * Wi + 2 * x + (q & 1);
    const uint16_t h = fin.p[ip * fin.cs + fin.co + c];
    const float f = bf2f(h);
    if (q == 0 || f > bv) {
      bv = f;
      bh = h;
      arg = ip;
    }
  }
  if (!unet::bf_pos(bh)) return;
  uint16_t* dst = gin.p + arg * gin.cs + gin.co + c;
  *dst = f2bf(bf2f(*dst) + bf2f(gout.p[p * gout.cs + gout.co + c]));
}

// Output layer (1 x 1 convolution, 32 -> 2 channels) and residual, one
// thread per pixel: o[p] = b + W d[p] in FP32 (the network output, kept for
// the loss) and, when dst is set, dst[p] = u[p] + o[p].  d: BF16 [P][32];
// W: BF16 [2][32]; b: FP32 [2].
__global__ void __launch_bounds__(kThreads) k_unet_head(const uint16_t* __restrict__ d,
                                                        const uint16_t* __restrict__ W,
                                                        const float* __restrict__ b,
                                                        const float2* __restrict__ u, long long P,
                                                        float2* __restrict__ o, float2* __restrict__ dst) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float a0 = 0.f, a1 = 0.f;
#pragma unroll
  for (int c8 = 0; c8 < 4; ++c8) {
    const uint4 q = *reinterpret_cast<const uint4*>(d + p * 32 + 8 * c8);
    const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float f = unet::bf2f((uint16_t)(w4[e >> 1] >> (16 * (e & 1))));
      a0 = fmaf(f, unet::bf2f(W[8 * c8 + e]), a0);
      a1 = fmaf(f, unet::bf2f(W[32 + 8 * c8 + e]), a1);
    }
  }
  const float2 r = make_float2(a0 + b[0], a1 + b[1]);
  o[p] = r;
  if (dst) {
    const float2 x = u[p];
    dst[p] = make_float2(x.x + r.x, x.y + r.y);
  }
}

__device__ __forceinline__ float sgnf(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// l1 loss of D(u) = u + out against the target, mean over the 2P real
// values; gout = d loss / d out in BF16 (channels 2..7 zero).  loss must be
// zero on entry.
__global__ void __launch_bounds__(kThreads) k_unet_l1(const float2* __restrict__ u, const float2* __restrict__ o,
                                                      const float2* __restrict__ t, long long P, float scale,
                                                      uint16_t* __restrict__ gout, double* __restrict__ loss) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (long long)gridDim.x * blockDim.x) {
    const float2 a = u[p], b = o[p], c = t[p];
    const float dx = (a.x + b.x) - c.x, dy = (a.y + b.y) - c.y;
    acc += (double)fabsf(dx) + (double)fabsf(dy);
    uint4 g;
    g.x = (uint32_t)f2bf(sgnf(dx) * scale) | ((uint32_t)f2bf(sgnf(dy) * scale) << 16);
    g.y = 0u;
    g.z = 0u;
    g.w = 0u;
    *reinterpret_cast<uint4*>(gout + p * 8) = g;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * (double)scale);
}

// Neighbor2Neighbor sub-samplers: in every 2 x 2 cell (i, j) of image b,
// code c picks an ordered pair of 4-adjacent pixels, the first to g1 and
// the second to g2 (offsets (dy, dx) within the cell):
//   0 (0,0)(0,1)  1 (0,0)(1,0)  2 (0,1)(0,0)  3 (0,1)(1,1)
//   4 (1,0)(0,0)  5 (1,0)(1,1)  6 (1,1)(0,1)  7 (1,1)(1,0)
__constant__ int8_t kN2NPair[8][4] = {{0, 0, 0, 1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {0, 1, 1, 1},
                                      {1, 0, 0, 0}, {1, 0, 1, 1}, {1, 1, 0, 1}, {1, 1, 1, 0}};
__device__ __forceinline__ void n2n_pair(int code, int& a1, int& b1, int& a2, int& b2) {
  const int c = code & 7;
  a1 = kN2NPair[c][0];
  b1 = kN2NPair[c][1];
  a2 = kN2NPair[c][2];
  b2 = kN2NPair[c][3];
}

__global__ void __launch_bounds__(kThreads) k_n2n_sub(const float2* __restrict__ x, const uint8_t* __restrict__ codes,
                                                      int h, int w, long long P, float2* __restrict__ g1,
                                                      float2* __restrict__ g2) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < P;
       q += (long long)gridDim.x * blockDim.x) {
    const long long b = q / ((long long)h * w);
    const int i = (int)((q / w) % h), j = (int)(q % w);
    int a1, b1, a2, b2;
    n2n_pair(codes[q], a1, b1, a2, b2);
    const long long row = b * 2 * h;
    g1[q] = x[(row + 2 * i + a1) * 2 * w + 2 * j + b1];
    g2[q] = x[(row + 2 * i + a2) * 2 * w + 2 * j + b2];
  }
}

// Loss of Sec. 3.1 as a mean over the 2P real values of
//   d^2 + eta (d - e)^2,  d = f(g1) - g2,  e = g1(f(x)) - g2(f(x))
// (f(x) held fixed); its gradient with respect to f(g1) into gout.
__global__ void __launch_bounds__(kThreads) k_n2n_loss(const float2* __restrict__ D, const float2* __restrict__ g2,
                                                       const float2* __restrict__ fx,
                                                       const uint8_t* __restrict__ codes, int h, int w, long long P,
                                                       float eta, float scale, uint16_t* __restrict__ gout,
                                                       double* __restrict__ loss) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < P;
       q += (long long)gridDim.x * blockDim.x) {
    const long long b = q / ((long long)h * w);
    const int i = (int)((q / w) % h), j = (int)(q % w);
    int a1, b1, a2, b2;
    n2n_pair(codes[q], a1, b1, a2, b2);
    const long long row = b * 2 * h;
    const float2 f1 = fx[(row + 2 * i + a1) * 2 * w + 2 * j + b1];
    const float2 f2 = fx[(row + 2 * i + a2) * 2 * w + 2 * j + b2];
    const float2 Dv = D[q], tv = g2[q];
    const float dx = Dv.x - tv.x, dy = Dv.y - tv.y;
    const float rx = dx - (f1.x - f2.x), ry = dy - (f1.y - f2.y);
    acc += (double)dx * dx + (double)dy * dy + (double)eta * ((double)rx * rx + (double)ry * ry);
    uint4 g;
    g.x = (uint32_t)f2bf(scale * 2.f * (dx + eta * rx)) | ((uint32_t)f2bf(scale * 2.f * (dy + eta * ry)) << 16);
    g.y = 0u;
    g.z = 0u;
    g.w = 0u;
    *reinterpret_cast<uint4*>(gout + q * 8) = g;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int hh = kThreads / 2; hh > 0; hh >>= 1) {
    if ((int)threadIdx.x < hh) red[threadIdx.x] += red[threadIdx.x + hh];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * (double)scale);
}

// Adam (bias-corrected moments), FP32 master weights, refreshed BF16 copy
__global__ void k_unet_adam(long long n, float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, uint16_t* __restrict__ wbf, float b1,
                            float b2, float eps, float step, float inv_sqrt_bc2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - step * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
  w[i] = wi;
  wbf[i] = f2bf(wi);
}

__global__ void k_unet_cast(long long n, const float* __restrict__ w, uint16_t* __restrict__ wbf) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wbf[i] = f2bf(w[i]);
}

struct WTJob {
  long long w_off, wt_off;
  int cin, cp, cout, coutp, taps;
};
struct WTTable {
  WTJob j[kLayers - 1];
};

// WT[c][t][o] = W[o][t][c] (zero for o >= cout), one layer per grid row
__global__ void k_unet_wt(WTTable tab, const uint16_t* __restrict__ wbf, uint16_t* __restrict__ wt) {
  const WTJob& J = tab.j[blockIdx.y];
  const long long n = (long long)J.cin * J.taps * J.coutp;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int per = J.taps * J.coutp;
  const int c = (int)(idx / per), rem = (int)(idx - (long long)c * per);
  const int t = rem / J.coutp, o = rem - t * J.coutp;
  wt[J.wt_off + idx] = o < J.cout ? wbf[J.w_off + ((long long)o * J.taps + t) * J.cp + c] : (uint16_t)0;
}

// ------------------------------------------------------------ workspace
long long dw_part_total(int B, int H, int W);

struct UWs {
  uint16_t *x0, *e1a, *c1, *d1a, *d1b, *p1, *e2a, *c2, *d2a, *d2b, *p2, *e3a, *c3, *d3a, *d3b, *p3, *ba, *bb;
  float* out;
  uint16_t *gout, *gd1b, *gd1a, *gc1, *gd2b, *gd2a, *gc2, *gd3b, *gd3a, *gc3, *gbb, *gba, *gp3, *ge3a, *gp2,
      *ge2a, *gp1, *ge1a;
  float* dwpart;   // weight-gradient partial tiles of every layer (dw_layout)
  size_t bytes;
};

UWs unet_ws(int B, int H, int W, bool train, void* base) {
  UWs w{};
  const long long P0 = (long long)B * H * W, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
  size_t off = 0;
  char* b = static_cast<char*>(base);
  auto bf = [&](long long n) {
    off = (off + 255) & ~(size_t)255;
    uint16_t* p = b ? reinterpret_cast<uint16_t*>(b + off) : nullptr;
    off += (size_t)n * 2;
    return p;
  };
  w.x0 = bf(P0 * 8);
  w.e1a = bf(P0 * 32);
  w.c1 = bf(P0 * 64);
  w.d1a = bf(P0 * 32);
  w.d1b = bf(P0 * 32);
  w.p1 = bf(P1 * 32);
  w.e2a = bf(P1 * 64);
  w.c2 = bf(P1 * 128);
  w.d2a = bf(P1 * 64);
  w.d2b = bf(P1 * 64);
  w.p2 = bf(P2 * 64);
  w.e3a = bf(P2 * 128);
  w.c3 = bf(P2 * 256);
  w.d3a = bf(P2 * 128);
  w.d3b = bf(P2 * 128);
  w.p3 = bf(P3 * 128);
  w.ba = bf(P3 * 256);
  w.bb = bf(P3 * 256);
  w.out = reinterpret_cast<float*>(bf(P0 * 4));   // [P0][2] FP32
  if (train) {
    w.gout = bf(P0 * 8);
    w.gd1b = bf(P0 * 32);
    w.gd1a = bf(P0 * 32);
    w.gc1 = bf(P0 * 64);
    w.gd2b = bf(P1 * 64);
    w.gd2a = bf(P1 * 64);
    w.gc2 = bf(P1 * 128);
    w.gd3b = bf(P2 * 128);
    w.gd3a = bf(P2 * 128);
    w.gc3 = bf(P2 * 256);
    w.gbb = bf(P3 * 256);
    w.gba = bf(P3 * 256);
    w.gp3 = bf(P3 * 128);
    w.ge3a = bf(P2 * 128);
    w.gp2 = bf(P2 * 64);
    w.ge2a = bf(P1 * 64);
    w.gp1 = bf(P1 * 32);
    w.ge1a = bf(P0 * 32);
    w.dwpart = reinterpret_cast<float*>(bf(2 * dw_part_total(B, H, W)));
  }
  w.bytes = (off + 255) & ~(size_t)255;
  return w;
}

Act A(uint16_t* p, int cs, int co, int c) { return Act{p, cs, co, c}; }

}  // namespace

// ------------------------------------------------------------ the network
}  // namespace pnp

struct pnp_unet {
  int device;
  float* master;     // [n_params] FP32
  float* grad;       // [n_params]
  float* m;          // Adam moments
  float* v;
  uint16_t* wbf;     // [n_params] BF16 copy of master (bias entries unused)
  uint16_t* wt;      // transposed BF16 weights for the input gradients
  long long step;
};

namespace pnp {

namespace {

const LayerInfo& layer(int i) { return layout().L[i]; }

// Weight-gradient launch shape of a layer over P pixels: a 32 x 128 output
// tile where Cout <= 32, else 64 x 64 (a transposed convolution: one GEMM
// per tap, N = Cin + 1); the pixels split into a multiple of 8 slices of
// whole 128-pixel stages (slices past the end are empty and contribute
// zeros), about 512 workgroups and >= 4 stages a slice where the pixels
// allow.  (Fewer slices mean fewer partial tiles for k_dw_reduce to read:
// 10 x 128^2 training step 0.789 ms at 1024 workgroups, 0.776 at 512 and
// 384, 0.799 at 256.)
struct DWPlan {
  int tm, tn, mt, nt, taps, M, N, kchunk, splits;
  long long part_floats() const { return (long long)taps * splits * M * N; }
};
DWPlan dw_plan(const LayerInfo& l, long long P) {
  DWPlan d;
  const bool up = l.kind == kUp;
  d.tm = l.cout <= 32 ? 32 : 64;
  d.tn = 4096 / d.tm;
  d.M = l.cout;
  d.N = up ? l.cp + 1 : l.taps * l.cp + 1;
  d.taps = up ? 4 : 1;
  d.mt = (int)blocks_for(d.M, d.tm);
  d.nt = (int)blocks_for(d.N, d.tn);
  const long long tiles = (long long)d.mt * d.nt * d.taps;
  long long sp = std::max<long long>(1, std::min<long long>(P / 512, (512 + tiles - 1) / tiles));
  sp = (sp + 7) / 8 * 8;
  long long kc = (P + sp - 1) / sp;
  kc = (kc + 127) / 128 * 128;
  d.kchunk = (int)kc;
  d.splits = (int)sp;
  return d;
}

// every layer's partial tiles, one after another (256-byte aligned)
struct DWLayout {
  long long off[kLayers];
  long long total;
};
DWLayout dw_layout(int B, int H, int W) {
  DWLayout t{};
  for (int i = 0; i < kLayers; ++i) {
    t.off[i] = t.total;
    const long long P = (long long)B * (H >> kDWLevel[i]) * (W >> kDWLevel[i]);
    t.total += (dw_plan(layer(i), P).part_floats() + 63) / 64 * 64;
  }
  return t;
}
long long dw_part_total(int B, int H, int W) { return dw_layout(B, H, W).total; }

// K chunks of a forward convolution on the tiled kernels: fixed by the layer
// and the image size, never by the batch, so every image of a batch gets
// the arithmetic it gets alone.  Layers whose single-image launch has fewer
// than 256 64 x 64 tiles split K in 2 or 4 (chunks of a multiple of 3 steps).
int conv_chunks(const LayerInfo& l, int H, int W) {
  if (l.cp % 32 != 0 || l.cout % 64 != 0) return 1;
  const long long tiles = ((long long)H * W + 63) / 64 * (l.cout / 64);
  const int nsteps = l.taps * (l.cp / 32);
  int c = 1;
  while (c < 4 && tiles * c < 256 && nsteps % (6 * c) == 0) c *= 2;
  return c;
}

// `pool` (optional, pool.p == nullptr: none): the 2x2 max-pool of the output
// into that slice, fused where the halo-tile kernel runs; returns whether it
// was fused (else the caller pools).
// k_conv3_halo with its dynamic LDS (above 64 KB for 256 input channels)
template <class V, int CP, int TN, int G>
void launch_halo(dim3 grid, dim3 block, const V& v, hipStream_t s) {
  const size_t bytes = sizeof(uint16_t) * unet::Halo<CP, TN, G>::LDS;
  if (bytes > 65536)
    PNP_HIP(hipFuncSetAttribute((const void*)unet::k_conv3_halo<V, CP, TN, G>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  PNP_LAUNCH((unet::k_conv3_halo<V, CP, TN, G>), grid, block, bytes, s, v);
}

// `head` (optional): the output layer's operands, fused likewise.
struct HeadOut {
  const float2* u;
  float2* o;
  float2* dst;
};
bool launch_conv_fwd(const pnp_unet* net, int li, Act in, Act out, float* out32, Geo g, bool relu,
                     hipStream_t s, Act pool = Act{nullptr, 0, 0, 0}, const HeadOut* head = nullptr,
                     const unet::FirstIn* first = nullptr) {
  const LayerInfo& l = layer(li);
  const int chunks = conv_chunks(l, g.H, g.W);
  unet::ConvFwd v{in, net->wbf + l.w_off, net->master + l.b_off, out, out32, g, l.taps, l.cp, l.cout,
                  relu ? 1 : 0, chunks};
  const long long P = (long long)g.B * g.H * g.W;
  const int nsteps = l.taps * (l.cp / 32);     // K steps of the tiled kernels
  if (l.cp == 8 && l.taps == 9 && l.cout == 32) {  // the first layer (3 channels padded to 8)
    PNP_LAUNCH(unet::k_conv_first, dim3(blocks_for(P, 128)), dim3(256), 0, s, v,
               first ? *first : unet::FirstIn{nullptr, nullptr, 0.f, nullptr});
    return false;
  }
  // 3x3 layers with 32, 64 or 128 input channels: the halo-tile kernel, one
  // group of four waves per K chunk (bit-identical to the tiled kernel)
  if (l.taps == 9 && (l.cp == 32 || l.cp == 64 || l.cp == 128 || l.cp == 256) && l.cout % 32 == 0 &&
      out32 == nullptr && (chunks == 1 || chunks == 2 || chunks == 4)) {
    const unsigned patches = (unsigned)(g.B * ((g.H + unet::kHaloPY - 1) / unet::kHaloPY) *
                                        ((g.W + unet::kHaloPX - 1) / unet::kHaloPX));
    // 64 output channels a workgroup, unless that leaves fewer than 256
    // workgroups (single small images: 32, bit-identical; 320^2 forward at
    // batch 1 161.8 -> 159.3 us)
    const bool wide = l.cout % 64 == 0 && chunks <= 2 && (long long)patches * (l.cout / 64) >= 256;
    const dim3 grid(patches, l.cout / (wide ? 64 : 32)), block(256 * chunks);
#define PNP_HALO(CPV, TNV, GV)                                                           \
  if (l.cp == CPV && (wide ? 64 : 32) == TNV && chunks == GV) {                          \
    v.pool = g.H % 2 == 0 && g.W % 2 == 0 ? pool : Act{nullptr, 0, 0, 0};               \
    if (head && TNV == 32 && l.cout == 32) {                                             \
      const LayerInfo& lh = layer(kLayers - 1);                                          \
      v.head_w = net->wbf + lh.w_off;                                                    \
      v.head_b = net->master + lh.b_off;                                                 \
      v.head_u = head->u;                                                                \
      v.head_o = head->o;                                                                \
      v.head_dst = head->dst;                                                            \
    }                                                                                    \
    launch_halo<unet::ConvFwd, CPV, TNV, GV>(grid, block, v, s);                         \
    return head ? v.head_w != nullptr : v.pool.p != nullptr;                             \
  }
    PNP_HALO(32, 32, 1) PNP_HALO(32, 64, 1) PNP_HALO(64, 32, 1) PNP_HALO(64, 64, 1)
    PNP_HALO(128, 32, 1) PNP_HALO(128, 64, 1)
    PNP_HALO(64, 32, 2) PNP_HALO(64, 64, 2) PNP_HALO(128, 32, 2) PNP_HALO(128, 64, 2) PNP_HALO(128, 32, 4)
    PNP_HALO(256, 32, 1) PNP_HALO(256, 64, 1) PNP_HALO(256, 32, 2) PNP_HALO(256, 64, 2) PNP_HALO(256, 32, 4)
#undef PNP_HALO
  }
  // larger tiles where the input channels come in 32-wide chunks and the
  // launch still has a workgroup per compute unit (K chunks in sequence);
  // else 64 x 64 tiles with one wave group per K chunk and a deeper load
  // pipeline; the generic kernel for the rest (3-channel input, 1 x 1
  // output), whose layers have a single chunk
  if (l.cp % 32 == 0 && l.cout == 32 && P / 256 >= 512) {
    PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 256, 32, 4, 1, 1, false>), dim3(blocks_for(P, 256), 1, 1), dim3(256), 0, s, v);
  } else if (l.cp % 32 == 0 && l.cout == 32 && P / 128 >= 256) {
    PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 128, 32, 4, 1, 1, false>), dim3(blocks_for(P, 128), 1, 1), dim3(256), 0, s, v);
  } else if (l.cp % 32 == 0 && l.cout % 64 == 0 && (P / 128) * (l.cout / 64) >= 256) {
    const dim3 grid(blocks_for(P, 128), l.cout / 64, 1);
    if (chunks > 1)
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 128, 64, 2, 1, 1, true>), grid, dim3(256), 0, s, v);
    else
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 128, 64, 2, 1, 1, false>), grid, dim3(256), 0, s, v);
  } else if (l.cp % 32 == 0 && l.cout % 64 == 0 && (nsteps / chunks) % 3 == 0) {
    const dim3 grid(blocks_for(P, 64), l.cout / 64, 1);
    if (chunks == 4)
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 64, 64, 2, 3, 4, true>), grid, dim3(1024), 0, s, v);
    else if (chunks == 2)
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 64, 64, 2, 3, 2, true>), grid, dim3(512), 0, s, v);
    else
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvFwd, 64, 64, 2, 3, 1, false>), grid, dim3(256), 0, s, v);
  } else {
    if (chunks != 1) fail(PNP_ERR_UNSUPPORTED, "layer %d: K chunks on the generic convolution kernel", li);
    PNP_LAUNCH(unet::k_mfma_gemm<unet::ConvFwd>, dim3(blocks_for(P, 64), blocks_for(l.cout, 64), 1), dim3(256),
               0, s, v);
  }
  return false;
}

void launch_up_fwd(const pnp_unet* net, int li, Act in, Act out, Geo g, hipStream_t s) {
  const LayerInfo& l = layer(li);
  unet::UpFwd v{in, net->wbf + l.w_off, net->master + l.b_off, out, g, l.cin, l.cout, 1, l.cin, 1};
  const long long P = (long long)g.B * g.H * g.W;
  // the tiled kernels (K = Cin in 32-wide steps) where the channels allow,
  // one grid slice per output sub-pixel
  if (l.cin % 64 == 0 && l.cout % 64 == 0) {
    PNP_LAUNCH((unet::k_gemm_tiled<unet::UpFwd, 64, 64, 2, 2, 1, false>), dim3(blocks_for(P, 64), l.cout / 64, 4),
               dim3(256), 0, s, v);
  } else if (l.cin % 32 == 0 && l.cout == 32) {
    PNP_LAUNCH((unet::k_gemm_tiled<unet::UpFwd, 128, 32, 4, 1, 1, false>), dim3(blocks_for(P, 128), 1, 4),
               dim3(256), 0, s, v);
  } else {
    PNP_LAUNCH(unet::k_mfma_gemm<unet::UpFwd>, dim3(blocks_for(P, 64), blocks_for(l.cout, 64), 4), dim3(256), 0,
               s, v);
  }
}

void launch_pool(Act in, Act out, Geo go, int C, hipStream_t s) {
  const long long n = (long long)go.B * go.H * go.W * (C / 8);
  PNP_LAUNCH(k_unet_pool, dim3(blocks_for(n)), dim3(kThreads), 0, s, in, out, go, C);
}

void launch_pool_bwd(Act fin, Act gout, Act gin, Geo go, int C, hipStream_t s) {
  const long long n = (long long)go.B * go.H * go.W * C;
  PNP_LAUNCH(k_unet_pool_bwd, dim3(blocks_for(n)), dim3(kThreads), 0, s, fin, gout, gin, go, C);
}

// Partial weight-gradient tiles of layer li (dz: output gradient, in: the
// layer input, g: the pixel space of the sum) into its part of dwpart
void launch_dw(int li, Act dz, Act in, Geo g, float* dwpart, hipStream_t s) {
  const LayerInfo& l = layer(li);
  const long long P = (long long)g.B * g.H * g.W;
  const DWPlan d = dw_plan(l, P);
  const DWLayout lay = dw_layout(g.B, g.H << kDWLevel[li], g.W << kDWLevel[li]);
  const bool up = l.kind == kUp;
  unet::DWArgs a{dz.p + dz.co, in.p + in.co, dwpart + lay.off[li], dz.cs, in.cs, g.H, g.W, (int)P,
                 up ? 1 : l.taps, l.cp, d.M, d.N, up ? 1 : 0, d.kchunk, 128 % g.W, (128 / g.W) % g.H,
                 d.mt, d.mt * d.nt, d.mt * d.nt * d.taps, d.splits};
  const dim3 grid((unsigned)(d.mt * d.nt * d.taps * d.splits));
  const bool al = g.W % 8 == 0;
  if (d.tm == 32 && al) PNP_LAUNCH((unet::k_dw_gemm<32, 128, true>), grid, dim3(256), 0, s, a);
  if (d.tm == 32 && !al) PNP_LAUNCH((unet::k_dw_gemm<32, 128, false>), grid, dim3(256), 0, s, a);
  if (d.tm == 64 && al) PNP_LAUNCH((unet::k_dw_gemm<64, 64, true>), grid, dim3(256), 0, s, a);
  if (d.tm == 64 && !al) PNP_LAUNCH((unet::k_dw_gemm<64, 64, false>), grid, dim3(256), 0, s, a);
}

// Every layer's dW and db from its partial tiles (each gradient entry is
// written: the gradient buffer needs no clearing)
void launch_dw_reduce(pnp_unet* net, int B, int H, int W, const float* dwpart, hipStream_t s) {
  const DWLayout lay = dw_layout(B, H, W);
  unet::DWJobs jobs{};
  unsigned blocks = 0;
  for (int i = 0; i < kLayers; ++i) {
    const LayerInfo& l = layer(i);
    const long long P = (long long)B * (H >> kDWLevel[i]) * (W >> kDWLevel[i]);
    const DWPlan d = dw_plan(l, P);
    const bool up = l.kind == kUp;
    // slice groups: at most 8 slices a thread where 16 groups allow
    int G = 1;
    while (G < 16 && d.splits > 8 * G) G *= 2;
    const long long entries = (long long)d.M * (up ? 4 * l.cp + 1 : d.N);
    unet::DWJob& J = jobs.j[jobs.n++];
    J = unet::DWJob{dwpart + lay.off[i], net->grad + l.w_off, net->grad + l.b_off, d.splits, d.M, d.N,
                    up ? 1 : 0, l.cp, G, blocks};
    blocks += (unsigned)((entries + 256 / G - 1) / (256 / G));
  }
  PNP_LAUNCH(unet::k_dw_reduce, dim3(blocks), dim3(256), 0, s, jobs);
}

void launch_conv_dx(const pnp_unet* net, int li, Act dz, Act dx, Mask mask, Geo g, hipStream_t s) {
  const LayerInfo& l = layer(li);
  const long long P = (long long)g.B * g.H * g.W;
  // 3x3 layers whose output gradient has 32, 64 or 128 channels: the
  // halo-tile kernel (mirrored taps; bit-identical to the tiled kernel)
  if (l.taps == 9 && (l.coutp == 32 || l.coutp == 64 || l.coutp == 128 || l.coutp == 256) && l.cin % 32 == 0) {
    unet::ConvDXT v{dz, net->wt + l.wt_off, dx, mask, g, l.taps, l.coutp, l.cin, 1};
    const unsigned patches = (unsigned)(g.B * ((g.H + unet::kHaloPY - 1) / unet::kHaloPY) *
                                        ((g.W + unet::kHaloPX - 1) / unet::kHaloPX));
    const bool wide = l.cin % 64 == 0;
    const dim3 grid(patches, l.cin / (wide ? 64 : 32));
#define PNP_HALO_DX(CPV, TNV)                                                            \
  if (l.coutp == CPV && (wide ? 64 : 32) == TNV) {                                       \
    launch_halo<unet::ConvDXT, CPV, TNV, 1>(grid, dim3(256), v, s);                      \
    return;                                                                              \
  }
    PNP_HALO_DX(32, 32) PNP_HALO_DX(32, 64) PNP_HALO_DX(64, 32) PNP_HALO_DX(64, 64) PNP_HALO_DX(128, 32)
    PNP_HALO_DX(128, 64) PNP_HALO_DX(256, 32) PNP_HALO_DX(256, 64)
#undef PNP_HALO_DX
  }
  // the tiled kernels where the output-gradient channels come in 32-wide
  // chunks (every layer but the 2-channel output); the generic kernel else
  if (l.coutp % 32 == 0 && (l.taps * (l.coutp / 32)) % 3 == 0 && (l.cin == 32 || l.cin % 64 == 0)) {
    unet::ConvDXT v{dz, net->wt + l.wt_off, dx, mask, g, l.taps, l.coutp, l.cin, 1};
    if (l.cin == 32 && P / 256 >= 512)
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvDXT, 256, 32, 4, 1, 1, false>), dim3(blocks_for(P, 256), 1, 1),
                 dim3(256), 0, s, v);
    else if (l.cin == 32)
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvDXT, 128, 32, 4, 1, 1, false>), dim3(blocks_for(P, 128), 1, 1),
                 dim3(256), 0, s, v);
    else if ((P / 128) * (l.cin / 64) >= 256)
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvDXT, 128, 64, 2, 1, 1, false>),
                 dim3(blocks_for(P, 128), l.cin / 64, 1), dim3(256), 0, s, v);
    else
      PNP_LAUNCH((unet::k_gemm_tiled<unet::ConvDXT, 64, 64, 2, 3, 1, false>), dim3(blocks_for(P, 64), l.cin / 64, 1),
                 dim3(256), 0, s, v);
    return;
  }
  unet::ConvDX v{dz, net->wt + l.wt_off, dx, mask, g, l.taps, l.coutp, l.cin};
  PNP_LAUNCH(unet::k_mfma_gemm<unet::ConvDX>, dim3(blocks_for(P, 64), blocks_for(l.cin, 64), 1), dim3(256), 0,
             s, v);
}

void launch_up_dx(const pnp_unet* net, int li, Act dout, Act dx, Mask mask, Geo g, hipStream_t s) {
  const LayerInfo& l = layer(li);
  unet::UpDX v{dout, net->wt + l.wt_off, dx, mask, g, l.cin, l.cout};
  const long long P = (long long)g.B * g.H * g.W;
  PNP_LAUNCH(unet::k_mfma_gemm<unet::UpDX>, dim3(blocks_for(P, 64), blocks_for(l.cin, 64), 1), dim3(256), 0, s,
             v);
}

Mask relu_mask(const uint16_t* p, int cs, int co, int mc) { return Mask{p, cs, co, mc}; }
constexpr Mask kNoMask{nullptr, 0, 0, 0};

void check_dims(int B, int H, int W) {
  if (B < 1 || H < 8 || W < 8 || H % 8 || W % 8)
    fail(PNP_ERR_SHAPE, "UNet input %dx%dx%d: batch >= 1 and sides divisible by 8 (>= 8) required", B, H, W);
  if ((long long)B * H * W > (1LL << 31) / 64)
    fail(PNP_ERR_SHAPE, "UNet input %dx%dx%d too large", B, H, W);
}

void refresh_weights(pnp_unet* net, hipStream_t s) {
  const NetLayout& lay = layout();
  WTTable tab{};
  long long maxn = 0;
  for (int i = 1; i < kLayers; ++i) {
    const LayerInfo& l = lay.L[i];
    tab.j[i - 1] = WTJob{l.w_off, l.wt_off, l.cin, l.cp, l.cout, l.coutp, l.taps};
    maxn = std::max(maxn, (long long)l.cin * l.taps * l.coutp);
  }
  PNP_LAUNCH(k_unet_wt, dim3(blocks_for(maxn), kLayers - 1), dim3(kThreads), 0, s, tab, net->wbf, net->wt);
}

}  // namespace

long long unet_param_count() { return layout().n_params; }
long long unet_real_param_count() { return layout().n_real; }
int unet_layer_count() { return kLayers; }
void unet_layer_info(int i, pnp_unet_layer* out) {
  if (i < 0 || i >= kLayers) fail(PNP_ERR_ARG, "layer index %d out of range", i);
  const LayerInfo& l = layer(i);
  out->kind = l.kind;
  out->cin = l.cin;
  out->cin_padded = l.cp;
  out->cout = l.cout;
  out->taps = l.taps;
  out->w_offset = l.w_off;
  out->b_offset = l.b_off;
}

size_t unet_ws_bytes(int B, int H, int W, bool train) {
  check_dims(B, H, W);
  return unet_ws(B, H, W, train, nullptr).bytes;
}

pnp_unet* unet_create(const float* params, hipStream_t s) {
  const NetLayout& lay = layout();
  pnp_unet* net = new pnp_unet{};
  hipError_t e = hipGetDevice(&net->device);
  const size_t nb = (size_t)lay.n_params;
  void* blk = nullptr;
  const size_t bytes = nb * 4 * 4 + nb * 2 + (size_t)lay.n_wt * 2 + 1024;
  if (e == hipSuccess) e = hipMalloc(&blk, bytes);
  if (e != hipSuccess) {
    delete net;
    fail_hip(e, "hipMalloc(UNet parameters)", __FILE__, __LINE__);
  }
  char* b = static_cast<char*>(blk);
  auto take = [&](size_t n) {
    char* p = b;
    b += (n + 255) & ~(size_t)255;
    return p;
  };
  net->master = reinterpret_cast<float*>(take(nb * 4));
  net->grad = reinterpret_cast<float*>(take(nb * 4));
  net->m = reinterpret_cast<float*>(take(nb * 4));
  net->v = reinterpret_cast<float*>(take(nb * 4));
  net->wbf = reinterpret_cast<uint16_t*>(take(nb * 2));
  net->wt = reinterpret_cast<uint16_t*>(take((size_t)lay.n_wt * 2));
  try {
    PNP_HIP(hipMemcpyAsync(net->master, params, nb * 4, hipMemcpyDeviceToDevice, s));
    // gradient and Adam moments start at zero (each buffer on its own: the
    // 256-byte alignment of the blocks leaves gaps between them)
    PNP_HIP(hipMemsetAsync(net->grad, 0, nb * 4, s));
    PNP_HIP(hipMemsetAsync(net->m, 0, nb * 4, s));
    PNP_HIP(hipMemsetAsync(net->v, 0, nb * 4, s));
    PNP_LAUNCH(k_unet_cast, dim3(blocks_for(lay.n_params)), dim3(kThreads), 0, s, lay.n_params, net->master,
               net->wbf);
    refresh_weights(net, s);
  } catch (...) {
    (void)hipFree(net->master);
    delete net;
    throw;
  }
  return net;
}

void unet_destroy(pnp_unet* net) {
  if (!net) return;
  (void)hipFree(net->master);
  delete net;
}

float* unet_buffer(pnp_unet* net, int which) {
  switch (which) {
    case PNP_UNET_PARAMS: return net->master;
    case PNP_UNET_GRAD: return net->grad;
    case PNP_UNET_ADAM_M: return net->m;
    case PNP_UNET_ADAM_V: return net->v;
    default: fail(PNP_ERR_ARG, "unknown UNet buffer %d", which);
  }
}

void unet_set(pnp_unet* net, int which, const float* src, hipStream_t s) {
  const long long n = layout().n_params;
  float* dst = unet_buffer(net, which);
  PNP_HIP(hipMemcpyAsync(dst, src, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  if (which == PNP_UNET_PARAMS) {
    PNP_LAUNCH(k_unet_cast, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, net->master, net->wbf);
    refresh_weights(net, s);
  }
}

void unet_get(pnp_unet* net, int which, float* dst, hipStream_t s) {
  const long long n = layout().n_params;
  PNP_HIP(hipMemcpyAsync(dst, unet_buffer(net, which), (size_t)n * 4, hipMemcpyDeviceToDevice, s));
}

long long& unet_step(pnp_unet* net) { return net->step; }

void unet_forward(const pnp_unet* net, const float2* u, const float* sigma, float sigma_c, int B, int H, int W,
                  float2* out, void* ws, hipStream_t s) {
  check_dims(B, H, W);
  const UWs w = unet_ws(B, H, W, false, ws);
  const Geo g0{B, H, W}, g1{B, H / 2, W / 2}, g2{B, H / 4, W / 4}, g3{B, H / 8, W / 8};
  const long long P0 = (long long)B * H * W;
  // encoder.  A few images: the first layer forms its packed input from u and
  // sigma itself (one launch less: 167 -> 164 us at 1 x 320^2); many: the
  // packing pass first, which converts each pixel once instead of once per
  // tap (1.60 against 1.58 ms at 24 x 320^2).  x0 holds the packed input
  // either way.
  if (B <= 4) {
    const unet::FirstIn first{u, sigma, sigma_c, w.x0};
    launch_conv_fwd(net, 0, A(w.x0, 8, 0, 8), A(w.e1a, 32, 0, 32), nullptr, g0, true, s, Act{nullptr, 0, 0, 0},
                    nullptr, &first);
  } else {
    PNP_LAUNCH(k_unet_pack, dim3(blocks_for((long long)H * W), B), dim3(kThreads), 0, s, u, sigma, sigma_c,
               (long long)H * W, w.x0);
    launch_conv_fwd(net, 0, A(w.x0, 8, 0, 8), A(w.e1a, 32, 0, 32), nullptr, g0, true, s);
  }
  if (!launch_conv_fwd(net, 1, A(w.e1a, 32, 0, 32), A(w.c1, 64, 0, 32), nullptr, g0, true, s, A(w.p1, 32, 0, 32)))
    launch_pool(A(w.c1, 64, 0, 32), A(w.p1, 32, 0, 32), g1, 32, s);
  launch_conv_fwd(net, 2, A(w.p1, 32, 0, 32), A(w.e2a, 64, 0, 64), nullptr, g1, true, s);
  if (!launch_conv_fwd(net, 3, A(w.e2a, 64, 0, 64), A(w.c2, 128, 0, 64), nullptr, g1, true, s, A(w.p2, 64, 0, 64)))
    launch_pool(A(w.c2, 128, 0, 64), A(w.p2, 64, 0, 64), g2, 64, s);
  launch_conv_fwd(net, 4, A(w.p2, 64, 0, 64), A(w.e3a, 128, 0, 128), nullptr, g2, true, s);
  if (!launch_conv_fwd(net, 5, A(w.e3a, 128, 0, 128), A(w.c3, 256, 0, 128), nullptr, g2, true, s,
                       A(w.p3, 128, 0, 128)))
    launch_pool(A(w.c3, 256, 0, 128), A(w.p3, 128, 0, 128), g3, 128, s);
  launch_conv_fwd(net, 6, A(w.p3, 128, 0, 128), A(w.ba, 256, 0, 256), nullptr, g3, true, s);
  launch_conv_fwd(net, 7, A(w.ba, 256, 0, 256), A(w.bb, 256, 0, 256), nullptr, g3, true, s);
  // decoder
  launch_up_fwd(net, 8, A(w.bb, 256, 0, 256), A(w.c3, 256, 128, 128), g3, s);
  launch_conv_fwd(net, 9, A(w.c3, 256, 0, 256), A(w.d3a, 128, 0, 128), nullptr, g2, true, s);
  launch_conv_fwd(net, 10, A(w.d3a, 128, 0, 128), A(w.d3b, 128, 0, 128), nullptr, g2, true, s);
  launch_up_fwd(net, 11, A(w.d3b, 128, 0, 128), A(w.c2, 128, 64, 64), g2, s);
  launch_conv_fwd(net, 12, A(w.c2, 128, 0, 128), A(w.d2a, 64, 0, 64), nullptr, g1, true, s);
  launch_conv_fwd(net, 13, A(w.d2a, 64, 0, 64), A(w.d2b, 64, 0, 64), nullptr, g1, true, s);
  launch_up_fwd(net, 14, A(w.d2b, 64, 0, 64), A(w.c1, 64, 32, 32), g1, s);
  launch_conv_fwd(net, 15, A(w.c1, 64, 0, 64), A(w.d1a, 32, 0, 32), nullptr, g0, true, s);
  const HeadOut head{u, reinterpret_cast<float2*>(w.out), out};
  if (!launch_conv_fwd(net, 16, A(w.d1a, 32, 0, 32), A(w.d1b, 32, 0, 32), nullptr, g0, true, s,
                       Act{nullptr, 0, 0, 0}, &head)) {
    const LayerInfo& l = layer(17);
    PNP_LAUNCH(k_unet_head, dim3(blocks_for(P0)), dim3(kThreads), 0, s, w.d1b, net->wbf + l.w_off,
               net->master + l.b_off, u, P0, reinterpret_cast<float2*>(w.out), out);
  }
}

// Parameter gradients from the output gradient w.gout of a train-sized
// workspace holding the activations of the preceding forward pass.
static void unet_backprop(pnp_unet* net, const UWs& w, int B, int H, int W, hipStream_t s) {
  const Geo g0{B, H, W}, g1{B, H / 2, W / 2}, g2{B, H / 4, W / 4}, g3{B, H / 8, W / 8};
  // output layer and the last decoder stage
  launch_dw(17, A(w.gout, 8, 0, 2), A(w.d1b, 32, 0, 32), g0, w.dwpart, s);
  launch_conv_dx(net, 17, A(w.gout, 8, 0, 8), A(w.gd1b, 32, 0, 32), relu_mask(w.d1b, 32, 0, 32), g0, s);
  launch_dw(16, A(w.gd1b, 32, 0, 32), A(w.d1a, 32, 0, 32), g0, w.dwpart, s);
  launch_conv_dx(net, 16, A(w.gd1b, 32, 0, 32), A(w.gd1a, 32, 0, 32), relu_mask(w.d1a, 32, 0, 32), g0, s);
  launch_dw(15, A(w.gd1a, 32, 0, 32), A(w.c1, 64, 0, 64), g0, w.dwpart, s);
  launch_conv_dx(net, 15, A(w.gd1a, 32, 0, 32), A(w.gc1, 64, 0, 64), relu_mask(w.c1, 64, 0, 32), g0, s);
  launch_dw(14, A(w.gc1, 64, 32, 32), A(w.d2b, 64, 0, 64), g1, w.dwpart, s);
  launch_up_dx(net, 14, A(w.gc1, 64, 32, 32), A(w.gd2b, 64, 0, 64), relu_mask(w.d2b, 64, 0, 64), g1, s);
  launch_dw(13, A(w.gd2b, 64, 0, 64), A(w.d2a, 64, 0, 64), g1, w.dwpart, s);
  launch_conv_dx(net, 13, A(w.gd2b, 64, 0, 64), A(w.gd2a, 64, 0, 64), relu_mask(w.d2a, 64, 0, 64), g1, s);
  launch_dw(12, A(w.gd2a, 64, 0, 64), A(w.c2, 128, 0, 128), g1, w.dwpart, s);
  launch_conv_dx(net, 12, A(w.gd2a, 64, 0, 64), A(w.gc2, 128, 0, 128), relu_mask(w.c2, 128, 0, 64), g1, s);
  launch_dw(11, A(w.gc2, 128, 64, 64), A(w.d3b, 128, 0, 128), g2, w.dwpart, s);
  launch_up_dx(net, 11, A(w.gc2, 128, 64, 64), A(w.gd3b, 128, 0, 128), relu_mask(w.d3b, 128, 0, 128), g2, s);
  launch_dw(10, A(w.gd3b, 128, 0, 128), A(w.d3a, 128, 0, 128), g2, w.dwpart, s);
  launch_conv_dx(net, 10, A(w.gd3b, 128, 0, 128), A(w.gd3a, 128, 0, 128), relu_mask(w.d3a, 128, 0, 128), g2, s);
  launch_dw(9, A(w.gd3a, 128, 0, 128), A(w.c3, 256, 0, 256), g2, w.dwpart, s);
  launch_conv_dx(net, 9, A(w.gd3a, 128, 0, 128), A(w.gc3, 256, 0, 256), relu_mask(w.c3, 256, 0, 128), g2, s);
  launch_dw(8, A(w.gc3, 256, 128, 128), A(w.bb, 256, 0, 256), g3, w.dwpart, s);
  launch_up_dx(net, 8, A(w.gc3, 256, 128, 128), A(w.gbb, 256, 0, 256), relu_mask(w.bb, 256, 0, 256), g3, s);
  // bottleneck
  launch_dw(7, A(w.gbb, 256, 0, 256), A(w.ba, 256, 0, 256), g3, w.dwpart, s);
  launch_conv_dx(net, 7, A(w.gbb, 256, 0, 256), A(w.gba, 256, 0, 256), relu_mask(w.ba, 256, 0, 256), g3, s);
  launch_dw(6, A(w.gba, 256, 0, 256), A(w.p3, 128, 0, 128), g3, w.dwpart, s);
  launch_conv_dx(net, 6, A(w.gba, 256, 0, 256), A(w.gp3, 128, 0, 128), kNoMask, g3, s);
  // encoder (skip gradients already hold the decoder's share)
  launch_pool_bwd(A(w.c3, 256, 0, 128), A(w.gp3, 128, 0, 128), A(w.gc3, 256, 0, 128), g3, 128, s);
  launch_dw(5, A(w.gc3, 256, 0, 128), A(w.e3a, 128, 0, 128), g2, w.dwpart, s);
  launch_conv_dx(net, 5, A(w.gc3, 256, 0, 128), A(w.ge3a, 128, 0, 128), relu_mask(w.e3a, 128, 0, 128), g2, s);
  launch_dw(4, A(w.ge3a, 128, 0, 128), A(w.p2, 64, 0, 64), g2, w.dwpart, s);
  launch_conv_dx(net, 4, A(w.ge3a, 128, 0, 128), A(w.gp2, 64, 0, 64), kNoMask, g2, s);
  launch_pool_bwd(A(w.c2, 128, 0, 64), A(w.gp2, 64, 0, 64), A(w.gc2, 128, 0, 64), g2, 64, s);
  launch_dw(3, A(w.gc2, 128, 0, 64), A(w.e2a, 64, 0, 64), g1, w.dwpart, s);
  launch_conv_dx(net, 3, A(w.gc2, 128, 0, 64), A(w.ge2a, 64, 0, 64), relu_mask(w.e2a, 64, 0, 64), g1, s);
  launch_dw(2, A(w.ge2a, 64, 0, 64), A(w.p1, 32, 0, 32), g1, w.dwpart, s);
  launch_conv_dx(net, 2, A(w.ge2a, 64, 0, 64), A(w.gp1, 32, 0, 32), kNoMask, g1, s);
  launch_pool_bwd(A(w.c1, 64, 0, 32), A(w.gp1, 32, 0, 32), A(w.gc1, 64, 0, 32), g1, 32, s);
  launch_dw(1, A(w.gc1, 64, 0, 32), A(w.e1a, 32, 0, 32), g0, w.dwpart, s);
  launch_conv_dx(net, 1, A(w.gc1, 64, 0, 32), A(w.ge1a, 32, 0, 32), relu_mask(w.e1a, 32, 0, 32), g0, s);
  launch_dw(0, A(w.ge1a, 32, 0, 32), A(w.x0, 8, 0, 8), g0, w.dwpart, s);
  launch_dw_reduce(net, B, H, W, w.dwpart, s);
}

void unet_backward(pnp_unet* net, const float2* u, const float2* target, int B, int H, int W, double* loss,
                   void* ws, hipStream_t s) {
  check_dims(B, H, W);
  const UWs w = unet_ws(B, H, W, true, ws);
  const long long P0 = (long long)B * H * W;
  PNP_HIP(hipMemsetAsync(loss, 0, sizeof(double), s));
  {
    const unsigned nb = std::min<unsigned>(blocks_for(P0), 1024);
    PNP_LAUNCH(k_unet_l1, dim3(nb), dim3(kThreads), 0, s, u, reinterpret_cast<const float2*>(w.out), target, P0,
               (float)(0.5 / (double)P0), w.gout, loss);
  }
  unet_backprop(net, w, B, H, W, s);
}

// ---- Neighbor2Neighbor training (Sec. 3.1): sub-samplers and loss
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t unet_n2n_ws_bytes(int B, int H, int W) {
  if (H % 16 || W % 16) fail(PNP_ERR_SHAPE, "Neighbor2Neighbor needs H and W divisible by 16 (%d x %d)", H, W);
  const long long P = (long long)B * H * W, p = P / 4;
  return al256(unet_ws_bytes(B, H, W, false)) + al256(unet_ws_bytes(B, H / 2, W / 2, true)) +
         al256(sizeof(float2) * P) + 3 * al256(sizeof(float2) * p);
}

void unet_n2n_backward(pnp_unet* net, const float2* x, const uint8_t* codes, double eta, int B, int H, int W,
                       double* loss, void* ws, hipStream_t s) {
  const int h = H / 2, wd = W / 2;
  const long long P = (long long)B * H * W, p = P / 4;
  char* c = (char*)ws;
  void* ws_full = c;
  c += al256(unet_ws_bytes(B, H, W, false));
  void* ws_sub = c;
  c += al256(unet_ws_bytes(B, h, wd, true));
  float2* fx = (float2*)c;
  c += al256(sizeof(float2) * P);
  float2* g1 = (float2*)c;
  c += al256(sizeof(float2) * p);
  float2* g2 = (float2*)c;
  c += al256(sizeof(float2) * p);
  float2* dsub = (float2*)c;
  const unsigned nb = std::min<unsigned>(blocks_for(p), 1024);
  PNP_LAUNCH(k_n2n_sub, dim3(nb), dim3(kThreads), 0, s, x, codes, h, wd, p, g1, g2);
  unet_forward(net, x, nullptr, 0.f, B, H, W, fx, ws_full, s);        // f(x), no gradient
  unet_forward(net, g1, nullptr, 0.f, B, h, wd, dsub, ws_sub, s);    // f(g1(x)), activations kept
  const UWs w = unet_ws(B, h, wd, true, ws_sub);
  PNP_HIP(hipMemsetAsync(loss, 0, sizeof(double), s));
  PNP_LAUNCH(k_n2n_loss, dim3(nb), dim3(kThreads), 0, s, dsub, g2, fx, codes, h, wd, p, (float)eta,
             (float)(0.5 / (double)p), w.gout, loss);
  unet_backprop(net, w, B, h, wd, s);
}

void unet_adam(pnp_unet* net, double lr, double b1, double b2, double eps, hipStream_t s) {
  const long long n = layout().n_params;
  net->step += 1;
  const double bc1 = 1.0 - std::pow(b1, (double)net->step);
  const double bc2 = 1.0 - std::pow(b2, (double)net->step);
  PNP_LAUNCH(k_unet_adam, dim3(blocks_for(n)), dim3(kThreads), 0, s, n, net->master, net->grad, net->m, net->v,
             net->wbf, (float)b1, (float)b2, (float)eps, (float)(lr / bc1), (float)(1.0 / std::sqrt(bc2)));
  refresh_weights(net, s);
}

// Device pointer and layout of a named activation of the workspace
// (0..18 forward tensors, 19.. gradients), for inspection.
void unet_tensor(int B, int H, int W, bool train, void* ws, int id, void** ptr, int32_t dims[4]) {
  check_dims(B, H, W);
  const UWs w = unet_ws(B, H, W, train, ws);
  struct T {
    void* p;
    int div, cs;
  };
  const T t[] = {{w.x0, 1, 8},    {w.e1a, 1, 32},  {w.c1, 1, 64},   {w.d1a, 1, 32},  {w.d1b, 1, 32},
                 {w.p1, 2, 32},   {w.e2a, 2, 64},  {w.c2, 2, 128},  {w.d2a, 2, 64},  {w.d2b, 2, 64},
                 {w.p2, 4, 64},   {w.e3a, 4, 128}, {w.c3, 4, 256},  {w.d3a, 4, 128}, {w.d3b, 4, 128},
                 {w.p3, 8, 128},  {w.ba, 8, 256},  {w.bb, 8, 256},  {w.out, 1, 2},
                 {w.gout, 1, 8},  {w.gd1b, 1, 32}, {w.gd1a, 1, 32}, {w.gc1, 1, 64},  {w.gd2b, 2, 64},
                 {w.gd2a, 2, 64}, {w.gc2, 2, 128}, {w.gd3b, 4, 128}, {w.gd3a, 4, 128}, {w.gc3, 4, 256},
                 {w.gbb, 8, 256}, {w.gba, 8, 256}, {w.gp3, 8, 128}, {w.ge3a, 4, 128}, {w.gp2, 4, 64},
                 {w.ge2a, 2, 64}, {w.gp1, 2, 32}, {w.ge1a, 1, 32}};
  const int n = (int)(sizeof(t) / sizeof(t[0]));
  if (id < 0 || id >= n || (!train && id > 18)) fail(PNP_ERR_ARG, "UNet tensor id %d out of range", id);
  *ptr = t[id].p;
  dims[0] = B;
  dims[1] = H / t[id].div;
  dims[2] = W / t[id].div;
  dims[3] = t[id].cs;
}

}  // namespace pnp
