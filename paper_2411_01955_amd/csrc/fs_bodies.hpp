// Register four-step FFT pass bodies (K = K1*K2, fft_reg.hpp) shared by the
// 2D and 3D operators and the batched kernels: the row passes (pre /
// zero-pad / FFT along x, and inverse FFT / crop / coil sum) and the column
// passes along a strided axis.  Pixel r = i - n/2 of an image axis sits at
// grid index r mod K; grid index j is frequency j (mod K).
#pragma once

#include "cg_scalars.hpp"
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

// Zero padding of the 2x-oversampled transforms (HALF: image side n = K/2).
// K1 and K2 are multiples of 4, so with Q = K1/4 a grid index j = n1*K2 + t
// (t < K2) is padding exactly for Q <= n1 < 3Q, holds image index
// (n1 + Q)*K2 + t for n1 < Q and (n1 - 3Q)*K2 + t for n1 >= 3Q; likewise
// j = t + K1*k2 (t < K1) with P = K2/4: padding for P <= k2 < 3P, image
// index t + K1*(k2 + P) or t + K1*(k2 - 3P).  The patterns are known at
// compile time: no per-element index tests.  Without HALF (a transform of
// a full grid-sized array) img_of_grid decides at run time.
//
// Addresses are a workgroup-uniform base plus a per-thread byte offset of
// type OFF (32-bit where every offset of the launch fits, 64-bit else).
template <typename OFF, typename T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, OFF byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename OFF, typename T>
__device__ __forceinline__ void st_off(T* __restrict__ base, OFF byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Buffer accesses at a workgroup-uniform base: the byte offset is the
// thread's own part (a register) plus a workgroup-uniform part (a scalar
// register), so an access needs no per-thread address arithmetic.  Raw
// untyped buffer of 2^31 - 1 bytes (32-bit format word).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ float buf_ld1(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float2 v) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}

// Image input of the forward row pass: the image x, or -- inside CG -- the
// next residual r' = r - alpha (w + beta s) formed on the fly from the
// previous CG vectors (alpha, beta read from the device scalars); the
// workgroups of coil group 0 also store r', s' = w + beta s, p' = r + beta p
// and u' = u + alpha p'.
struct ImgIn {
  const float2* x;
  CGUpdate cg;   // cg.r == nullptr: plain image input
};

// Sum of one double over a workgroup of NT threads (NT < 64: one partial
// wave, shuffles of that width); a fixed order, so deterministic.  Every
// thread receives the sum.  sh: NT / 64 doubles of LDS.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* sh) {
  if constexpr (NT < 64) {
#pragma unroll
    for (int o = NT / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, NT);
    return v;
  } else {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += sh[w];
    return t;
  }
}

struct ImgScal {
  float alpha, beta;
};
// (called by every thread of the workgroup, outside any branch)
__device__ __forceinline__ ImgScal img_scal(const ImgIn& in) {
  if (!in.cg.r) return ImgScal{0.f, 0.f};
  if (in.cg.fin.parts) {
    const CgStep st = cg_finish_deferred(in.cg.fin);
    return ImgScal{(float)st.alpha, (float)st.beta};
  }
  return ImgScal{(float)*in.cg.alpha, (float)*in.cg.beta};
}
// element ix of the image row starting at pixel row0
// (buffer accesses: the row's base is workgroup-uniform, ix * 8 the thread's offset)
__device__ __forceinline__ float2 img_at(const ImgIn& in, long long row0, int ix, ImgScal sc, bool store) {
  const unsigned b = (unsigned)ix * 8u;
  const CGUpdate& c = in.cg;
  if (c.b0) {   // the CG start: r = gamma (b0 - N x) from the previous operator's partial images
    const auto rp = buf_rsrc(c.part + row0);
    float2 nv = buf_ld2(rp, b, 0u);
    for (int g = 1; g < c.G; ++g) nv = cadd(nv, buf_ld2(rp, b, (unsigned)((long long)g * c.N * 8)));
    const float2 bv = buf_ld2(buf_rsrc(c.b0 + row0), b, 0u);
    const float2 rv = make_float2(c.gamma * (bv.x - nv.x), c.gamma * (bv.y - nv.y));
    if (store) {
      const float2 z = make_float2(0.f, 0.f);
      buf_st2(buf_rsrc(c.u2 + row0), b, 0u, buf_ld2(buf_rsrc(c.u + row0), b, 0u));
      buf_st2(buf_rsrc(c.r2 + row0), b, 0u, rv);
      buf_st2(buf_rsrc(c.p2 + row0), b, 0u, z);
      buf_st2(buf_rsrc(c.s2 + row0), b, 0u, z);
    }
    return rv;
  }
  if (!c.r) return buf_ld2(buf_rsrc(in.x + row0), b, 0u);
  const float2 rv = buf_ld2(buf_rsrc(c.r + row0), b, 0u), sv = buf_ld2(buf_rsrc(c.s + row0), b, 0u);
  float2 wv;
  if (c.w) {
    wv = buf_ld2(buf_rsrc(c.w + row0), b, 0u);
  } else {   // w = c0 r + cg N r from the previous operator's coil-group partial images
    const auto rp = buf_rsrc(c.part + row0);
    float2 nv = buf_ld2(rp, b, 0u);
    for (int g = 1; g < c.G; ++g) nv = cadd(nv, buf_ld2(rp, b, (unsigned)((long long)g * c.N * 8)));
    wv = make_float2(c.c0 * rv.x + c.cg * nv.x, c.c0 * rv.y + c.cg * nv.y);
  }
  const float2 sn = make_float2(fmaf(sc.beta, sv.x, wv.x), fmaf(sc.beta, sv.y, wv.y));
  const float2 rn = make_float2(fmaf(-sc.alpha, sn.x, rv.x), fmaf(-sc.alpha, sn.y, rv.y));
  if (store) {
    const float2 pv = buf_ld2(buf_rsrc(c.p + row0), b, 0u), uv = buf_ld2(buf_rsrc(c.u + row0), b, 0u);
    const float2 pn = make_float2(fmaf(sc.beta, pv.x, rv.x), fmaf(sc.beta, pv.y, rv.y));
    buf_st2(buf_rsrc(c.p2 + row0), b, 0u, pn);
    buf_st2(buf_rsrc(c.s2 + row0), b, 0u, sn);
    buf_st2(buf_rsrc(c.u2 + row0), b, 0u, make_float2(fmaf(sc.alpha, pn.x, uv.x), fmaf(sc.alpha, pn.y, uv.y)));
    buf_st2(buf_rsrc(c.r2 + row0), b, 0u, rn);
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
  static_assert(K1 % 4 == 0 && K2 % 4 == 0, "padding patterns need factors divisible by 4");
};

// Twiddles of the four-step split (t < K2): W^(t k1) from the table's
// second part, laid out [k1][t] after the K roots, so the row offset
// k1 K2 is workgroup-uniform and the thread's offset t is shared by all k1.
template <int K1, int K2, bool INV>
__device__ __forceinline__ void fs_twiddle(float2 (&v)[K1], int t, const float2* __restrict__ tw) {
  const auto rsrc = buf_rsrc(tw + K1 * K2);
  const unsigned tb = (unsigned)t * 8u;
#pragma unroll
  for (int k1 = 1; k1 < K1; ++k1) {
    float2 w = buf_ld2(rsrc, tb + (unsigned)(k1 * K2 * 8), 0u);
    if (INV) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
}

// Row pass of the forward operator for image row iy and coil group g
// (RC coils, one line of K1 threads each: blockDim = RC * K1).  The
// workgroup first forms the row's input (image or CG residual, times the
// deapodisation) once into X, then each line multiplies by its coil map,
// zero-pads and transforms.  A: RC LA blocks of float2 LDS; X: nx float2.
// Shared by the single-slice, batched and 3D kernels.
template <int K1, int K2, int RC, bool HALF, typename OFF>
__device__ __forceinline__ void rows_fwd_body(const ImgIn& in, const float2* __restrict__ S, int L, int nx,
                                              int ny, const float* __restrict__ dax,
                                              const float* __restrict__ day, const float2* __restrict__ tw,
                                              float2* __restrict__ mid, int iy, int g, float2* A, float2* X) {
  using F = FS<K1, K2>;
  const int line = threadIdx.x / K1;
  const int t = threadIdx.x % K1;
  const int l0 = g * RC;
  const bool active = l0 + line < L;
  const long long N = (long long)nx * ny;
  const long long row0 = (long long)iy * nx;
  const float2* Sg = S ? S + (long long)l0 * N + row0 : nullptr;
  const OFF sb = (OFF)line * (OFF)N * 8u;
  // HALF: the map values of the line's K1/2 image pixels are loaded first,
  // so that their latency overlaps the row staging below
  constexpr int Q = K1 / 4;
  float2 sp[HALF ? 2 * Q : 1];
  if constexpr (HALF) {
    if (active && t < K2 && S) {
#pragma unroll
      for (int m = 0; m < 2 * Q; ++m) {
        const int ix = m < Q ? (m + Q) * K2 + t : (m - Q) * K2 + t;
        sp[m] = ld_off(Sg, sb + (OFF)ix * 8u);
      }
    }
  }
  {
    const float sy = day ? day[iy] : 1.f;     // no deapodisation table: Toeplitz operator
    const ImgScal bt = img_scal(in);
    const bool store = g == 0;
    for (int ix = threadIdx.x; ix < nx; ix += RC * K1)
      X[ix] = cscale(img_at(in, row0, ix, bt, store), (dax ? dax[ix] : 1.f) * sy);
  }
  __syncthreads();
  float2* Al = A + line * F::LA;
  if (active && t < K2) {
    float2 v[K1];
    auto at = [&](int ix) {
      return S ? cmul(ld_off(Sg, sb + (OFF)ix * 8u), X[ix]) : X[ix];
    };
    if constexpr (HALF) {
      // (S is uniform: one branch, not a select per element)
      if (S) {
#pragma unroll
        for (int n1 = 0; n1 < K1; ++n1) {
          if (n1 < Q) v[n1] = cmul(sp[n1], X[(n1 + Q) * K2 + t]);
          else if (n1 >= 3 * Q) v[n1] = cmul(sp[n1 - 2 * Q], X[(n1 - 3 * Q) * K2 + t]);
          else v[n1] = make_float2(0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int n1 = 0; n1 < K1; ++n1) {
          if (n1 < Q) v[n1] = X[(n1 + Q) * K2 + t];
          else if (n1 >= 3 * Q) v[n1] = X[(n1 - 3 * Q) * K2 + t];
          else v[n1] = make_float2(0.f, 0.f);
        }
      }
    } else {
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) {
        const int ix = img_of_grid(n1 * K2 + t, nx, F::K);
        v[n1] = ix >= 0 ? at(ix) : make_float2(0.f, 0.f);
      }
    }
    if constexpr (HALF) reg::dft_halfzero<K1, false>(v);
    else reg::dft<K1, false>(v);
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
    float2* dst = mid + ((long long)l0 * ny + iy) * F::K;
    const OFF db = ((OFF)line * (OFF)ny * (OFF)F::K + (OFF)t) * 8u;
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) st_off(dst, db + (OFF)(K1 * k2 * 8), u[k2]);
  }
}

// Row pass of the adjoint for image row iy and coil group g: inverse row
// FFT, crop, deapodisation, conj(S_l) and the sum over the group's RC coils
// into part[g]; A: RC LA blocks of float2 LDS.
template <int K1, int K2, int RC, bool HALF, typename OFF>
__device__ __forceinline__ void rows_adj_body(const float2* __restrict__ mid, const float2* __restrict__ S, int L,
                                              int nx, int ny, const float* __restrict__ dax,
                                              const float* __restrict__ day, const float2* __restrict__ tw,
                                              float2* __restrict__ part, int iy, int g, float2* A,
                                              const FusedDots& fd) {
  using F = FS<K1, K2>;
  const int line = threadIdx.x / K1;
  const int t = threadIdx.x % K1;
  const int l0 = g * RC;
  const bool active = l0 + line < L;
  const long long N = (long long)nx * ny;
  float2* Al = A + line * F::LA;
  const float2* Sg = S ? S + (long long)l0 * N + (long long)iy * nx : nullptr;
  const OFF sbm = (OFF)line * (OFF)N * 8u;
  // HALF: the map values of the line's K2/2 kept pixels are loaded with the
  // grid row, ahead of the transforms that produce the values they multiply
  constexpr int P = K2 / 4;
  float2 sp[HALF ? 2 * P : 1];
  if constexpr (HALF && sizeof(OFF) == 4) {
    if (active && S) {   // (buffer loads: the thread's offset plus a constant scalar one)
      const auto rs = buf_rsrc(Sg);
#pragma unroll
      for (int m = 0; m < 2 * P; ++m)
        sp[m] = buf_ld2(rs, (unsigned)sbm + (unsigned)t * 8u, (unsigned)(K1 * (m < P ? m + P : m - P) * 8));
    }
  } else if constexpr (HALF) {
    if (active && S) {
#pragma unroll
      for (int m = 0; m < 2 * P; ++m) {
        const int ix = m < P ? t + K1 * (m + P) : t + K1 * (m - P);
        sp[m] = ld_off(Sg, sbm + (OFF)ix * 8u);
      }
    }
  }
  if (active && t < K2) {
    float2 v[K1];
    const float2* src = mid + ((long long)l0 * ny + iy) * F::K;
    const OFF sb = ((OFF)line * (OFF)ny * (OFF)F::K + (OFF)t) * 8u;
    if constexpr (sizeof(OFF) == 4) {
      const auto rs = buf_rsrc(src);
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) v[n1] = buf_ld2(rs, (unsigned)sb, (unsigned)(n1 * K2 * 8));
    } else {
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) v[n1] = ld_off(src, sb + (OFF)(n1 * K2 * 8));
    }
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
    auto put = [&](int ix, float2 v) { Z[line * nx + ix] = S ? cmulc(ld_off(Sg, sbm + (OFF)ix * 8u), v) : v; };
    if constexpr (HALF) {
      // (S is uniform: one branch, not a select per element)
      if (S) {
#pragma unroll
        for (int k2 = 0; k2 < K2; ++k2) {
          if (k2 < P) Z[line * nx + t + K1 * (k2 + P)] = cmulc(sp[k2], u[k2]);
          else if (k2 >= 3 * P) Z[line * nx + t + K1 * (k2 - 3 * P)] = cmulc(sp[k2 - 2 * P], u[k2]);
        }
      } else {
#pragma unroll
        for (int k2 = 0; k2 < K2; ++k2) {
          if (k2 < P) Z[line * nx + t + K1 * (k2 + P)] = u[k2];
          else if (k2 >= 3 * P) Z[line * nx + t + K1 * (k2 - 3 * P)] = u[k2];
        }
      }
    } else {
#pragma unroll
      for (int k2 = 0; k2 < K2; ++k2) {
        const int ix = img_of_grid(t + K1 * k2, nx, F::K);
        if (ix >= 0) put(ix, u[k2]);
      }
    }
  }
  __syncthreads();
  const int nl = min(RC, L - l0);
  const float sy = day ? day[iy] : 1.f;     // no deapodisation table: Toeplitz operator
  float2* pg = part + (long long)g * N + (long long)iy * nx;
  const float2* rrow = fd.r ? fd.r + (long long)iy * nx : nullptr;
  double rr = 0.0, d = 0.0;
  for (int ix = threadIdx.x; ix < nx; ix += blockDim.x) {
    float2 acc = Z[ix];
    for (int li = 1; li < nl; ++li) acc = cadd(acc, Z[li * nx + ix]);
    const float2 v = cscale(acc, (dax ? dax[ix] : 1.f) * sy);
    pg[ix] = v;
    if (rrow) {
      const float2 rv = rrow[ix];
      d += (double)v.x * rv.x + (double)v.y * rv.y;
      if (g == 0) rr += (double)rv.x * rv.x + (double)rv.y * rv.y;
    }
  }
  if (fd.parts) {                             // (uniform) |r|^2 (group 0) and Re<part_g, r> over the row
    __shared__ double sh[2][(RC * K1 + 63) / 64];
    d = wg_sum<RC * K1>(d, sh[0]);
    if (g == 0) rr = wg_sum<RC * K1>(rr, sh[1]);
    if (threadIdx.x == 0) {
      double* slot = fd.parts + 2 * ((long long)fd.ny * g + iy);
      slot[0] = rr;
      slot[1] = d;
    }
  }
}

// Column passes over a strip of 8 grid columns (one thread column c per
// grid column, threads t < K1 along the column), in registers with LDS
// transposes.  `strip` is the workgroup's column 0; column c, grid row j
// sits at strip[c + j * rs].  The column is the zero-padded image of
// `nimg` rows (img_of_grid placement) on the input side of the forward
// transform and on the output side of the inverse one.
//   forward   n = n1*K2 + n2, k = k1 + K1*k2: thread n2 runs the DFT over n1,
//             twiddle, transpose, thread k1 runs the DFT over n2
//             -> u[k2] = X[t + K1*k2]
//   inverse   k = k1 + K1*k2, r = r2 + K2*r1: thread k1 runs the inverse DFT
//             over k2, twiddle exp(+2 pi i k1 r2 / K), transpose, thread r2
//             runs the inverse DFT over k1 -> y[r2 + K2*r1]
// lds: 8 * CS float2.  Every thread of the workgroup must call these.
template <int K1, int K2, bool HALF, typename OFF>
__device__ __forceinline__ void col_fwd(const float2* __restrict__ strip, OFF rs, int nimg, bool colok,
                                        const float2* __restrict__ tw, float2* lds, float2 (&u)[K2]) {
  using F = FS<K1, K2>;
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  if (colok && t < K2) {
    float2 v[K1];
    const OFF rb = rs * 8u;
    const OFF cb = (OFF)c * 8u + (OFF)t * rb;
    if constexpr (HALF && sizeof(OFF) == 4) {
      constexpr int Q = K1 / 4;
      const auto rsrc = buf_rsrc(strip);
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) {
        if (n1 < Q) v[n1] = buf_ld2(rsrc, cb, (unsigned)((n1 + Q) * K2) * rb);
        else if (n1 >= 3 * Q) v[n1] = buf_ld2(rsrc, cb, (unsigned)((n1 - 3 * Q) * K2) * rb);
        else v[n1] = make_float2(0.f, 0.f);
      }
    } else if constexpr (HALF) {
      constexpr int Q = K1 / 4;
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) {
        if (n1 < Q) v[n1] = ld_off(strip, cb + (OFF)((n1 + Q) * K2) * rb);
        else if (n1 >= 3 * Q) v[n1] = ld_off(strip, cb + (OFF)((n1 - 3 * Q) * K2) * rb);
        else v[n1] = make_float2(0.f, 0.f);
      }
    } else {
#pragma unroll
      for (int n1 = 0; n1 < K1; ++n1) {
        const int iy = img_of_grid(n1 * K2 + t, nimg, F::K);
        v[n1] = iy >= 0 ? ld_off(strip, (OFF)c * 8u + (OFF)iy * rb) : make_float2(0.f, 0.f);
      }
    }
    if constexpr (HALF) reg::dft_halfzero<K1, false>(v);
    else reg::dft<K1, false>(v);
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

template <int K1, int K2, bool HALF, typename OFF>
__device__ __forceinline__ void col_inv(float2* __restrict__ strip, OFF rs, int nimg, bool colok,
                                        const float2* __restrict__ tw, float2* lds, float2 (&u)[K2]) {
  using F = FS<K1, K2>;
  constexpr int AS2 = K1 + 1;          // row stride of the second transpose
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  if (colok) {
    reg::dft<K2, true>(u);
    // W^(t r2) from the table's third part, laid out [r2][t] (t < K1)
    const auto rsrc = buf_rsrc(tw + 2 * K1 * K2);
    const unsigned tb = (unsigned)t * 8u;
#pragma unroll
    for (int r2 = 1; r2 < K2; ++r2) {
      float2 w = buf_ld2(rsrc, tb + (unsigned)(r2 * K1 * 8), 0u);
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
    const OFF rb = rs * 8u;
    const OFF cb = (OFF)c * 8u + (OFF)t * rb;
    if constexpr (HALF && sizeof(OFF) == 4) {
      constexpr int Q = K1 / 4;
      const auto rsrc = buf_rsrc(strip);
#pragma unroll
      for (int r1 = 0; r1 < K1; ++r1) {
        if (r1 < Q) buf_st2(rsrc, cb, (unsigned)(K2 * (r1 + Q)) * rb, z[r1]);
        else if (r1 >= 3 * Q) buf_st2(rsrc, cb, (unsigned)(K2 * (r1 - 3 * Q)) * rb, z[r1]);
      }
    } else if constexpr (HALF) {
      constexpr int Q = K1 / 4;
#pragma unroll
      for (int r1 = 0; r1 < K1; ++r1) {
        if (r1 < Q) st_off(strip, cb + (OFF)(K2 * (r1 + Q)) * rb, z[r1]);
        else if (r1 >= 3 * Q) st_off(strip, cb + (OFF)(K2 * (r1 - 3 * Q)) * rb, z[r1]);
      }
    } else {
#pragma unroll
      for (int r1 = 0; r1 < K1; ++r1) {
        const int iy = img_of_grid(t + K2 * r1, nimg, F::K);
        if (iy >= 0) st_off(strip, (OFF)c * 8u + (OFF)iy * rb, z[r1]);
      }
    }
  }
  __syncthreads();
}

// Toeplitz column pass (2D): zero-padded column FFT, multiplication by the
// real transfer function T, inverse FFT, for grid columns [c0, c0 + tile) of
// coil l; only the ny = K/2 image rows of mid are read and written (in
// place).  Every offset within one coil's mid fits 32 bits.
template <int K1, int K2>
__device__ __forceinline__ void cols_toep_body(float2* __restrict__ mid, int ny, int Kx,
                                               const float2* __restrict__ tw, int tile,
                                               const float* __restrict__ T, int c0, int l, float2* lds) {
  const int c = threadIdx.x % 8;
  const int t = threadIdx.x / 8;
  const bool colok = c < tile;
  float2* strip = mid + (long long)l * ny * Kx + c0;
  float2 u[K2];
  col_fwd<K1, K2, true, unsigned>(strip, (unsigned)Kx, ny, colok, tw, lds, u);
  if (colok) {
    const auto rsrc = buf_rsrc(T + c0);
    const unsigned tb = ((unsigned)c + (unsigned)t * (unsigned)Kx) * 4u;
#pragma unroll
    for (int k2 = 0; k2 < K2; ++k2) u[k2] = cscale(u[k2], buf_ld1(rsrc, tb, (unsigned)(K1 * k2) * (unsigned)Kx * 4u));
  }
  col_inv<K1, K2, true, unsigned>(strip, (unsigned)Kx, ny, colok, tw, lds, u);
}

}  // namespace pnp
