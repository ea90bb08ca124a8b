// Haar soft-threshold prior D_sigma(u) (the plain method's plug-in denoiser).
//
// An orthonormal Haar transform with J levels never mixes pixels of
// different 2^J x 2^J (x 2^J) blocks, so the whole prior -- J analysis
// levels, soft threshold of the detail coefficients, J synthesis levels --
// runs block by block in LDS with one read and one write of the image.
// Within a block the coefficients sit in the usual pyramid layout; the
// single coarsest approximation coefficient of a block (index 0) is the
// only one left unthresholded.  Soft threshold: c * max(0, 1 - tau/|c|).
#include "cg_scalars.hpp"
#include "common.hpp"
#include "trace.hpp"

namespace pnp {

namespace {

constexpr float kInvSqrt2 = 0.70710678118654752440f;

// One analysis (INV=false) or synthesis (INV=true) step along `axis` on the
// leading m^ndim region of a B^ndim block (B = 2^J), src -> dst (whole block
// copied).  Coordinates by shifts and masks: B is a power of two.
template <bool INV>
__device__ void haar_step(const float2* __restrict__ src, float2* __restrict__ dst, int ndim, int J,
                          int m, int axis) {
  const int B = 1 << J;
  const int total = ndim == 3 ? B * B * B : B * B;
  const int h = m >> 1;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int q[3];
    q[0] = t & (B - 1);                       // x
    q[1] = (t >> J) & (B - 1);                // y
    q[2] = ndim == 3 ? t >> (2 * J) : 0;      // z
    const bool in = q[0] < m && q[1] < m && (ndim == 2 || q[2] < m);
    if (!in) {
      dst[t] = src[t];
      continue;
    }
    const int stride = axis == 0 ? 1 : (axis == 1 ? B : B * B);
    const int qa = q[axis];
    const int base = t - qa * stride;
    float2 o;
    if (!INV) {
      const int k = qa < h ? qa : qa - h;
      const float2 e = src[base + (2 * k) * stride];
      const float2 od = src[base + (2 * k + 1) * stride];
      o = qa < h ? make_float2((e.x + od.x) * kInvSqrt2, (e.y + od.y) * kInvSqrt2)
                 : make_float2((e.x - od.x) * kInvSqrt2, (e.y - od.y) * kInvSqrt2);
    } else {
      const int k = qa >> 1;
      const float2 lo = src[base + k * stride];
      const float2 hi = src[base + (h + k) * stride];
      o = (qa & 1) ? make_float2((lo.x - hi.x) * kInvSqrt2, (lo.y - hi.y) * kInvSqrt2)
                   : make_float2((lo.x + hi.x) * kInvSqrt2, (lo.y + hi.y) * kInvSqrt2);
    }
    dst[t] = o;
  }
}

// Linear image index of element t of block `blk` (2^J pixels per axis).
__device__ __forceinline__ long long haar_index(int t, int ndim, int nx, int ny, int J, int blk) {
  const int B = 1 << J;
  const int bx = nx / B, by = ny / B;
  const int ox = (blk % bx) * B;
  const int oy = ((blk / bx) % by) * B;
  const int oz = ndim == 3 ? (blk / (bx * by)) * B : 0;
  const int x = t & (B - 1), y = (t >> J) & (B - 1), z = ndim == 3 ? t >> (2 * J) : 0;
  return ((long long)(oz + z) * ny + (oy + y)) * nx + ox + x;
}

// One 2^J (per axis) block `blk` of the image: analysis, soft threshold
// of every detail coefficient, synthesis; lds: 2 * 2^(J*ndim) float2.
// load(t, i) gives the input pixel of linear index i (element t of the block).
template <class Load>
__device__ void haar_block(Load load, float2* __restrict__ out, int ndim, int nx, int ny, int J, float tau,
                           int blk, float2* lds) {
  const int B = 1 << J;
  const int total = ndim == 3 ? B * B * B : B * B;
  float2* a = lds;
  float2* b = lds + total;
  for (int t = threadIdx.x; t < total; t += blockDim.x) a[t] = load(t, haar_index(t, ndim, nx, ny, J, blk));
  __syncthreads();
  for (int l = 0; l < J; ++l) {
    const int m = B >> l;
    for (int ax = 0; ax < ndim; ++ax) {
      haar_step<false>(a, b, ndim, J, m, ax);
      __syncthreads();
      float2* t = a; a = b; b = t;
    }
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    if (t == 0) continue;
    const float2 c = a[t];
    const float mag = sqrtf(c.x * c.x + c.y * c.y);
    const float f = mag > tau ? 1.0f - tau / mag : 0.0f;
    a[t] = make_float2(c.x * f, c.y * f);
  }
  __syncthreads();
  for (int l = J - 1; l >= 0; --l) {
    const int m = B >> l;
    for (int ax = ndim - 1; ax >= 0; --ax) {
      haar_step<true>(a, b, ndim, J, m, ax);
      __syncthreads();
      float2* t = a; a = b; b = t;
    }
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) out[haar_index(t, ndim, nx, ny, J, blk)] = a[t];
}

__global__ void k_haar_prior(const float2* __restrict__ in, float2* __restrict__ out, int ndim,
                             int nx, int ny, int nz, int J, float tau) {
  extern __shared__ float2 lds[];
  haar_block([in](int, long long i) { return in[i]; }, out, ndim, nx, ny, J, tau, blockIdx.x, lds);
}

// The prior applied to the last CG update u + alpha (r + beta p), formed on
// the fly: alpha and beta come from the step's block sums, summed by every
// wave in the fixed order (workgroup 0 records the step's state).  The
// thread's first pixel of r, p and u is loaded before the sums, so that its
// latency overlaps theirs (in 2D with 16 x 16 blocks that is every pixel).
__global__ void __launch_bounds__(256)
k_haar_prior_cg(const float2* __restrict__ r, const float2* __restrict__ p, const float2* __restrict__ u,
                CGFinish fin, float2* __restrict__ out, int ndim, int nx, int ny, int nz, int J, float tau) {
  extern __shared__ float2 lds[];
  const int total = ndim == 3 ? 1 << (3 * J) : 1 << (2 * J);
  const int t0 = threadIdx.x;
  float2 r0 = make_float2(0.f, 0.f), p0 = r0, u0 = r0;
  if (t0 < total) {
    const long long i0 = haar_index(t0, ndim, nx, ny, J, blockIdx.x);
    r0 = r[i0];
    p0 = p[i0];
    u0 = u[i0];
  }
  const CgStep st = cg_finish_deferred(fin);
  const float a = (float)st.alpha, b = (float)st.beta;
  haar_block(
      [=](int t, long long i) {
        const bool first = t == t0;
        const float2 rv = first ? r0 : r[i], pv = first ? p0 : p[i], uv = first ? u0 : u[i];
        const float2 pn = make_float2(fmaf(b, pv.x, rv.x), fmaf(b, pv.y, rv.y));
        return make_float2(fmaf(a, pn.x, uv.x), fmaf(a, pn.y, uv.y));
      },
      out, ndim, nx, ny, J, tau, blockIdx.x, lds);
}

// Batched 2D prior: workgroup b belongs to the last slice with block0 <= b.
__global__ void k_haar_prior_batched(const HaarSlice* __restrict__ sl, int n_slices, int J, float tau) {
  extern __shared__ float2 lds[];
  int s = 0;
  while (s + 1 < n_slices && sl[s + 1].block0 <= (int)blockIdx.x) ++s;
  const float2* in = sl[s].in;
  haar_block([in](int, long long i) { return in[i]; }, sl[s].out, 2, sl[s].nx, sl[s].ny, J, tau,
             blockIdx.x - sl[s].block0, lds);
}

}  // namespace

int wavelet_default_levels(int nmin) {
  int lg = 0;
  while ((2 << lg) <= nmin) ++lg;  // floor(log2 nmin)
  int J = lg - 3;
  if (J > 4) J = 4;
  if (J < 1) J = 1;
  return J;
}

void wavelet_apply_batched(const HaarSlice* sl, int n_slices, int total_blocks, int levels, float tau,
                           hipStream_t s) {
  const int B = 1 << levels;
  const size_t lds = sizeof(float2) * 2 * B * B;
  PNP_LAUNCH(k_haar_prior_batched, dim3((unsigned)total_blocks), dim3(256), lds, s, sl, n_slices, levels, tau);
}

void wavelet_apply_cg(int ndim, const int* n, int levels, float tau, const float2* r, const float2* p,
                      const float2* u, const CGFinish& fin, float2* out, hipStream_t s) {
  const int B = 1 << levels;
  for (int a = 0; a < ndim; ++a)
    if (n[a] % B) fail(PNP_ERR_SHAPE, "image side %d not divisible by 2^%d", n[a], levels);
  long long blocks = 1;
  for (int a = 0; a < ndim; ++a) blocks *= n[a] / B;
  const int total = ndim == 3 ? B * B * B : B * B;
  const size_t lds = sizeof(float2) * 2 * total;
  PNP_LAUNCH(k_haar_prior_cg, dim3((unsigned)blocks), dim3(256), lds, s, r, p, u, fin, out, ndim, n[0], n[1],
             ndim == 3 ? n[2] : 1, levels, tau);
  PNP_CHECK_LAUNCH();
}

void wavelet_apply(int ndim, const int* n, int levels, float tau, const float2* in, float2* out,
                   hipStream_t s) {
  const int B = 1 << levels;
  for (int a = 0; a < ndim; ++a)
    if (n[a] % B) fail(PNP_ERR_SHAPE, "image side %d not divisible by 2^%d", n[a], levels);
  long long blocks = 1;
  for (int a = 0; a < ndim; ++a) blocks *= n[a] / B;
  const int total = ndim == 3 ? B * B * B : B * B;
  const size_t lds = sizeof(float2) * 2 * total;
  PNP_LAUNCH(k_haar_prior, dim3((unsigned)blocks), dim3(256), lds, s, in, out, ndim, n[0],
                     n[1], ndim == 3 ? n[2] : 1, levels, tau);
  PNP_CHECK_LAUNCH();
}

}  // namespace pnp
