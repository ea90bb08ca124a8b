// Device-resident scalar state of the CG proximal solver and power
// iteration, and the scalar updates that close a CG reduction.
#pragma once

#include "common.hpp"

namespace pnp {

constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 256;

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-reduce Q values into parts[bidx*Q + q]; the last of `nblocks`
// blocks to arrive (atomic ticket on *cnt) sums all partials in a fixed
// order into out[], resets the ticket and returns true (for every thread of
// that block).  Deterministic.
template <int Q>
__device__ bool reduce_last_of(double (&v)[Q], double* __restrict__ parts, unsigned* cnt, int nblocks, int bidx,
                               double (&out)[Q]) {
  __shared__ double sh[Q][kRedThreads / 64];
  __shared__ double fin[Q][kRedThreads];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double s = warp_sum(v[q]);
    if (lane == 0) sh[q][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[q][w];
      parts[bidx * Q + q] = s;
    }
    __threadfence();
    const unsigned prev = atomicAdd(cnt, 1u);
    last = prev == (unsigned)(nblocks - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const volatile double* vp = parts;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += vp[b * Q + q];
    fin[q][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < Q; ++q) fin[q][threadIdx.x] += fin[q][threadIdx.x + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) out[q] = fin[q][0];
  if (threadIdx.x == 0) *cnt = 0u;
  return true;
}

template <int Q>
__device__ bool reduce_last(double (&v)[Q], double* __restrict__ parts, unsigned* cnt, double (&out)[Q]) {
  return reduce_last_of<Q>(v, parts, cnt, (int)gridDim.x, (int)blockIdx.x, out);
}

// Two-kernel form of the same reduction, for the reductions on the CG
// path: every block writes its Q block sums to parts[bidx*Q + q] with
// plain stores (block_parts), and a following one-workgroup kernel sums
// the partial sets in the same fixed order (sum_parts).  The kernel
// boundary orders the stores, so no block pays a device-scope fence and an
// atomic ticket.
template <int Q>
__device__ void block_parts(double (&v)[Q], double* __restrict__ parts, int bidx) {
  __shared__ double sh[Q][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double s = warp_sum(v[q]);
    if (lane == 0) sh[q][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < Q) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[threadIdx.x][w];
    parts[bidx * Q + threadIdx.x] = s;
  }
}

// Sum of `nblocks` partial sets by one wave (launch with kFinThreads = 64
// threads): lane j adds sets j, j + 64, ... in order, then a shuffle tree
// combines the lanes -- no barriers; a fixed order, so deterministic.
// Every lane receives the sums.
constexpr int kFinThreads = 64;
template <int Q>
__device__ void sum_parts(const double* __restrict__ parts, int nblocks, double (&out)[Q]) {
  const int lane = threadIdx.x & 63;
  // eight sets per lane loaded before they are added (in the same order)
  double s[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) s[q] = 0.0;
  // (buffer loads: the set offsets u * 64 * Q doubles are scalar, the lane's own offset shared)
  const auto rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(parts), (short)0, 0x7fffffff, 0x00020000);
  int b = lane;
  for (; b + 7 * 64 < nblocks; b += 8 * 64) {
    double v[8][Q];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int q = 0; q < Q; ++q)
        v[u][q] = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(rsrc, (b * Q + q) * 8, u * 64 * Q * 8, 0));
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int q = 0; q < Q; ++q) s[q] += v[u][q];
  }
  for (; b < nblocks; b += 64)
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] += parts[b * Q + q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o, 64);
    out[q] = s[q];
  }
}

// sum_parts for a workgroup of 32 lanes or of whole waves: with 32 lanes,
// lane j also adds the sets of lane j + 32 of the 64-lane order and the
// first level of the tree becomes that addition, so the result equals
// sum_parts' bit for bit.
template <int Q>
__device__ void sum_parts_any(const double* __restrict__ parts, int nblocks, double (&out)[Q]) {
  if (blockDim.x >= 64) {
    sum_parts<Q>(parts, nblocks, out);
    return;
  }
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double a = 0.0, b = 0.0;
    for (int k = lane; k < nblocks; k += 64) a += parts[k * Q + q];
    for (int k = lane + 32; k < nblocks; k += 64) b += parts[k * Q + q];
    double s = a + b;
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    out[q] = s;
  }
}

struct DevScalars {
  double rr;        // <r, r>
  double pq;        // Re <w, r> of the last step (w = M r)
  double alpha;     // CG step
  double beta;      // CG direction update
  double yw2;       // ||y||^2_w
  double lam;       // power iteration: Rayleigh quotient
  double inv;       // power iteration: 1/||w||
  int bad;          // set when a CG denominator is not positive / finite
  unsigned cnt;     // last-block ticket (reset by the last block)
  int bad_saved;    // `bad` as of the last CG start (restored when a queued CG is discarded)
};

// Chronopoulos-Gear step sizes from g = <r,r> and d = Re<M r, r>:
//   first step:  beta = 0, alpha = g / d
//   later steps: beta = g / rr, alpha = g / (d - beta g / alpha)
// then rr = g.  A zero residual gives alpha = beta = 0; a non-positive or
// non-finite denominator sets `bad` and alpha = beta = 0 (u stops moving).
struct CgStep {
  double alpha, beta, rr;
  int bad;
};
__device__ inline CgStep cg_step(double g, double d, int first, double rr_prev, double alpha_prev) {
  CgStep st{0.0, 0.0, g, 0};
  if (g > 0.0 && isfinite(g)) {
    const bool restart = first || !(alpha_prev != 0.0) || !(rr_prev > 0.0);
    st.beta = restart ? 0.0 : g / rr_prev;
    const double den = restart ? d : d - st.beta * g / alpha_prev;
    if (den > 0.0 && isfinite(den)) {
      st.alpha = g / den;
    } else {
      st.beta = 0.0;
      st.bad = 1;
    }
  } else if (!isfinite(g)) {
    st.bad = 1;
  }
  return st;
}
__device__ inline void cg_finish_dots(DevScalars* sc, double g, double d, int first) {
  const CgStep st = cg_step(g, d, first, sc->rr, sc->alpha);
  if (st.bad) sc->bad = 1;
  sc->pq = d;
  sc->alpha = st.alpha;
  sc->beta = st.beta;
  sc->rr = st.rr;
}
// The finisher of CGFinish f run by every wave of a consuming pass (all
// lanes active; workgroups of 32 lanes or of whole waves); workgroup 0
// stores the state.
__device__ inline CgStep cg_finish_deferred(const CGFinish& f) {
  double s[2];
  sum_parts_any<2>(f.parts, f.nparts, s);
  if (f.fused) s[1] = (double)f.c0 * s[0] + (double)f.cg * s[1];
  const double rr_prev = f.first ? 0.0 : f.prev->rr;
  const double alpha_prev = f.first ? 0.0 : f.prev->alpha;
  const CgStep st = cg_step(s[0], s[1], f.first, rr_prev, alpha_prev);
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) {
    f.next->pq = s[1];
    f.next->alpha = st.alpha;
    f.next->beta = st.beta;
    f.next->rr = st.rr;
    if (st.bad) *f.bad = 1;
  }
  return st;
}

// CG start: rr = <r0,r0>; rho(x) = <x,Nx> - 2 Re<x,b0> + ||y||_w^2.
__device__ inline void cg_finish_init(DevScalars* sc, double rr, double xnx, double xb0, double* rho_out) {
  sc->rr = rr;
  if (rho_out) *rho_out = xnx - 2.0 * xb0 + sc->yw2;
}

}  // namespace pnp
