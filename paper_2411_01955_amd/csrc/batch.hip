// Batched annealed PnP-HQS over many 2D slices of different sizes, coil
// counts and trajectories (one GPU).  Every stage of the Toeplitz normal
// operator is one launch per grid size over the work items of all slices of
// that size (largest size first); the CG vector work and its FP64
// reductions are single launches over (slice, chunk) items with one
// last-block ticket per slice; the Haar prior is one launch over all
// slices' blocks and the UNet prior one batched forward per image size.
// The slices are independent problems that share the sigma schedule, the
// preconditioner and n_cg (Sec. 3.3-3.4 per slice).
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <vector>

#include "cg_scalars.hpp"
#include "common.hpp"
#include "trace.hpp"

namespace pnp {

constexpr int kMaxBatch = 64;
constexpr int kChunk = 8192;            // vector elements per (slice, chunk) item
constexpr int kBatchMaxOuter = 1024;

// per-slice vectors (device table entry)
struct BVec {
  float2 *x, *b0, *w, *u[2], *r[2], *p[2], *s[2];
  float2* xout;                          // caller's output
  const float2* part;                    // coil-group partials of the operator
  int G;
  long long N;
};

struct SliceCoef {
  float gamma[kMaxBatch];
  float cg[kMaxBatch];
};

namespace {

__device__ __forceinline__ double re_dot(float2 a, float2 b) { return (double)a.x * b.x + (double)a.y * b.y; }

__device__ __forceinline__ float2 sum_groups(const float2* __restrict__ part, int G, long long N, long long i) {
  float2 v = part[i];
  for (int g = 1; g < G; ++g) v = cadd(v, part[(long long)g * N + i]);
  return v;
}

// chunk items: {slice, first element, chunk index within the slice, chunks of the slice}
__global__ void __launch_bounds__(kRedThreads)
k_bcg_init(const int4* __restrict__ ch, const BVec* __restrict__ vec, SliceCoef co, double* __restrict__ parts) {
  const int4 c = ch[blockIdx.x];
  const BVec& v = vec[c.x];
  const long long e = std::min<long long>((long long)c.y + kChunk, v.N);
  const float gamma = co.gamma[c.x];
  double acc[3] = {0.0, 0.0, 0.0};
  const float2 z = make_float2(0.f, 0.f);
  for (long long i = c.y + threadIdx.x; i < e; i += blockDim.x) {
    const float2 xv = v.x[i], nv = sum_groups(v.part, v.G, v.N, i), bv = v.b0[i];
    const float2 rv = make_float2(gamma * (bv.x - nv.x), gamma * (bv.y - nv.y));
    v.u[0][i] = xv;
    v.r[0][i] = rv;
    v.p[0][i] = z;
    v.s[0][i] = z;
    acc[0] += re_dot(rv, rv);
    acc[1] += re_dot(xv, nv);
    acc[2] += re_dot(xv, bv);
  }
  block_parts<3>(acc, parts + (long long)c.x * kRedBlocks * 3, c.z);
}

// one workgroup per slice: the slice's chunk sums -> rr and rho
__global__ void __launch_bounds__(kFinThreads)
k_bcg_init_fin(const BVec* __restrict__ vec, const double* __restrict__ parts, DevScalars* __restrict__ sc,
               double* __restrict__ rho, int k) {
  const int i = blockIdx.x;
  const int nch = (int)((vec[i].N + kChunk - 1) / kChunk);
  double s[3];
  sum_parts<3>(parts + (long long)i * kRedBlocks * 3, nch, s);
  if (threadIdx.x == 0) cg_finish_init(&sc[i], s[0], s[1], s[2], rho + (long long)i * (kBatchMaxOuter + 1) + k);
}

__global__ void __launch_bounds__(kRedThreads)
k_bcg_dots(const int4* __restrict__ ch, const BVec* __restrict__ vec, SliceCoef co, float c0, int cur,
           double* __restrict__ parts) {
  const int4 c = ch[blockIdx.x];
  const BVec& v = vec[c.x];
  const long long e = std::min<long long>((long long)c.y + kChunk, v.N);
  const float cg = co.cg[c.x];
  const float2* r = v.r[cur];
  double acc[2] = {0.0, 0.0};
  for (long long i = c.y + threadIdx.x; i < e; i += blockDim.x) {
    const float2 rv = r[i], nv = sum_groups(v.part, v.G, v.N, i);
    const float2 wv = make_float2(c0 * rv.x + cg * nv.x, c0 * rv.y + cg * nv.y);
    v.w[i] = wv;
    acc[0] += re_dot(rv, rv);
    acc[1] += re_dot(wv, rv);
  }
  block_parts<2>(acc, parts + (long long)c.x * kRedBlocks * 3, c.z);
}

// one workgroup per slice: the slice's chunk sums -> alpha, beta, rr
__global__ void __launch_bounds__(kFinThreads)
k_bcg_dots_fin(const BVec* __restrict__ vec, const double* __restrict__ parts, int first,
               DevScalars* __restrict__ sc) {
  const int i = blockIdx.x;
  const int nch = (int)((vec[i].N + kChunk - 1) / kChunk);
  double s[2];
  sum_parts<2>(parts + (long long)i * kRedBlocks * 3, nch, s);
  if (threadIdx.x == 0) cg_finish_dots(&sc[i], s[0], s[1], first);
}

// u[1-cur] = u[cur] + alpha (r[cur] + beta p[cur])
__global__ void k_bcg_final(const int4* __restrict__ ch, const BVec* __restrict__ vec, int cur,
                            const DevScalars* __restrict__ sc) {
  const int4 c = ch[blockIdx.x];
  const BVec& v = vec[c.x];
  const long long e = std::min<long long>((long long)c.y + kChunk, v.N);
  const float a = (float)sc[c.x].alpha, b = (float)sc[c.x].beta;
  for (long long i = c.y + threadIdx.x; i < e; i += blockDim.x) {
    const float2 rv = v.r[cur][i], pv = v.p[cur][i], uv = v.u[cur][i];
    const float2 pn = make_float2(fmaf(b, pv.x, rv.x), fmaf(b, pv.y, rv.y));
    v.u[1 - cur][i] = make_float2(fmaf(a, pn.x, uv.x), fmaf(a, pn.y, uv.y));
  }
}

// which: 0 x = b0, 1 xout = x, 2 out = sum of the operator's group partials (out table)
__global__ void k_bcopy(const int4* __restrict__ ch, const BVec* __restrict__ vec, int which,
                        float2* const* __restrict__ outs) {
  const int4 c = ch[blockIdx.x];
  const BVec& v = vec[c.x];
  const long long e = std::min<long long>((long long)c.y + kChunk, v.N);
  for (long long i = c.y + threadIdx.x; i < e; i += blockDim.x) {
    if (which == 0)
      v.x[i] = v.b0[i];
    else if (which == 1)
      v.xout[i] = v.x[i];
    else
      outs[c.x][i] = sum_groups(v.part, v.G, v.N, i);
  }
}

__global__ void k_binit_scalars(DevScalars* sc, int B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  sc[s].rr = sc[s].pq = sc[s].alpha = sc[s].beta = sc[s].yw2 = sc[s].lam = sc[s].inv = 0.0;
  sc[s].bad = 0;
  sc[s].cnt = 0u;
}

// ||y||^2_w of one slice into sc->yw2
__global__ void __launch_bounds__(kRedThreads)
k_bwnorm(long long M, int L, const float2* __restrict__ y, const float* __restrict__ dcf,
         double* __restrict__ parts, DevScalars* sc) {
  double acc[1] = {0.0};
  const long long T = M * L;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T;
       t += (long long)gridDim.x * blockDim.x) {
    const float2 v = y[t];
    acc[0] += (dcf ? (double)dcf[t % M] : 1.0) * re_dot(v, v);
  }
  double s[1];
  if (reduce_last<1>(acc, parts, &sc->cnt, s) && threadIdx.x == 0) sc->yw2 = s[0];
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace pnp

struct pnp_batch {
  struct Host {
    pnp_slice s;
    int n, K, G;
    long long N;
    int group;             // image-size group
    long long voff;        // offset of the slice's vectors (memory order)
  };
  int B = 0;
  std::vector<Host> h;
  std::vector<int> order;                 // slices in memory order (grouped by size)
  std::vector<std::pair<int, std::vector<int>>> groups;   // (n, slices in memory order)
  void* block = nullptr;
  pnp::BatchSlice* d_sl = nullptr;
  pnp::BVec* d_vec = nullptr;
  pnp::NormalIn* d_in[5] = {};            // x | r0 | CG 0->1 | CG 1->0 | caller's x
  float2** d_outs = nullptr;
  int4* d_rows = nullptr;
  int4* d_cols = nullptr;
  struct SizeClass {
    int K;
    int rows_off, rows_cnt, cols_off, cols_cnt;
  };
  std::vector<SizeClass> classes;          // one launch per stage and class
  int4* d_chunks = nullptr;
  int n_chunks = 0;
  pnp::HaarSlice* d_haar = nullptr;       // u[c] -> x, for c = 0 / 1: two tables of B
  int haar_blocks = 0;
  int haar_levels = 0;
  pnp::DevScalars* d_sc = nullptr;
  double* d_parts = nullptr;
  double* d_rho = nullptr;
  float2* d_vecs[11] = {};                // vector kind bases (all slices, grouped by size)
  void* opws = nullptr;                   // gridded-operator workspace (b0), largest slice
  size_t opws_bytes = 0;
};

namespace pnp {

static void launch_stages(pnp_batch* b, const NormalIn* ins, hipStream_t s) {
  for (auto& c : b->classes) batch_rows_fwd(c.K, b->d_sl, ins, b->d_rows + c.rows_off, c.rows_cnt, s);
  for (auto& c : b->classes) batch_cols_toep(c.K, b->d_sl, b->d_cols + c.cols_off, c.cols_cnt, s);
  for (auto& c : b->classes) batch_rows_adj(c.K, b->d_sl, b->d_rows + c.rows_off, c.rows_cnt, s);
}

pnp_batch* batch_create(int B, const pnp_slice* sl, hipStream_t s) {
  if (B < 1 || B > kMaxBatch) fail(PNP_ERR_ARG, "batch size %d outside 1..%d", B, kMaxBatch);
  auto* b = new pnp_batch();
  try {
    b->B = B;
    b->h.resize(B);
    int levels = 0;
    for (int i = 0; i < B; ++i) {
      const pnp_slice& x = sl[i];
      const pnp_plan* p = x.plan;
      if (!p || !x.toeplitz || !x.y || !x.smaps || !x.x_out) fail(PNP_ERR_ARG, "slice %d: missing pointer", i);
      if (x.toeplitz->plan != p) fail(PNP_ERR_ARG, "slice %d: Toeplitz built for another plan", i);
      if (p->ndim != 2 || p->ax[0].n != p->ax[1].n)
        fail(PNP_ERR_UNSUPPORTED, "slice %d: batched slices must be square 2D images", i);
      if (!batch_grid_supported(p->ax[0].K))
        fail(PNP_ERR_UNSUPPORTED, "slice %d: image side %d has no register-FFT grid (n in 64, 96, 128, "
             "256, 320, 384, 512)", i, p->ax[0].n);
      if (x.L < 1) fail(PNP_ERR_ARG, "slice %d: L must be >= 1", i);
      if (!(x.opnorm > 0.0) || !(x.lambda > 0.0)) fail(PNP_ERR_ARG, "slice %d: opnorm and lambda must be > 0", i);
      auto& hh = b->h[i];
      hh.s = x;
      hh.n = p->ax[0].n;
      hh.K = p->ax[0].K;
      hh.G = batch_groups(x.L);
      hh.N = image_size(p);
      const int J = wavelet_default_levels(hh.n);
      if (levels && J != levels) fail(PNP_ERR_UNSUPPORTED, "batched slices need one Haar depth");
      levels = J;
    }
    b->haar_levels = levels;
    // size groups (larger first), memory order = group-major
    std::map<int, std::vector<int>, std::greater<int>> by_n;
    for (int i = 0; i < B; ++i) by_n[b->h[i].n].push_back(i);
    for (auto& kv : by_n) {
      for (int i : kv.second) {
        b->h[i].group = (int)b->groups.size();
        b->order.push_back(i);
      }
      b->groups.push_back(kv);
    }
    // sizes
    long long Ntot = 0, midtot = 0, parttot = 0;
    for (auto& hh : b->h) {
      Ntot += hh.N;
      midtot += (long long)hh.s.L * hh.n * hh.K;
      parttot += (long long)hh.G * hh.N;
    }
    // work items per grid-size class (largest first); within a class the
    // items of one image row (its coil groups) or one strip (its coils) are
    // adjacent
    std::vector<int4> rows, cols, chunks;
    for (auto& g : b->groups) {
      pnp_batch::SizeClass c{b->h[g.second[0]].K, (int)rows.size(), 0, (int)cols.size(), 0};
      for (int i : g.second) {
        const auto& hh = b->h[i];
        for (int iy = 0; iy < hh.n; ++iy)
          for (int gg = 0; gg < hh.G; ++gg) rows.push_back(make_int4(i, iy, gg, 0));
        for (int st = 0; st < hh.K / 8; ++st)
          for (int l = 0; l < hh.s.L; ++l) cols.push_back(make_int4(i, st, l, 0));
      }
      c.rows_cnt = (int)rows.size() - c.rows_off;
      c.cols_cnt = (int)cols.size() - c.cols_off;
      b->classes.push_back(c);
    }
    for (int i = 0; i < B; ++i) {
      const int nch = (int)((b->h[i].N + kChunk - 1) / kChunk);
      if (nch > kRedBlocks) fail(PNP_ERR_SHAPE, "slice %d too large for the batched reductions", i);
      for (int c = 0; c < nch; ++c) chunks.push_back(make_int4(i, c * kChunk, c, nch));
    }
    b->n_chunks = (int)chunks.size();
    // gridded workspace for b0, largest slice
    for (auto& hh : b->h) b->opws_bytes = std::max(b->opws_bytes, op_workspace_bytes(hh.s.plan, hh.s.L));
    // one allocation
    size_t bytes = 0;
    auto add = [&](size_t n) { const size_t o = bytes; bytes += al(n); return o; };
    const size_t o_sl = add(sizeof(BatchSlice) * B), o_vec = add(sizeof(BVec) * B);
    size_t o_in[5];
    for (auto& o : o_in) o = add(sizeof(NormalIn) * B);
    const size_t o_outs = add(sizeof(float2*) * B);
    const size_t o_rows = add(sizeof(int4) * rows.size()), o_cols = add(sizeof(int4) * cols.size());
    const size_t o_ch = add(sizeof(int4) * chunks.size());
    const size_t o_haar = add(sizeof(HaarSlice) * 2 * B);
    const size_t o_sc = add(sizeof(DevScalars) * B);
    const size_t o_parts = add(sizeof(double) * 3 * kRedBlocks * B);
    const size_t o_rho = add(sizeof(double) * (kBatchMaxOuter + 1) * B);
    const size_t o_mid = add(sizeof(float2) * midtot), o_part = add(sizeof(float2) * parttot);
    size_t o_v[11];
    for (auto& o : o_v) o = add(sizeof(float2) * Ntot);
    const size_t o_ws = add(b->opws_bytes);
    PNP_HIP(hipMalloc(&b->block, bytes));
    char* base = static_cast<char*>(b->block);
    b->d_sl = (BatchSlice*)(base + o_sl);
    b->d_vec = (BVec*)(base + o_vec);
    for (int k = 0; k < 5; ++k) b->d_in[k] = (NormalIn*)(base + o_in[k]);
    b->d_outs = (float2**)(base + o_outs);
    b->d_rows = (int4*)(base + o_rows);
    b->d_cols = (int4*)(base + o_cols);
    b->d_chunks = (int4*)(base + o_ch);
    b->d_haar = (HaarSlice*)(base + o_haar);
    b->d_sc = (DevScalars*)(base + o_sc);
    b->d_parts = (double*)(base + o_parts);
    b->d_rho = (double*)(base + o_rho);
    for (int k = 0; k < 11; ++k) b->d_vecs[k] = (float2*)(base + o_v[k]);
    b->opws = base + o_ws;
    // host tables
    std::vector<BatchSlice> hsl(B);
    std::vector<BVec> hv(B);
    std::vector<NormalIn> hin[4];
    for (auto& t : hin) t.resize(B);
    std::vector<HaarSlice> hh2(2 * B);
    long long voff = 0, moff = 0, poff = 0;
    int blk0 = 0;
    const int Bh = 1 << levels;
    for (int pos = 0; pos < B; ++pos) {
      const int i = b->order[pos];
      auto& hh = b->h[i];
      hh.voff = voff;
      float2* mid = (float2*)(base + o_mid) + moff;
      float2* part = (float2*)(base + o_part) + poff;
      hsl[i] = BatchSlice{hh.n, hh.n, hh.K, hh.s.L, hh.N, (const float2*)hh.s.smaps, mid, part,
                          hh.s.toeplitz->T, hh.s.plan->ax[0].fft.tw};
      BVec v{};
      float2* vk[11];
      for (int k = 0; k < 11; ++k) vk[k] = b->d_vecs[k] + voff;
      v.x = vk[0];
      v.b0 = vk[1];
      v.w = vk[2];
      v.u[0] = vk[3];
      v.u[1] = vk[4];
      v.r[0] = vk[5];
      v.r[1] = vk[6];
      v.p[0] = vk[7];
      v.p[1] = vk[8];
      v.s[0] = vk[9];
      v.s[1] = vk[10];
      v.xout = (float2*)hh.s.x_out;
      v.part = part;
      v.G = hh.G;
      v.N = hh.N;
      hv[i] = v;
      DevScalars* sci = b->d_sc + i;
      hin[0][i] = plain_input(v.x);
      hin[1][i] = plain_input(v.r[0]);
      hin[2][i] = NormalIn{nullptr, CGUpdate{v.r[0], v.p[0], v.s[0], v.u[0], v.w, v.r[1], v.p[1], v.s[1], v.u[1],
                                             &sci->alpha, &sci->beta}};
      hin[3][i] = NormalIn{nullptr, CGUpdate{v.r[1], v.p[1], v.s[1], v.u[1], v.w, v.r[0], v.p[0], v.s[0], v.u[0],
                                             &sci->alpha, &sci->beta}};
      const int nb = (hh.n / Bh) * (hh.n / Bh);
      for (int c = 0; c < 2; ++c) hh2[c * B + pos] = HaarSlice{v.u[c], v.x, hh.n, hh.n, blk0};
      blk0 += nb;
      voff += hh.N;
      moff += (long long)hh.s.L * hh.n * hh.K;
      poff += (long long)hh.G * hh.N;
    }
    b->haar_blocks = blk0;
    PNP_HIP(hipMemcpyAsync(b->d_sl, hsl.data(), sizeof(BatchSlice) * B, hipMemcpyHostToDevice, s));
    PNP_HIP(hipMemcpyAsync(b->d_vec, hv.data(), sizeof(BVec) * B, hipMemcpyHostToDevice, s));
    for (int k = 0; k < 4; ++k)
      PNP_HIP(hipMemcpyAsync(b->d_in[k], hin[k].data(), sizeof(NormalIn) * B, hipMemcpyHostToDevice, s));
    PNP_HIP(hipMemcpyAsync(b->d_rows, rows.data(), sizeof(int4) * rows.size(), hipMemcpyHostToDevice, s));
    PNP_HIP(hipMemcpyAsync(b->d_cols, cols.data(), sizeof(int4) * cols.size(), hipMemcpyHostToDevice, s));
    PNP_HIP(hipMemcpyAsync(b->d_chunks, chunks.data(), sizeof(int4) * chunks.size(), hipMemcpyHostToDevice, s));
    PNP_HIP(hipMemcpyAsync(b->d_haar, hh2.data(), sizeof(HaarSlice) * 2 * B, hipMemcpyHostToDevice, s));
    PNP_HIP(hipStreamSynchronize(s));   // host tables go out of scope
  } catch (...) {
    if (b->block) (void)hipFree(b->block);
    delete b;
    throw;
  }
  return b;
}

void batch_destroy(pnp_batch* b) {
  if (!b) return;
  if (b->block) (void)hipFree(b->block);
  delete b;
}

void batch_normal(pnp_batch* b, const float2* const* x, float2* const* out, hipStream_t s) {
  const int B = b->B;
  std::vector<NormalIn> in(B);
  for (int i = 0; i < B; ++i) in[i] = plain_input(x[i]);
  PNP_HIP(hipMemcpyAsync(b->d_in[4], in.data(), sizeof(NormalIn) * B, hipMemcpyHostToDevice, s));
  PNP_HIP(hipMemcpyAsync(b->d_outs, out, sizeof(float2*) * B, hipMemcpyHostToDevice, s));
  launch_stages(b, b->d_in[4], s);
  PNP_LAUNCH(k_bcopy, dim3(b->n_chunks), dim3(kRedThreads), 0, s, b->d_chunks, b->d_vec, 2,
             (float2* const*)b->d_outs);
  PNP_HIP(hipStreamSynchronize(s));   // the host input tables above
}

// One batched UNet forward per image size: out = D(u) for u, out laid out
// group-contiguous (the batch's memory order).
static void batch_unet_prior(pnp_batch* b, const pnp_prior* prior, int cur, double sigma, void* ws,
                             hipStream_t s) {
  long long off = 0;
  for (auto& g : b->groups) {
    const int n = g.first, cnt = (int)g.second.size();
    const float2* u = b->d_vecs[3 + cur] + off;   // u[cur] kind base
    float2* x = b->d_vecs[0] + off;
    unet_forward(prior->net, u, nullptr, (float)(prior->kappa * sigma), cnt, n, n, x, ws, s);
    off += (long long)cnt * n * n;
  }
}

size_t batch_unet_ws_bytes(const pnp_batch* b) {
  size_t m = 0;
  for (auto& g : b->groups) m = std::max(m, unet_ws_bytes((int)g.second.size(), g.first, g.first, false));
  return m;
}

void batch_hqs_solve(pnp_batch* b, const pnp_prior* prior, const double* sigmas, int n_out, int precond, int n_cg,
                     void* unet_ws, double* rho_host, int* bad_host, hipStream_t s) {
  if (n_out > kBatchMaxOuter) fail(PNP_ERR_SHAPE, "n_out %d exceeds %d", n_out, kBatchMaxOuter);
  const int B = b->B;
  static const double c0s[3] = {1.0, 2.0, 4.0};
  static const double c1s[3] = {0.0, 1.0, 10.0 / 3.0};
  const double c0 = c0s[precond];
  PNP_LAUNCH(k_binit_scalars, dim3(1), dim3(kMaxBatch), 0, s, b->d_sc, B);
  // b0 = A^H D_w y and ||y||_w^2 per slice (gridded adjoint)
  for (int i = 0; i < B; ++i) {
    const auto& hh = b->h[i];
    OpWorkspace w = op_workspace(hh.s.plan, hh.s.L, b->opws);
    op_adjoint(hh.s.plan, (const float2*)hh.s.y, (const float2*)hh.s.smaps, hh.s.L, hh.s.dcf,
               b->d_vecs[1] + hh.voff, w, s);
    PNP_LAUNCH(k_bwnorm, dim3(64), dim3(kRedThreads), 0, s, (long long)hh.s.plan->M, hh.s.L,
               (const float2*)hh.s.y, hh.s.dcf, b->d_parts + (long long)i * kRedBlocks * 3, b->d_sc + i);
  }
  const dim3 gch(b->n_chunks), bch(kRedThreads);
  PNP_LAUNCH(k_bcopy, gch, bch, 0, s, b->d_chunks, b->d_vec, 0, (float2* const*)nullptr);
  SliceCoef co{};
  for (int k = 0; k < n_out; ++k) {
    for (int i = 0; i < B; ++i) {
      const double gamma = b->h[i].s.lambda * sigmas[k];
      co.gamma[i] = (float)gamma;
      co.cg[i] = (float)(gamma - c1s[precond] / b->h[i].s.opnorm);
    }
    launch_stages(b, b->d_in[0], s);   // N x
    PNP_LAUNCH(k_bcg_init, gch, bch, 0, s, b->d_chunks, b->d_vec, co, b->d_parts);
    PNP_LAUNCH(k_bcg_init_fin, dim3(B), dim3(kFinThreads), 0, s, b->d_vec, b->d_parts, b->d_sc, b->d_rho, k);
    int c = 0;
    for (int j = 0; j < n_cg; ++j) {
      const NormalIn* ins = b->d_in[1];
      if (j > 0) {
        ins = b->d_in[c == 0 ? 2 : 3];
        c = 1 - c;
      }
      launch_stages(b, ins, s);
      PNP_LAUNCH(k_bcg_dots, gch, bch, 0, s, b->d_chunks, b->d_vec, co, (float)c0, c, b->d_parts);
      PNP_LAUNCH(k_bcg_dots_fin, dim3(B), dim3(kFinThreads), 0, s, b->d_vec, b->d_parts, j == 0 ? 1 : 0, b->d_sc);
    }
    PNP_LAUNCH(k_bcg_final, gch, bch, 0, s, b->d_chunks, b->d_vec, c, (const DevScalars*)b->d_sc);
    const int cur = 1 - c;               // the prox result u lives in set cur
    if (prior->kind == 1) {
      batch_unet_prior(b, prior, cur, sigmas[k], unet_ws, s);
    } else {
      const int J = prior->levels > 0 ? prior->levels : b->haar_levels;
      if (J != b->haar_levels) fail(PNP_ERR_UNSUPPORTED, "batched Haar prior uses %d levels", b->haar_levels);
      wavelet_apply_batched(b->d_haar + cur * B, B, b->haar_blocks, J, (float)(prior->kappa * sigmas[k]), s);
    }
  }
  if (rho_host) {
    SliceCoef zero{};
    launch_stages(b, b->d_in[0], s);
    PNP_LAUNCH(k_bcg_init, gch, bch, 0, s, b->d_chunks, b->d_vec, zero, b->d_parts);
    PNP_LAUNCH(k_bcg_init_fin, dim3(B), dim3(kFinThreads), 0, s, b->d_vec, b->d_parts, b->d_sc, b->d_rho, n_out);
  }
  PNP_LAUNCH(k_bcopy, gch, bch, 0, s, b->d_chunks, b->d_vec, 1, (float2* const*)nullptr);
  if (rho_host || bad_host) {
    std::vector<double> r((size_t)B * (kBatchMaxOuter + 1));
    std::vector<DevScalars> hs(B);
    PNP_HIP(hipMemcpyAsync(r.data(), b->d_rho, sizeof(double) * r.size(), hipMemcpyDeviceToHost, s));
    PNP_HIP(hipMemcpyAsync(hs.data(), b->d_sc, sizeof(DevScalars) * B, hipMemcpyDeviceToHost, s));
    PNP_HIP(hipStreamSynchronize(s));
    if (rho_host)
      for (int i = 0; i < B; ++i)
        for (int k = 0; k < n_out; ++k) rho_host[(long long)i * n_out + k] = r[(long long)i * (kBatchMaxOuter + 1) + k + 1];
    if (bad_host) {
      *bad_host = 0;
      for (int i = 0; i < B; ++i) *bad_host |= hs[i].bad;
    }
  }
}

}  // namespace pnp
