// Conjugate-gradient proximal step, power iteration and the annealed
// PnP-HQS loop (Sec. 3.3-3.4), with every scalar kept on the device.
//
// Vectors are complex64; inner products, step sizes (alpha, beta), the
// residual norms and the data-consistency residual are accumulated in FP64.
// Each reduction kernel writes one FP64 partial per block; the last block to
// finish (atomic ticket) sums the partials in a fixed order and updates the
// scalar state, so results are deterministic, there is no separate
// finalisation launch and no host round trip inside the loop.
//
// The prox system (Sec. 3.4, read with the density weighting D_w):
//   M u = b,  M = gamma N + P = c0 I + (gamma - c1 alpha) N,  N = A^H D_w A,
//   b = P x + gamma b0,  b0 = A^H D_w y,  started at u = x so that
//   r0 = gamma (b0 - N x).  CG runs in the Chronopoulos-Gear arrangement
//   (same iterates as the textbook recurrence in exact arithmetic): with
//   w = M r, both inner products <r,r> and <w,r> of a step are reduced in
//   one pass, and the vector updates
//     p = r + beta p, s = w + beta s, u = u + alpha p, r = r - alpha s
//   are formed inside the next normal operator's first pass, so a step is
//   one normal operator plus one reduction kernel.
// The residual rho(x) = ||D_w^{1/2}(A x - y)||^2 = <x,Nx> - 2 Re<x,b0> + ||y||_w^2
// comes for free from the N x that r0 needs.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cg_scalars.hpp"
#include "common.hpp"
#include "trace.hpp"

namespace pnp {

constexpr int kMaxOuter = 1024;


namespace {

__device__ __forceinline__ double re_dot(float2 a, float2 b) {
  return (double)a.x * b.x + (double)a.y * b.y;
}

__device__ __forceinline__ float2 sum_groups(const float2* __restrict__ part, int G, long long N,
                                             long long i) {
  float2 v = part[i];
  for (int g = 1; g < G; ++g) v = cadd(v, part[(long long)g * N + i]);
  return v;
}

__global__ void k_init_scalars(DevScalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->rr = sc->pq = sc->alpha = sc->beta = sc->yw2 = sc->lam = sc->inv = 0.0;
    sc->bad = 0;
    sc->cnt = 0u;
    sc->bad_saved = 0;
  }
}

__global__ void k_copy(long long N, const float2* __restrict__ a, float2* __restrict__ b) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Nx = sum of the normal operator's partial images; u = x; r = gamma (b0 - Nx);
// p = s = 0; block sums of <r,r>, <x,Nx>, Re<x,b0> (k_cg_init_fin: rr = <r,r>,
// rho(x) = <x,Nx> - 2 Re<x,b0> + ||y||_w^2).
__global__ void __launch_bounds__(kRedThreads)
k_cg_init(long long N, int G, const float2* __restrict__ x, const float2* __restrict__ part,
          const float2* __restrict__ b0, float gamma, float2* __restrict__ u, float2* __restrict__ r,
          float2* __restrict__ p, float2* __restrict__ sv, double* __restrict__ parts) {
  double acc[3] = {0.0, 0.0, 0.0};
  const float2 z = make_float2(0.f, 0.f);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 xv = x[i], nv = sum_groups(part, G, N, i), bv = b0[i];
    const float2 rv = make_float2(gamma * (bv.x - nv.x), gamma * (bv.y - nv.y));
    u[i] = xv;
    r[i] = rv;
    p[i] = z;
    sv[i] = z;
    acc[0] += re_dot(rv, rv);
    acc[1] += re_dot(xv, nv);
    acc[2] += re_dot(xv, bv);
  }
  block_parts<3>(acc, parts, blockIdx.x);
}

// one workgroup: the three sums of k_cg_init -> rr and rho.  The breakdown
// flag is saved (restore == 0) or put back to the saved value (restore != 0:
// a CG queued after the previous start is being discarded).
__global__ void __launch_bounds__(kFinThreads)
k_cg_init_fin(const double* __restrict__ parts, int nblocks, DevScalars* sc, double* rho_out, int restore) {
  double s[3];
  sum_parts<3>(parts, nblocks, s);
  if (threadIdx.x == 0) {
    if (restore)
      sc->bad = sc->bad_saved;
    else
      sc->bad_saved = sc->bad;
    cg_finish_init(sc, s[0], s[1], s[2], rho_out);
  }
}

// w = c0 r + cg N r, block sums of g = <r,r> and d = Re<w,r> (turned into
// the step sizes by the pass that uses them: cg_finish_deferred)
__global__ void __launch_bounds__(kRedThreads)
k_cg_dots(long long N, int G, const float2* __restrict__ r, const float2* __restrict__ part, float c0,
          float cg, float2* __restrict__ w, double* __restrict__ parts) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 rv = r[i], nv = sum_groups(part, G, N, i);
    const float2 wv = make_float2(c0 * rv.x + cg * nv.x, c0 * rv.y + cg * nv.y);
    w[i] = wv;
    acc[0] += re_dot(rv, rv);
    acc[1] += re_dot(wv, rv);
  }
  block_parts<2>(acc, parts, blockIdx.x);
}

// Last CG step: p = r + beta p, u = u + alpha p (writes u2), with alpha and
// beta of the last step formed here from its block sums.
__global__ void k_cg_final(long long N, const float2* __restrict__ r, const float2* __restrict__ p,
                           const float2* __restrict__ u, float2* __restrict__ u2, CGFinish fin) {
  const CgStep st = cg_finish_deferred(fin);
  const float a = (float)st.alpha, b = (float)st.beta;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 rv = r[i], pv = p[i], uv = u[i];
    const float2 pn = make_float2(fmaf(b, pv.x, rv.x), fmaf(b, pv.y, rv.y));
    u2[i] = make_float2(fmaf(a, pn.x, uv.x), fmaf(a, pn.y, uv.y));
  }
}

// ||y||_w^2 over L*M entries
__global__ void __launch_bounds__(kRedThreads)
k_wnorm(long long M, int L, const float2* __restrict__ y, const float* __restrict__ dcf,
        double* __restrict__ parts, DevScalars* sc) {
  double acc[1] = {0.0};
  const long long T = M * L;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T;
       t += (long long)gridDim.x * blockDim.x) {
    const long long m = t % M;
    const float2 v = y[t];
    const double w = dcf ? (double)dcf[m] : 1.0;
    acc[0] += w * re_dot(v, v);
  }
  double s[1];
  if (reduce_last<1>(acc, parts, &sc->cnt, s) && threadIdx.x == 0) sc->yw2 = s[0];
}

// ---- power iteration
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // splitmix64 finaliser (Steele, Lea, Flood 2014)
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_randn(long long N, uint64_t seed, float2* __restrict__ v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const uint64_t h1 = mix64(seed ^ mix64((uint64_t)i * 2));
    const uint64_t h2 = mix64(seed ^ mix64((uint64_t)i * 2 + 1));
    const double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    v[i] = make_float2((float)(rad * cs), (float)(rad * sn));
  }
}

// w = sum of partial images (or w itself when part == nullptr);
// last block: lam = Re<v, w>, inv = 1/||w||
__global__ void __launch_bounds__(kRedThreads)
k_pow_dot(long long N, int G, const float2* __restrict__ v, const float2* __restrict__ part,
          float2* __restrict__ w, double* __restrict__ parts, DevScalars* sc) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 b = part ? sum_groups(part, G, N, i) : w[i];
    if (part) w[i] = b;
    acc[0] += v ? re_dot(v[i], b) : 0.0;
    acc[1] += re_dot(b, b);
  }
  double s[2];
  if (reduce_last<2>(acc, parts, &sc->cnt, s) && threadIdx.x == 0) {
    sc->lam = s[0];
    sc->inv = s[1] > 0.0 ? 1.0 / sqrt(s[1]) : 0.0;
  }
}

__global__ void k_scale_into(long long N, const float2* __restrict__ w, const DevScalars* __restrict__ sc,
                             float2* __restrict__ v) {
  const float s = (float)sc->inv;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    v[i] = cscale(w[i], s);
}

// ---- PnP-PGD and FISTA vector steps
// PnP-PGD with P = Id: u = x - gc0 (N x - b0), N x the sum of the partials
__global__ void k_pgd_id(long long N, int G, const float2* __restrict__ x, const float2* __restrict__ part,
                         const float2* __restrict__ b0, float gc0, float2* __restrict__ u) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 xv = x[i], nv = sum_groups(part, G, N, i), bv = b0[i];
    u[i] = make_float2(xv.x - gc0 * (nv.x - bv.x), xv.y - gc0 * (nv.y - bv.y));
  }
}

// g = N x - b0 (the data-term gradient)
__global__ void k_grad(long long N, int G, const float2* __restrict__ part, const float2* __restrict__ b0,
                       float2* __restrict__ g) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 nv = sum_groups(part, G, N, i), bv = b0[i];
    g[i] = make_float2(nv.x - bv.x, nv.y - bv.y);
  }
}

// preconditioned step: u = x - gamma P g = x - gc0 g + gc1a N g
__global__ void k_pgd_step(long long N, int G, const float2* __restrict__ x, const float2* __restrict__ g,
                           const float2* __restrict__ part, float gc0, float gc1a, float2* __restrict__ u) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 xv = x[i], gv = g[i], nv = sum_groups(part, G, N, i);
    u[i] = make_float2(xv.x - gc0 * gv.x + gc1a * nv.x, xv.y - gc0 * gv.y + gc1a * nv.y);
  }
}

// FISTA: z_k, x_{k-1} -> x_k (v = z - gamma (N z - b0) first, then the
// wavelet prox) -> z_{k+1} = x_k + beta (x_k - x_{k-1}); x_{k-1} <- x_k
__global__ void k_fista_mom(long long N, const float2* __restrict__ x, float2* __restrict__ xp, float beta,
                            float2* __restrict__ z) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 xv = x[i], pv = xp[i];
    z[i] = make_float2(fmaf(beta, xv.x - pv.x, xv.x), fmaf(beta, xv.y - pv.y, xv.y));
    xp[i] = xv;
  }
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

unsigned vec_blocks(long long N) {
  long long b = (N + kRedThreads - 1) / kRedThreads;
  return (unsigned)std::min<long long>(std::max<long long>(b, 1), kRedBlocks);
}

}  // namespace

// ------------------------------------------------------------ host side
struct SolverWs {
  OpWorkspace op;
  float2 *b0, *Nv, *w;
  float2 *u[2], *r[2], *p[2], *s[2];   // CG vectors, double-buffered
  double* parts;
  DevScalars* sc;
  DevScalars* cgs;   // [2] CG step state, alternating between steps
  double* rho;   // [kMaxOuter + 1]
  double* fparts[2];   // CG inner products formed by the row passes (FusedDots), by step parity
};

// slots of one FusedDots set: image rows x coil groups; 2D only
static long long fused_slots(const pnp_plan* p, int L) {
  return p->ndim == 2 ? (long long)p->ax[1].n * op_groups_max(L) : 0;
}

size_t hqs_workspace_bytes(const pnp_plan* p, int L) {
  const int64_t N = image_size(p);
  size_t b = al(op_workspace_bytes(p, L));
  b += 11 * al(sizeof(float2) * N);
  b += al(sizeof(double) * 4 * kRedBlocks);
  b += al(sizeof(DevScalars) * 3);
  b += al(sizeof(double) * (kMaxOuter + 1));
  b += 2 * al(sizeof(double) * 2 * (size_t)std::max<long long>(1, fused_slots(p, L)));
  return b;
}

static SolverWs solver_ws(const pnp_plan* p, int L, void* ws) {
  SolverWs w;
  const int64_t N = image_size(p);
  char* c = (char*)ws;
  w.op = op_workspace(p, L, c);
  c += al(op_workspace_bytes(p, L));
  float2** vecs[11] = {&w.b0, &w.Nv, &w.w, &w.u[0], &w.u[1], &w.r[0], &w.r[1], &w.p[0], &w.p[1],
                        &w.s[0], &w.s[1]};
  for (auto v : vecs) {
    *v = (float2*)c;
    c += al(sizeof(float2) * N);
  }
  w.parts = (double*)c;
  c += al(sizeof(double) * 4 * kRedBlocks);
  w.sc = (DevScalars*)c;
  w.cgs = w.sc + 1;
  c += al(sizeof(DevScalars) * 3);
  w.rho = (double*)c;
  c += al(sizeof(double) * (kMaxOuter + 1));
  for (int i = 0; i < 2; ++i) {
    w.fparts[i] = (double*)c;
    c += al(sizeof(double) * 2 * (size_t)std::max<long long>(1, fused_slots(p, L)));
  }
  return w;
}

size_t opnorm_workspace_bytes(const pnp_plan* p, int L) { return hqs_workspace_bytes(p, L); }

// Power iteration: v <- N v / ||N v||, `iters` times; returns the last
// Rayleigh quotient Re<v, N v> (|v| = 1).  Synchronises the stream.
// Normal operator with the result left as coil-group partial images: the
// Toeplitz embedding when given, else the gridded operator.
static void normal_parts(const pnp_plan* p, const pnp_toeplitz* tp, const NormalIn& in,
                         const float2* smaps, int L, const float* dcf, const OpWorkspace& w,
                         hipStream_t s) {
  if (tp)
    op_normal_toep_parts(tp, in, smaps, L, w, s);
  else
    op_normal_parts(p, in, smaps, L, dcf, w, s);   // gridded
}

double power_iteration(const pnp_plan* p, const pnp_toeplitz* tp, const float2* smaps, int L,
                       const float* dcf, int iters, uint64_t seed, void* ws, hipStream_t s) {
  SolverWs w = solver_ws(p, L, ws);
  const long long N = image_size(p);
  const int G = op_groups(p, L);
  const unsigned nb = vec_blocks(N);
  float2* v = w.u[0];
  PNP_LAUNCH(k_init_scalars, dim3(1), dim3(64), 0, s, w.sc);
  PNP_LAUNCH(k_randn, dim3(nb), dim3(kRedThreads), 0, s, N, seed, w.Nv);
  PNP_LAUNCH(k_pow_dot, dim3(nb), dim3(kRedThreads), 0, s, N, G, (const float2*)nullptr,
             (const float2*)nullptr, w.Nv, w.parts, w.sc);
  PNP_LAUNCH(k_scale_into, dim3(nb), dim3(kRedThreads), 0, s, N, w.Nv, w.sc, v);
  for (int it = 0; it < iters; ++it) {
    normal_parts(p, tp, plain_input(v), smaps, L, dcf, w.op, s);
    PNP_LAUNCH(k_pow_dot, dim3(nb), dim3(kRedThreads), 0, s, N, G, v, w.op.part, w.Nv, w.parts, w.sc);
    PNP_LAUNCH(k_scale_into, dim3(nb), dim3(kRedThreads), 0, s, N, w.Nv, w.sc, v);
  }
  DevScalars h;
  PNP_HIP(hipMemcpyAsync(&h, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  PNP_HIP(hipStreamSynchronize(s));
  return h.lam;
}

void prior_apply(const pnp_prior* prior, int ndim, const int* n, const float2* u, float2* x, double sigma,
                 hipStream_t s) {
  if (prior->kind == 1) {
    const int B = ndim == 3 ? n[2] : 1;
    if (B != prior->batch || n[1] != prior->ny || n[0] != prior->nx)
      fail(PNP_ERR_SHAPE, "UNet prior was created for %d x %d x %d images, not %d x %d x %d", prior->batch,
           prior->ny, prior->nx, B, n[1], n[0]);
    if (u == x) fail(PNP_ERR_ARG, "the UNet prior cannot run in place");
    unet_forward(prior->net, u, nullptr, (float)(prior->kappa * sigma), B, n[1], n[0], x, prior->ws, s);
    return;
  }
  int nmin = n[0];
  for (int a = 1; a < ndim; ++a) nmin = std::min(nmin, n[a]);
  const int J = prior->levels > 0 ? prior->levels : wavelet_default_levels(nmin);
  wavelet_apply(ndim, n, J, (float)(prior->kappa * sigma), u, x, s);
}

// The wavelet prior applied to the last CG update u + alpha (r + beta p)
static void prior_apply_cg(const pnp_prior* prior, int ndim, const int* n, const float2* r, const float2* pv,
                           const float2* u, const CGFinish& fin, float2* x, double sigma, hipStream_t s) {
  int nmin = n[0];
  for (int a = 1; a < ndim; ++a) nmin = std::min(nmin, n[a]);
  const int J = prior->levels > 0 ? prior->levels : wavelet_default_levels(nmin);
  wavelet_apply_cg(ndim, n, J, (float)(prior->kappa * sigma), r, pv, u, fin, x, s);
}

// Pinned host copies of the residuals read by the prior check: one buffer
// per host thread, allocated on first use and kept for the thread's
// lifetime (a solve reads its values before it returns).
static double* pinned_residuals() {
  static thread_local double* buf = nullptr;
  if (!buf) PNP_HIP(hipHostMalloc((void**)&buf, sizeof(double) * (kMaxOuter + 1), hipHostMallocDefault));
  return buf;
}

struct EventHandle {
  hipEvent_t e = nullptr;
  EventHandle() = default;
  EventHandle(const EventHandle&) = delete;
  EventHandle& operator=(const EventHandle&) = delete;
  ~EventHandle() {
    if (e) (void)hipEventDestroy(e);
  }
};

void hqs_solve(const pnp_plan* p, const HQSArgs& a, void* ws, hipStream_t s, double* rho_host,
               int* bad_host, int* fb_host) {
  if (a.n_out > kMaxOuter) fail(PNP_ERR_SHAPE, "n_out %d exceeds %d", a.n_out, kMaxOuter);
  SolverWs w = solver_ws(p, a.L, ws);
  const long long N = image_size(p);
  const int G = op_groups(p, a.L);
  const unsigned nb = vec_blocks(N);
  static const double c0s[3] = {1.0, 2.0, 4.0};
  static const double c1s[3] = {0.0, 1.0, 10.0 / 3.0};
  const double c0 = c0s[a.precond];
  const double c1a = c1s[a.precond] / a.opnorm;

  PNP_LAUNCH(k_init_scalars, dim3(1), dim3(64), 0, s, w.sc);
  // b0 = A^H D_w y, ||y||_w^2
  op_adjoint(p, a.y, a.smaps, a.L, a.dcf, w.b0, w.op, s);
  {
    const long long T = p->M * a.L;
    const unsigned nbk =
        (unsigned)std::max<long long>(1, std::min<long long>((T + kRedThreads - 1) / kRedThreads, kRedBlocks));
    PNP_LAUNCH(k_wnorm, dim3(nbk), dim3(kRedThreads), 0, s, (long long)p->M, a.L, a.y, a.dcf, w.parts,
               w.sc);
  }
  float2* x = a.x_out;
  PNP_LAUNCH(k_copy, dim3(nb), dim3(kRedThreads), 0, s, N, a.x0 ? a.x0 : w.b0, x);

  const int nd[3] = {p->ax[0].n, p->ax[1].n, p->ax[2].n};
  // A prior with a fallback is checked after every outer iteration: when the
  // new image is not finite or its residual rho_k exceeds (1 + rise_tol)
  // rho_{k-1}, it is replaced by the fallback prior's output.  The host
  // reads rho from pinned memory while the GPU already runs the next
  // iteration's CG, queued on the guess that the image is kept (that CG
  // writes only its own vectors, so a rejection discards it and starts the
  // CG again from the fallback image).  The normal operator of the accepted
  // image is reused by the next iteration's CG start.
  const bool guard = a.prior->fallback != nullptr;
  bool started = false;   // N x and the CG start of iteration k already done
  double rho_prev = 0.0;
  if (fb_host)
    for (int k = 0; k < a.n_out; ++k) fb_host[k] = 0;
  double* rho_pin = guard ? pinned_residuals() : nullptr;
  EventHandle ev;
  if (guard) PNP_HIP(hipEventCreateWithFlags(&ev.e, hipEventDisableTiming));
  // rho_i to the pinned copy, then the event the host waits on
  auto post_rho = [&](int i) {
    PNP_HIP(hipMemcpyAsync(rho_pin + i, w.rho + i, sizeof(double), hipMemcpyDeviceToHost, s));
    PNP_HIP(hipEventRecord(ev.e, s));
  };
  // N x, then the CG start in set 0: u = x, r = gamma (b0 - N x), p = s = 0.
  // Its sums only form rho_k (the CG steps keep their own state), so their
  // finisher runs only when rho is read: by the check or the report.
  // Without rho the start's vectors are formed by the first CG step's first
  // pass instead (CGUpdate::b0), with the same arithmetic.
  const bool want_rho = guard || rho_host != nullptr;
  double start_gamma = 0.0;
  auto cg_start = [&](double gamma, double* rho_out, int restore_bad) {
    normal_parts(p, a.toep, plain_input(x), a.smaps, a.L, a.dcf, w.op, s);
    if (!want_rho) {
      start_gamma = gamma;
      return;
    }
    PNP_LAUNCH(k_cg_init, dim3(nb), dim3(kRedThreads), 0, s, N, G, x, w.op.part, w.b0, (float)gamma, w.u[0],
               w.r[0], w.p[0], w.s[0], w.parts);
    if (want_rho)
      PNP_LAUNCH(k_cg_init_fin, dim3(1), dim3(kFinThreads), 0, s, w.parts, (int)nb, w.sc, rho_out, restore_bad);
  };
  // step 0: w = M r0; steps 1..n_cg-1: update (p, s, u, r) inside the
  // operator's first pass, w = M r; then the last u update.  The step sizes
  // of step j are formed by the pass that uses them (the first pass of step
  // j + 1, or the last update) from step j's block sums; step j's state goes
  // to cgs[j % 2], the previous step's is read from the other.
  // On the 2D register-FFT Toeplitz operator the row passes form the sums
  // (FusedDots, by step parity) and the next pass forms w = c0 r + cg N r
  // from the coil-group partial images; elsewhere k_cg_dots does both.
  const bool fused = toep_fused_dots(a.toep);
  const int ny = p->ax[1].n;
  auto cg_of = [&](int k) { return (float)(a.lambda * a.sigmas[k] - c1a); };
  auto fin_of = [&](int k, int j) {
    CGFinish f{w.parts, (int)nb, j == 0 ? 1 : 0, w.cgs + ((j + 1) & 1), w.cgs + (j & 1), &w.sc->bad};
    if (fused) {
      f.parts = w.fparts[j & 1];
      f.nparts = ny * G;
      f.fused = 1;
      f.c0 = (float)c0;
      f.cg = cg_of(k);
    }
    return f;
  };
  // the n_cg CG steps of outer iteration k from the CG start in set 0;
  // returns c, the set that holds the last step's (r, p, u); with `final`,
  // the last u update is made into w.u[1 - c]
  auto cg_solve = [&](int k, bool final) -> int {
    const float cg = cg_of(k);
    int c = 0;
    for (int j = 0; j < a.n_cg; ++j) {
      NormalIn in = plain_input(w.r[0]);
      if (j == 0 && !want_rho) {
        in.cg.u = x;
        in.cg.b0 = w.b0;
        in.cg.gamma = (float)start_gamma;
        in.cg.part = w.op.part;
        in.cg.G = G;
        in.cg.N = N;
        in.cg.r2 = w.r[0];
        in.cg.p2 = w.p[0];
        in.cg.s2 = w.s[0];
        in.cg.u2 = w.u[0];
      }
      if (j > 0) {
        in.x = nullptr;
        in.cg = CGUpdate{w.r[c], w.p[c], w.s[c], w.u[c], w.w, w.r[1 - c], w.p[1 - c], w.s[1 - c], w.u[1 - c],
                         nullptr, nullptr, fin_of(k, j - 1)};
        if (fused) {
          in.cg.w = nullptr;
          in.cg.part = w.op.part;
          in.cg.G = G;
          in.cg.N = N;
          in.cg.c0 = (float)c0;
          in.cg.cg = cg;
        }
        c = 1 - c;
      }
      if (fused) {
        in.fd = FusedDots{w.fparts[j & 1], w.r[c], ny};
        normal_parts(p, a.toep, in, a.smaps, a.L, a.dcf, w.op, s);
        continue;
      }
      normal_parts(p, a.toep, in, a.smaps, a.L, a.dcf, w.op, s);
      PNP_LAUNCH(k_cg_dots, dim3(nb), dim3(kRedThreads), 0, s, N, G, w.r[c], w.op.part, (float)c0, cg, w.w,
                 w.parts);
    }
    if (final)
      PNP_LAUNCH(k_cg_final, dim3(nb), dim3(kRedThreads), 0, s, N, w.r[c], w.p[c], w.u[c], w.u[1 - c],
                 fin_of(k, a.n_cg - 1));
    return c;
  };
  // a wavelet prior without a check forms the last u update while it loads
  // its blocks (no separate update pass)
  const bool fuse_final = !guard && a.prior->kind == 0;

  float2* u_next = nullptr;   // iteration k's CG, queued by iteration k - 1's check
  for (int k = 0; k < a.n_out; ++k) {
    if (!started) cg_start(a.lambda * a.sigmas[k], w.rho + k, 0);
    started = false;
    if (guard && k == 0) post_rho(0);
    if (fuse_final) {
      const int c = cg_solve(k, false);
      prior_apply_cg(a.prior, p->ndim, nd, w.r[c], w.p[c], w.u[c], fin_of(k, a.n_cg - 1), x, a.sigmas[k], s);
      continue;
    }
    float2* u_res = u_next;
    if (!u_res) u_res = w.u[1 - cg_solve(k, true)];
    u_next = nullptr;
    prior_apply(a.prior, p->ndim, nd, u_res, x, a.sigmas[k], s);
    if (!guard) continue;
    // candidate from the fallback, kept in Nv (free during the solve)
    prior_apply(a.prior->fallback, p->ndim, nd, u_res, w.Nv, a.sigmas[k], s);
    const double gnext = k + 1 < a.n_out ? a.lambda * a.sigmas[k + 1] : 0.0;
    cg_start(gnext, w.rho + k + 1, 0);
    post_rho(k + 1);
    if (k + 1 < a.n_out) u_next = w.u[1 - cg_solve(k + 1, true)];
    PNP_HIP(hipEventSynchronize(ev.e));   // rho_0 .. rho_{k+1} are in the pinned copy
    if (k == 0) rho_prev = rho_pin[0];
    double rho = rho_pin[k + 1];
    if (!(rho <= (1.0 + a.rise_tol) * rho_prev)) {
      PNP_LAUNCH(k_copy, dim3(nb), dim3(kRedThreads), 0, s, N, w.Nv, x);
      cg_start(gnext, w.rho + k + 1, 1);
      post_rho(k + 1);
      if (k + 1 < a.n_out) u_next = w.u[1 - cg_solve(k + 1, true)];
      PNP_HIP(hipEventSynchronize(ev.e));
      rho = rho_pin[k + 1];
      if (fb_host) fb_host[k] = 1;
    }
    rho_prev = rho;
    started = true;
  }
  if (rho_host) {
    // residual of the final image (one extra normal operator, unless the
    // check of the last iteration has formed it already)
    if (!started) cg_start(0.0, w.rho + a.n_out, 0);
    std::vector<double> r(a.n_out + 1);
    DevScalars h;
    PNP_HIP(hipMemcpyAsync(r.data(), w.rho, sizeof(double) * (a.n_out + 1), hipMemcpyDeviceToHost, s));
    PNP_HIP(hipMemcpyAsync(&h, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    PNP_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < a.n_out; ++k) rho_host[k] = r[k + 1];
    if (bad_host) *bad_host = h.bad;
  }
}

// b0 = A^H D_w y into w.b0, x = x0 (or b0) into x
static void start_from_data(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf,
                            const float2* x0, float2* x, const SolverWs& w, hipStream_t s) {
  const long long N = image_size(p);
  op_adjoint(p, y, smaps, L, dcf, w.b0, w.op, s);
  PNP_LAUNCH(k_copy, dim3(vec_blocks(N)), dim3(kRedThreads), 0, s, N, x0 ? x0 : w.b0, x);
}

void pgd_solve(const pnp_plan* p, const PGDArgs& a, void* ws, hipStream_t s) {
  SolverWs w = solver_ws(p, a.L, ws);
  const long long N = image_size(p);
  const int G = op_groups(p, a.L);
  const unsigned nb = vec_blocks(N);
  static const double c0s[3] = {1.0, 2.0, 4.0};
  static const double c1s[3] = {0.0, 1.0, 10.0 / 3.0};
  const float gc0 = (float)(a.gamma * c0s[a.precond]);
  const float gc1a = (float)(a.gamma * c1s[a.precond] / a.opnorm);
  float2* x = a.x_out;
  start_from_data(p, a.y, a.smaps, a.L, a.dcf, a.x0, x, w, s);
  const int nd[3] = {p->ax[0].n, p->ax[1].n, p->ax[2].n};
  float2* u = w.u[0];
  float2* g = w.r[0];
  for (int k = 0; k < a.n_iter; ++k) {
    normal_parts(p, a.toep, plain_input(x), a.smaps, a.L, a.dcf, w.op, s);
    if (a.precond == 0) {
      PNP_LAUNCH(k_pgd_id, dim3(nb), dim3(kRedThreads), 0, s, N, G, x, w.op.part, w.b0, gc0, u);
    } else {
      PNP_LAUNCH(k_grad, dim3(nb), dim3(kRedThreads), 0, s, N, G, w.op.part, w.b0, g);
      normal_parts(p, a.toep, plain_input(g), a.smaps, a.L, a.dcf, w.op, s);
      PNP_LAUNCH(k_pgd_step, dim3(nb), dim3(kRedThreads), 0, s, N, G, x, g, w.op.part, gc0, gc1a, u);
    }
    prior_apply(a.prior, p->ndim, nd, u, x, a.sigmas[k], s);
  }
}

void fista_wavelet(const pnp_plan* p, const FISTAArgs& a, void* ws, hipStream_t s) {
  SolverWs w = solver_ws(p, a.L, ws);
  const long long N = image_size(p);
  const int G = op_groups(p, a.L);
  const unsigned nb = vec_blocks(N);
  float2* x = a.x_out;
  start_from_data(p, a.y, a.smaps, a.L, a.dcf, a.x0, x, w, s);
  float2* xp = w.u[1];
  float2* z = w.p[0];
  float2* v = w.r[0];
  PNP_LAUNCH(k_copy, dim3(nb), dim3(kRedThreads), 0, s, N, x, xp);
  PNP_LAUNCH(k_copy, dim3(nb), dim3(kRedThreads), 0, s, N, x, z);
  const int nd[3] = {p->ax[0].n, p->ax[1].n, p->ax[2].n};
  int nmin = nd[0];
  for (int d = 1; d < p->ndim; ++d) nmin = std::min(nmin, nd[d]);
  const int J = a.levels > 0 ? a.levels : wavelet_default_levels(nmin);
  const float tau = (float)(a.gamma * a.lam);
  double t = 1.0;
  for (int k = 0; k < a.n_iter; ++k) {
    normal_parts(p, a.toep, plain_input(z), a.smaps, a.L, a.dcf, w.op, s);
    PNP_LAUNCH(k_pgd_id, dim3(nb), dim3(kRedThreads), 0, s, N, G, z, w.op.part, w.b0, (float)a.gamma, v);
    wavelet_apply(p->ndim, nd, J, tau, v, x, s);
    const double t_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    PNP_LAUNCH(k_fista_mom, dim3(nb), dim3(kRedThreads), 0, s, N, x, xp, (float)((t - 1.0) / t_next), z);
    t = t_next;
  }
}

}  // namespace pnp
