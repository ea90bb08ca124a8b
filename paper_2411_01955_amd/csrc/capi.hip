// C ABI: argument validation, error reporting and dispatch.  Nothing is
// enqueued before every argument has been checked; internal failures are
// converted to status codes here and never cross the ABI as exceptions.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "common.hpp"
#include "trace.hpp"

namespace pnp {

static thread_local std::string g_err;

void set_error_text(const std::string& s) { g_err = s; }

void fail(pnp_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  throw Failure{code};
}

void fail_hip(hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what,
           file, line);
  g_err = buf;
  throw Failure{PNP_ERR_DEVICE};
}

}  // namespace pnp

using namespace pnp;

namespace {

template <class F>
pnp_status guarded(F&& f) {
  try {
    g_err.clear();
    f();
    return PNP_OK;
  } catch (const Failure& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return PNP_ERR_DEVICE;
  } catch (...) {
    g_err = "unexpected internal error";
    return PNP_ERR_DEVICE;
  }
}

void need(const void* ptr, const char* name) {
  if (!ptr) fail(PNP_ERR_ARG, "%s must not be NULL", name);
}

void check_plan_L(const pnp_plan* p, int32_t L) {
  need(p, "plan");
  if (L < 1) fail(PNP_ERR_SHAPE, "L must be >= 1 (got %d)", L);
}

// Static device scratch of the no-allocation entry point.  In host code
// `scratch` only names the symbol: its device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and kept; the
// kernels always receive that address.  Every call on one device shares the
// array, so concurrent calls on one device race.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static void* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up on first use).
void* noalloc_scratch() {
  int dev = 0;
  PNP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(PNP_ERR_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    PNP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(PNP_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

void check_ws(size_t have, size_t need_bytes, const void* ws) {
  if (have < need_bytes)
    fail(PNP_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the required %zu", have, need_bytes);
  if (((uintptr_t)ws & 255) != 0) fail(PNP_ERR_ARG, "workspace must be 256-byte aligned");
}

}  // namespace

extern "C" {

const char* pnp_last_error(void) { return g_err.c_str(); }

int32_t pnp_version(void) { return 100; }

pnp_status pnp_trace_enable(int32_t on) {
  return guarded([&] { trace_enable(on != 0); });
}

pnp_status pnp_trace_read(char* buf, size_t len, size_t* needed) {
  return guarded([&] {
    const std::string s = trace_read_json();
    if (needed) *needed = s.size() + 1;
    if (buf && len) {
      const size_t n = std::min(len - 1, s.size());
      memcpy(buf, s.data(), n);
      buf[n] = 0;
      if (n < s.size()) fail(PNP_ERR_ARG, "trace buffer of %zu bytes is too small (%zu needed)", len, s.size() + 1);
    }
  });
}

pnp_status pnp_plan_create(pnp_plan** out, int32_t ndim, const int32_t* shape, int64_t M,
                           const float* traj, hipStream_t stream) {
  return guarded([&] {
    need(out, "out");
    need(shape, "shape");
    need(traj, "traj");
    *out = nullptr;
    *out = plan_create(ndim, shape, M, traj, stream);
  });
}

pnp_status pnp_plan_destroy(pnp_plan* plan) {
  return guarded([&] { plan_destroy(plan); });
}

pnp_status pnp_plan_info(const pnp_plan* p, int32_t* grid_shape, int32_t* n_tiles, int64_t* n_entries) {
  return guarded([&] {
    need(p, "plan");
    if (grid_shape)
      for (int a = 0; a < p->ndim; ++a) grid_shape[a] = p->ax[p->ndim - 1 - a].K;
    if (n_tiles) *n_tiles = p->ntiles;
    if (n_entries) *n_entries = p->E;
  });
}

pnp_status pnp_workspace_bytes(const pnp_plan* p, int32_t L, size_t* bytes) {
  return guarded([&] {
    check_plan_L(p, L);
    need(bytes, "bytes");
    *bytes = opnorm_workspace_bytes(p, L);
  });
}

pnp_status pnp_forward(const pnp_plan* p, const pnp_c64* x, const pnp_c64* smaps, int32_t L, pnp_c64* y,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(x, "x");
    need(smaps, "smaps");
    need(y, "y");
    need(ws, "ws");
    check_ws(ws_bytes, op_workspace_bytes(p, L), ws);
    op_forward(p, (const float2*)x, (const float2*)smaps, L, (float2*)y, op_workspace(p, L, ws), stream);
  });
}

pnp_status pnp_adjoint(const pnp_plan* p, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                       const float* dcf, pnp_c64* x, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(y, "y");
    need(smaps, "smaps");
    need(x, "x");
    need(ws, "ws");
    check_ws(ws_bytes, op_workspace_bytes(p, L), ws);
    op_adjoint(p, (const float2*)y, (const float2*)smaps, L, dcf, (float2*)x, op_workspace(p, L, ws),
               stream);
  });
}

pnp_status pnp_normal(const pnp_plan* p, const pnp_c64* x, const pnp_c64* smaps, int32_t L,
                      const float* dcf, pnp_c64* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(x, "x");
    need(smaps, "smaps");
    need(out, "out");
    need(ws, "ws");
    if ((const void*)x == (const void*)out) fail(PNP_ERR_ARG, "x and out must not alias");
    check_ws(ws_bytes, op_workspace_bytes(p, L), ws);
    op_normal(p, (const float2*)x, (const float2*)smaps, L, dcf, (float2*)out, op_workspace(p, L, ws),
              stream);
  });
}

pnp_status pnp_opnorm(const pnp_plan* p, const pnp_c64* smaps, int32_t L, const float* dcf,
                      int32_t iters, uint64_t seed, double* norm_out, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(smaps, "smaps");
    need(norm_out, "norm_out");
    need(ws, "ws");
    if (iters < 1) fail(PNP_ERR_ARG, "iters must be >= 1");
    check_ws(ws_bytes, opnorm_workspace_bytes(p, L), ws);
    const double v = power_iteration(p, nullptr, (const float2*)smaps, L, dcf, iters, seed, ws, stream);
    if (!std::isfinite(v)) fail(PNP_ERR_NUMERIC, "power iteration produced a non-finite norm");
    *norm_out = v;
  });
}

pnp_status pnp_toeplitz_create(pnp_toeplitz** out, const pnp_plan* plan, const float* dcf,
                               hipStream_t stream) {
  return guarded([&] {
    need(out, "out");
    need(plan, "plan");
    *out = nullptr;
    (void)noalloc_scratch();   // set-up of the no-allocation entry point on this device
    *out = toeplitz_create(plan, plan->traj, dcf, stream);
  });
}

pnp_status pnp_toeplitz_destroy(pnp_toeplitz* tp) {
  return guarded([&] { toeplitz_destroy(tp); });
}

pnp_status pnp_normal_toeplitz(const pnp_toeplitz* tp, const pnp_c64* x, const pnp_c64* smaps, int32_t L,
                               pnp_c64* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    need(tp, "toeplitz");
    check_plan_L(tp->plan, L);
    need(x, "x");
    need(smaps, "smaps");
    need(out, "out");
    need(ws, "ws");
    if ((const void*)x == (const void*)out) fail(PNP_ERR_ARG, "x and out must not alias");
    check_ws(ws_bytes, op_workspace_bytes(tp->plan, L), ws);
    op_normal_toep(tp, (const float2*)x, (const float2*)smaps, L, (float2*)out,
                   op_workspace(tp->plan, L, ws), stream);
  });
}

pnp_status pnp_noalloc_scratch_bytes(size_t* bytes) {
  return guarded([&] {
    need(bytes, "bytes");
    *bytes = kNoAllocScratchBytes;
  });
}

pnp_status pnp_normal_toeplitz_noalloc(const pnp_toeplitz* tp, const pnp_c64* x, const pnp_c64* smaps,
                                       int32_t L, pnp_c64* out, hipStream_t stream) {
  return guarded([&] {
    need(tp, "toeplitz");
    check_plan_L(tp->plan, L);
    need(x, "x");
    need(smaps, "smaps");
    need(out, "out");
    if ((const void*)x == (const void*)out) fail(PNP_ERR_ARG, "x and out must not alias");
    const size_t need_bytes = op_workspace_bytes(tp->plan, L);
    if (need_bytes > kNoAllocScratchBytes)
      fail(PNP_ERR_WORKSPACE,
           "pnp_normal_toeplitz_noalloc: %d coils on this plan need %zu bytes of scratch, more than the "
           "library's static %zu; use pnp_normal_toeplitz with a caller workspace",
           L, need_bytes, (size_t)kNoAllocScratchBytes);
    void* ws = noalloc_scratch();
    op_normal_toep(tp, (const float2*)x, (const float2*)smaps, L, (float2*)out, op_workspace(tp->plan, L, ws),
                   stream);
  });
}

pnp_status pnp_prior_wavelet(pnp_prior** out, int32_t levels, double kappa) {
  return guarded([&] {
    need(out, "out");
    if (levels < 0 || levels > 8) fail(PNP_ERR_ARG, "levels must be in 0..8");
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) fail(PNP_ERR_ARG, "kappa must be finite and >= 0");
    pnp_prior* p = new pnp_prior();
    p->kind = 0;
    p->levels = levels;
    p->kappa = kappa;
    *out = p;
  });
}

pnp_status pnp_prior_destroy(pnp_prior* prior) {
  return guarded([&] {
    if (prior && prior->ws) PNP_HIP(hipFree(prior->ws));
    delete prior;
  });
}

pnp_status pnp_prior_unet(pnp_prior** out, const pnp_unet* net, int32_t ndim, const int32_t* shape, double kappa,
                          const pnp_prior* fallback) {
  return guarded([&] {
    need(out, "out");
    need(net, "net");
    need(shape, "shape");
    if (ndim != 2 && ndim != 3) fail(PNP_ERR_SHAPE, "ndim must be 2 or 3");
    if (!(kappa > 0.0) || !std::isfinite(kappa)) fail(PNP_ERR_ARG, "kappa must be finite and > 0");
    if (fallback && fallback->kind != 0) fail(PNP_ERR_ARG, "the fallback must be a wavelet prior");
    const int B = ndim == 3 ? shape[0] : 1, H = shape[ndim - 2], W = shape[ndim - 1];
    const size_t bytes = unet_ws_bytes(B, H, W, false);
    void* ws = nullptr;
    PNP_HIP(hipMalloc(&ws, bytes));
    pnp_prior* p = new (std::nothrow) pnp_prior();
    if (!p) {
      (void)hipFree(ws);
      fail(PNP_ERR_DEVICE, "host allocation failed");
    }
    p->kind = 1;
    p->kappa = kappa;
    p->net = net;
    p->fallback = fallback;
    p->batch = B;
    p->ny = H;
    p->nx = W;
    p->ws = ws;
    *out = p;
  });
}

pnp_status pnp_prior_apply(const pnp_prior* prior, int32_t ndim, const int32_t* shape, const pnp_c64* in,
                           pnp_c64* out, double sigma, hipStream_t stream) {
  return guarded([&] {
    need(prior, "prior");
    need(shape, "shape");
    need(in, "in");
    need(out, "out");
    if (ndim != 2 && ndim != 3) fail(PNP_ERR_SHAPE, "ndim must be 2 or 3");
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) fail(PNP_ERR_ARG, "sigma must be finite and >= 0");
    int n[3] = {1, 1, 1};
    for (int a = 0; a < ndim; ++a) {
      n[a] = shape[ndim - 1 - a];
      if (n[a] < 2) fail(PNP_ERR_SHAPE, "image sides must be >= 2");
    }
    prior_apply(prior, ndim, n, (const float2*)in, (float2*)out, sigma, stream);
  });
}

pnp_status pnp_hqs_workspace_bytes(const pnp_plan* p, int32_t L, size_t* bytes) {
  return guarded([&] {
    check_plan_L(p, L);
    need(bytes, "bytes");
    *bytes = hqs_workspace_bytes(p, L);
  });
}

pnp_status pnp_hqs_solve(const pnp_plan* p, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                         const float* dcf, const pnp_prior* prior, const double* sigmas, int32_t n_out,
                         const pnp_hqs_opts* opts, pnp_c64* x_out, pnp_hqs_report* report, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(y, "y");
    need(smaps, "smaps");
    need(prior, "prior");
    need(sigmas, "sigmas");
    need(opts, "opts");
    need(x_out, "x_out");
    need(ws, "ws");
    if (opts->struct_size < offsetof(pnp_hqs_opts, k_start)) fail(PNP_ERR_ARG, "opts.struct_size too small");
    const int32_t k_start =
        opts->struct_size >= offsetof(pnp_hqs_opts, k_start) + sizeof(int32_t) ? opts->k_start : 0;
    if (n_out < 1) fail(PNP_ERR_SHAPE, "n_out must be >= 1");
    if (k_start < 0 || k_start >= n_out) fail(PNP_ERR_ARG, "k_start %d outside [0, n_out = %d)", k_start, n_out);
    if (opts->precond < 0 || opts->precond > 2) fail(PNP_ERR_ARG, "unknown preconditioner %d", opts->precond);
    if (opts->n_cg < 1) fail(PNP_ERR_ARG, "n_cg must be >= 1");
    if (!(opts->lambda > 0.0) || !std::isfinite(opts->lambda)) fail(PNP_ERR_ARG, "lambda must be > 0");
    for (int k = k_start; k < n_out; ++k)
      if (!(sigmas[k] > 0.0) || !std::isfinite(sigmas[k])) fail(PNP_ERR_ARG, "sigma[%d] must be > 0", k);
    if (report) {
      if (report->struct_size < sizeof(pnp_hqs_report)) fail(PNP_ERR_ARG, "report.struct_size too small");
      if (report->capacity < n_out) fail(PNP_ERR_ARG, "report capacity %d < n_out %d", report->capacity, n_out);
      need(report->rho, "report.rho");
    }
    if ((const void*)x_out == (const void*)y || (const void*)x_out == (const void*)smaps)
      fail(PNP_ERR_ARG, "x_out must not alias y or smaps");
    if (opts->toeplitz && opts->toeplitz->plan != p)
      fail(PNP_ERR_ARG, "opts.toeplitz was built for another plan");
    check_ws(ws_bytes, hqs_workspace_bytes(p, L), ws);
    double nrm = opts->opnorm;
    if (!(nrm > 0.0)) {
      const int its = opts->opnorm_iters > 0 ? opts->opnorm_iters : 50;
      nrm = power_iteration(p, opts->toeplitz, (const float2*)smaps, L, dcf, its, opts->opnorm_seed, ws,
                            stream);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) fail(PNP_ERR_NUMERIC, "operator norm is %g", nrm);
    }
    HQSArgs a;
    a.y = (const float2*)y;
    a.smaps = (const float2*)smaps;
    a.L = L;
    a.dcf = dcf;
    a.prior = prior;
    a.sigmas = sigmas + k_start;
    a.n_out = n_out - k_start;
    a.precond = opts->precond;
    a.n_cg = opts->n_cg;
    a.lambda = opts->lambda;
    a.opnorm = nrm;
    a.x0 = (const float2*)opts->x0;
    a.x_out = (float2*)x_out;
    a.toep = opts->toeplitz;
    a.rise_tol = opts->rise_tol;
    if (prior->fallback && (!(opts->rise_tol >= 0.0) || !std::isfinite(opts->rise_tol)))
      fail(PNP_ERR_ARG, "rise_tol must be finite and >= 0 for a prior with a fallback");
    int bad = 0;
    hqs_solve(p, a, ws, stream, report ? report->rho + k_start : nullptr, report ? &bad : nullptr,
              report && report->fallback ? report->fallback + k_start : nullptr);
    if (report) {
      report->opnorm_used = nrm;
      if (bad) fail(PNP_ERR_NUMERIC, "CG breakdown (non-positive or non-finite <p, Mp>)");
    }
  });
}

}  // extern "C"

// ------------------------------------------------------------------ UNet
int32_t pnp_unet_layer_count(void) { return unet_layer_count(); }

int64_t pnp_unet_param_count(void) { return unet_param_count(); }

pnp_status pnp_unet_layer_info(int32_t i, pnp_unet_layer* out) {
  return guarded([&] {
    need(out, "out");
    unet_layer_info(i, out);
  });
}

pnp_status pnp_unet_create(pnp_unet** out, const float* params, hipStream_t stream) {
  return guarded([&] {
    need(out, "out");
    need(params, "params");
    *out = unet_create(params, stream);
  });
}

pnp_status pnp_unet_destroy(pnp_unet* net) {
  return guarded([&] { unet_destroy(net); });
}

pnp_status pnp_unet_set(pnp_unet* net, int32_t which, const float* src, hipStream_t stream) {
  return guarded([&] {
    need(net, "net");
    need(src, "src");
    if (which == PNP_UNET_GRAD) fail(PNP_ERR_ARG, "gradients are written by pnp_unet_backward only");
    unet_set(net, which, src, stream);
  });
}

pnp_status pnp_unet_get(pnp_unet* net, int32_t which, float* dst, hipStream_t stream) {
  return guarded([&] {
    need(net, "net");
    need(dst, "dst");
    unet_get(net, which, dst, stream);
  });
}

pnp_status pnp_unet_get_step(const pnp_unet* net, int64_t* step) {
  return guarded([&] {
    need(net, "net");
    need(step, "step");
    *step = unet_step(const_cast<pnp_unet*>(net));
  });
}

pnp_status pnp_unet_set_step(pnp_unet* net, int64_t step) {
  return guarded([&] {
    need(net, "net");
    if (step < 0) fail(PNP_ERR_ARG, "step must be >= 0");
    unet_step(net) = step;
  });
}

pnp_status pnp_unet_workspace_bytes(int32_t B, int32_t H, int32_t W, int32_t train, size_t* bytes) {
  return guarded([&] {
    need(bytes, "bytes");
    *bytes = unet_ws_bytes(B, H, W, train != 0);
  });
}

pnp_status pnp_unet_forward(const pnp_unet* net, const pnp_c64* u, const float* sigma, int32_t B, int32_t H,
                            int32_t W, pnp_c64* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    need(net, "net");
    need(u, "u");
    need(sigma, "sigma");
    need(out, "out");
    check_ws(ws_bytes, unet_ws_bytes(B, H, W, false), ws);
    unet_forward(net, (const float2*)u, sigma, 0.f, B, H, W, (float2*)out, ws, stream);
  });
}

pnp_status pnp_unet_backward(pnp_unet* net, const pnp_c64* u, const pnp_c64* target, int32_t B, int32_t H,
                             int32_t W, double* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    need(net, "net");
    need(u, "u");
    need(target, "target");
    need(loss, "loss");
    check_ws(ws_bytes, unet_ws_bytes(B, H, W, true), ws);
    unet_backward(net, (const float2*)u, (const float2*)target, B, H, W, loss, ws, stream);
  });
}

pnp_status pnp_n2n_workspace_bytes(int32_t B, int32_t H, int32_t W, size_t* bytes) {
  return guarded([&] {
    need(bytes, "bytes");
    *bytes = unet_n2n_ws_bytes(B, H, W);
  });
}

pnp_status pnp_n2n_backward(pnp_unet* net, const pnp_c64* x, const uint8_t* codes, double eta, int32_t B,
                            int32_t H, int32_t W, double* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    need(net, "net");
    need(x, "x");
    need(codes, "codes");
    need(loss, "loss");
    if (!(eta >= 0.0) || !std::isfinite(eta)) fail(PNP_ERR_ARG, "eta must be finite and >= 0");
    check_ws(ws_bytes, unet_n2n_ws_bytes(B, H, W), ws);
    unet_n2n_backward(net, (const float2*)x, codes, eta, B, H, W, loss, ws, stream);
  });
}

pnp_status pnp_unet_adam_step(pnp_unet* net, double lr, double beta1, double beta2, double eps,
                              hipStream_t stream) {
  return guarded([&] {
    need(net, "net");
    if (!(lr >= 0.0) || !std::isfinite(lr)) fail(PNP_ERR_ARG, "lr must be finite and >= 0");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
      fail(PNP_ERR_ARG, "betas must lie in [0, 1)");
    if (!(eps > 0.0)) fail(PNP_ERR_ARG, "eps must be > 0");
    unet_adam(net, lr, beta1, beta2, eps, stream);
  });
}

pnp_status pnp_unet_tensor(int32_t B, int32_t H, int32_t W, int32_t train, void* ws, int32_t id, void** ptr,
                           int32_t* dims) {
  return guarded([&] {
    need(ptr, "ptr");
    need(dims, "dims");
    unet_tensor(B, H, W, train != 0, ws, id, ptr, dims);
  });
}

// --------------------------------------------------------------- batches
pnp_status pnp_batch_create(pnp_batch** out, int32_t B, const pnp_slice* slices, hipStream_t stream) {
  return guarded([&] {
    need(out, "out");
    need(slices, "slices");
    *out = batch_create(B, slices, stream);
  });
}

pnp_status pnp_batch_destroy(pnp_batch* batch) {
  return guarded([&] { batch_destroy(batch); });
}

pnp_status pnp_batch_normal(pnp_batch* batch, const pnp_c64* const* x, pnp_c64* const* out, hipStream_t stream) {
  return guarded([&] {
    need(batch, "batch");
    need(x, "x");
    need(out, "out");
    batch_normal(batch, (const float2* const*)x, (float2* const*)out, stream);
  });
}

pnp_status pnp_batch_workspace_bytes(const pnp_batch* batch, const pnp_prior* prior, size_t* bytes) {
  return guarded([&] {
    need(batch, "batch");
    need(prior, "prior");
    need(bytes, "bytes");
    *bytes = prior->kind == 1 ? batch_unet_ws_bytes(batch) : 0;
  });
}

pnp_status pnp_hqs_solve_batched(pnp_batch* batch, const pnp_prior* prior, const double* sigmas, int32_t n_out,
                                 int32_t precond, int32_t n_cg, double* rho, void* ws, size_t ws_bytes,
                                 hipStream_t stream) {
  return guarded([&] {
    need(batch, "batch");
    need(prior, "prior");
    need(sigmas, "sigmas");
    if (n_out < 1) fail(PNP_ERR_SHAPE, "n_out must be >= 1");
    if (precond < 0 || precond > 2) fail(PNP_ERR_ARG, "unknown preconditioner %d", precond);
    if (n_cg < 1) fail(PNP_ERR_ARG, "n_cg must be >= 1");
    for (int k = 0; k < n_out; ++k)
      if (!(sigmas[k] > 0.0) || !std::isfinite(sigmas[k])) fail(PNP_ERR_ARG, "sigma[%d] must be > 0", k);
    if (prior->kind == 1) check_ws(ws_bytes, batch_unet_ws_bytes(batch), ws);
    int bad = 0;
    batch_hqs_solve(batch, prior, sigmas, n_out, precond, n_cg, ws, rho, rho ? &bad : nullptr, stream);
    if (bad) fail(PNP_ERR_NUMERIC, "CG breakdown in a batched slice");
  });
}

pnp_status pnp_smaps_workspace_bytes(const pnp_plan* p, size_t* bytes) {
  return guarded([&] {
    need(p, "plan");
    need(bytes, "bytes");
    *bytes = smaps_workspace_bytes(p);
  });
}

pnp_status pnp_smaps_estimate(const pnp_plan* p, const pnp_c64* y, int32_t L, const float* dcf, double width,
                              double threshold, pnp_c64* smaps_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(y, "y");
    need(smaps_out, "smaps_out");
    need(ws, "ws");
    if (!(width > 0.0) || !std::isfinite(width)) fail(PNP_ERR_ARG, "width must be > 0");
    if (!(threshold >= 0.0 && threshold < 1.0)) fail(PNP_ERR_ARG, "threshold must be in [0, 1)");
    if ((const void*)smaps_out == (const void*)y) fail(PNP_ERR_ARG, "smaps_out must not alias y");
    check_ws(ws_bytes, smaps_workspace_bytes(p), ws);
    smaps_estimate(p, (const float2*)y, L, dcf, width, threshold, (float2*)smaps_out, ws, stream);
  });
}

pnp_status pnp_pgd_solve(const pnp_plan* p, const pnp_c64* y, const pnp_c64* smaps, int32_t L, const float* dcf,
                         const pnp_prior* prior, const double* sigmas, int32_t n_iter, double gamma,
                         int32_t precond, double opnorm, const pnp_toeplitz* toeplitz, const pnp_c64* x0,
                         pnp_c64* x_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(y, "y");
    need(smaps, "smaps");
    need(prior, "prior");
    need(sigmas, "sigmas");
    need(x_out, "x_out");
    need(ws, "ws");
    if (n_iter < 1) fail(PNP_ERR_SHAPE, "n_iter must be >= 1");
    if (precond < 0 || precond > 2) fail(PNP_ERR_ARG, "unknown preconditioner %d", precond);
    if (!(gamma > 0.0) || !std::isfinite(gamma)) fail(PNP_ERR_ARG, "gamma must be > 0");
    if (precond != 0 && (!(opnorm > 0.0) || !std::isfinite(opnorm)))
      fail(PNP_ERR_ARG, "a preconditioned PGD needs opnorm > 0");
    for (int k = 0; k < n_iter; ++k)
      if (!(sigmas[k] > 0.0) || !std::isfinite(sigmas[k])) fail(PNP_ERR_ARG, "sigma[%d] must be > 0", k);
    if ((const void*)x_out == (const void*)y || (const void*)x_out == (const void*)smaps)
      fail(PNP_ERR_ARG, "x_out must not alias y or smaps");
    if (toeplitz && toeplitz->plan != p) fail(PNP_ERR_ARG, "toeplitz was built for another plan");
    check_ws(ws_bytes, hqs_workspace_bytes(p, L), ws);
    PGDArgs a;
    a.y = (const float2*)y;
    a.smaps = (const float2*)smaps;
    a.L = L;
    a.dcf = dcf;
    a.prior = prior;
    a.sigmas = sigmas;
    a.n_iter = n_iter;
    a.precond = precond;
    a.gamma = gamma;
    a.opnorm = precond != 0 ? opnorm : 1.0;
    a.x0 = (const float2*)x0;
    a.x_out = (float2*)x_out;
    a.toep = toeplitz;
    pgd_solve(p, a, ws, stream);
  });
}

pnp_status pnp_fista_wavelet(const pnp_plan* p, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                             const float* dcf, int32_t levels, double lam, double gamma, int32_t n_iter,
                             const pnp_toeplitz* toeplitz, const pnp_c64* x0, pnp_c64* x_out, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    check_plan_L(p, L);
    need(y, "y");
    need(smaps, "smaps");
    need(x_out, "x_out");
    need(ws, "ws");
    if (n_iter < 1) fail(PNP_ERR_SHAPE, "n_iter must be >= 1");
    if (levels < 0) fail(PNP_ERR_ARG, "levels must be >= 0");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) fail(PNP_ERR_ARG, "gamma must be > 0");
    if (!(lam >= 0.0) || !std::isfinite(lam)) fail(PNP_ERR_ARG, "lam must be >= 0");
    if ((const void*)x_out == (const void*)y || (const void*)x_out == (const void*)smaps)
      fail(PNP_ERR_ARG, "x_out must not alias y or smaps");
    if (toeplitz && toeplitz->plan != p) fail(PNP_ERR_ARG, "toeplitz was built for another plan");
    check_ws(ws_bytes, hqs_workspace_bytes(p, L), ws);
    FISTAArgs a;
    a.y = (const float2*)y;
    a.smaps = (const float2*)smaps;
    a.L = L;
    a.dcf = dcf;
    a.levels = levels;
    a.lam = lam;
    a.gamma = gamma;
    a.n_iter = n_iter;
    a.x0 = (const float2*)x0;
    a.x_out = (float2*)x_out;
    a.toep = toeplitz;
    fista_wavelet(p, a, ws, stream);
  });
}

// ------------------------------------------------------------- autotuning
pnp_status pnp_autotune(pnp_plan* plan, const pnp_c64* smaps, int32_t L, const float* dcf,
                        const pnp_toeplitz* toeplitz, const char* cache_path, pnp_tuning* out,
                        hipStream_t stream) {
  return guarded([&] {
    check_plan_L(plan, L);
    need(smaps, "smaps");
    need(out, "out");
    if (out->struct_size < sizeof(pnp_tuning)) fail(PNP_ERR_ARG, "out.struct_size too small");
    if (toeplitz && toeplitz->plan != plan) fail(PNP_ERR_ARG, "toeplitz was built for another plan");
    autotune(plan, (const float2*)smaps, L, dcf, toeplitz, cache_path, out, stream);
  });
}

pnp_status pnp_plan_set_spread(pnp_plan* plan, int32_t split, int32_t dense_min, hipStream_t stream) {
  return guarded([&] {
    need(plan, "plan");
    plan_set_spread(plan, split, dense_min, stream);
  });
}

pnp_status pnp_plan_get_spread(const pnp_plan* plan, int32_t* split, int32_t* dense_min) {
  return guarded([&] {
    need(plan, "plan");
    need(split, "split");
    need(dense_min, "dense_min");
    if (plan->ndim != 2) fail(PNP_ERR_UNSUPPORTED, "the spread split applies to 2D plans");
    *split = plan->adj_split;
    *dense_min = plan->adj_dense_min;
  });
}

pnp_status pnp_plan_set_row_coils(pnp_plan* plan, int32_t row_coils) {
  return guarded([&] {
    need(plan, "plan");
    plan_set_row_coils(plan, row_coils, row_coils);
  });
}

pnp_status pnp_plan_get_row_coils(const pnp_plan* plan, int32_t* row_coils) {
  return guarded([&] {
    need(plan, "plan");
    need(row_coils, "row_coils");
    *row_coils = plan->row_coils;
  });
}

pnp_status pnp_plan_set_row_coils_pair(pnp_plan* plan, int32_t forward, int32_t adjoint) {
  return guarded([&] {
    need(plan, "plan");
    plan_set_row_coils(plan, forward, adjoint);
  });
}

pnp_status pnp_plan_get_row_coils_pair(const pnp_plan* plan, int32_t* forward, int32_t* adjoint) {
  return guarded([&] {
    need(plan, "plan");
    need(forward, "forward");
    need(adjoint, "adjoint");
    *forward = plan->row_coils_fwd;
    *adjoint = plan->row_coils;
  });
}
