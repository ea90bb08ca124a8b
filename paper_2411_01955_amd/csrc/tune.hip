// Autotuner for a plan's launch shape, with a JSON-lines cache.
//
// The tuned parameters are the numbers of coils a workgroup of the
// register-FFT row passes handles (2, 4 or 8), one for the adjoint pass and
// one for the forward pass: each sets that pass's workgroup count, the
// threads and LDS per workgroup, and how often an image row and its coil
// maps are read, and the best values depend on the grid size, the coil
// count and the device.  The two passes are separate launches, so they are
// tuned one after the other: first the adjoint choice with the forward pass
// at the default, then the forward choice with the adjoint one fixed.  Each
// candidate is timed on the normal operator the caller will run (Toeplitz
// when a handle is given, else gridded), with HIP events over repeated
// launches after a warm-up, in interleaved rounds (the best round of each
// candidate counts); the default of 4 is kept unless another choice is more
// than 2% faster.  A third sweep tunes the adjoint's type-1 spread, timed on
// the gridded adjoint A^H D_w (which forms b0 = A^H D_w y in every solve
// and serves A^H and the gridded normal operator): the split level of the
// heavy column strips (0: none; 1, 2, 3: parts of about 4, 2, 1 times the
// median strip's work, each part a workgroup taking every P-th chunk of the
// strip's entries) and the number of
// entries in a row block's window above which all waves of the workgroup
// share the block (128, 256, 512) -- 12 candidates, the default (split 0,
// 128) kept unless another is more than 2% faster.  Results are cached by
// (image shape, coils, samples, a hash of the histogram of gridding entries
// per column strip, operator kind, device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

namespace pnp {

namespace {

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string tune_key(const pnp_plan* p, int L, bool toeplitz, hipStream_t s) {
  std::vector<int32_t> off(p->ntiles + 1);
  PNP_HIP(hipMemcpyAsync(off.data(), p->tile_off, sizeof(int32_t) * off.size(), hipMemcpyDeviceToHost, s));
  PNP_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> hist(p->ntiles);
  for (int t = 0; t < p->ntiles; ++t) hist[t] = off[t + 1] - off[t];
  hipDeviceProp_t prop;
  int dev = 0;
  PNP_HIP(hipGetDevice(&dev));
  PNP_HIP(hipGetDeviceProperties(&prop, dev));
  char buf[512];
  snprintf(buf, sizeof(buf), "%s|n=%dx%d|L=%d|M=%lld|hist=%016llx|op=%s|v2", prop.gcnArchName, p->ax[1].n,
           p->ax[0].n, L, (long long)p->M, (unsigned long long)fnv1a(hist.data(), hist.size() * 4),
           toeplitz ? "toeplitz" : "gridded");
  return buf;
}

bool valid_rc(int rc) { return rc == 2 || rc == 4 || rc == 8; }

// the integer after `"name": ` in `line` (0 when absent)
int field(const std::string& line, const char* name) {
  const std::string tag = std::string("\"") + name + "\": ";
  const size_t at = line.find(tag);
  return at == std::string::npos ? 0 : std::atoi(line.c_str() + at + tag.size());
}

const int kSplits[4] = {0, 1, 2, 3};
const int kDenseMins[3] = {128, 256, 512};
bool valid_split(int v) { return v >= 0 && v <= 3; }
bool valid_dense(int v) { return v == 128 || v == 256 || v == 512; }

// the cached choice of `key`; false when absent (lines without every field
// are ignored; the last matching line wins)
bool cache_lookup(const char* path, const std::string& key, int* adj, int* fwd, int* split, int* dense) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  const std::string want = "\"key\": \"" + key + "\"";
  bool found = false;
  while (std::getline(f, line)) {
    if (line.find(want) == std::string::npos) continue;
    const int a = field(line, "row_coils"), b = field(line, "row_coils_fwd");
    const int sp = field(line, "spread_split"), dm = field(line, "spread_dense_min");
    if (valid_rc(a) && valid_rc(b) && valid_split(sp) && valid_dense(dm) &&
        line.find("\"spread_split\": ") != std::string::npos) {
      *adj = a;
      *fwd = b;
      *split = sp;
      *dense = dm;
      found = true;
    }
  }
  return found;
}

void cache_append(const char* path, const std::string& key, const pnp_tuning& t) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  if (!f) fail(PNP_ERR_ARG, "cannot write the tuning cache %s", path);
  f << "{\"key\": \"" << key << "\", \"row_coils\": " << t.row_coils << ", \"row_coils_fwd\": " << t.row_coils_fwd
    << ", \"spread_split\": " << t.spread_split << ", \"spread_dense_min\": " << t.spread_dense_min
    << ", \"us\": [" << t.time_us[0] << ", " << t.time_us[1] << ", " << t.time_us[2] << "], \"us_fwd\": ["
    << t.time_fwd_us[0] << ", " << t.time_fwd_us[1] << ", " << t.time_fwd_us[2] << "], \"us_spread\": [";
  for (int i = 0; i < 12; ++i) f << (i ? ", " : "") << t.time_spread_us[i];
  f << "]}\n";
}

}  // namespace

static const int kCandidates[3] = {2, 4, 8};

void autotune(pnp_plan* p, const float2* smaps, int L, const float* dcf, const pnp_toeplitz* tp,
              const char* cache_path, pnp_tuning* out, hipStream_t s) {
  if (p->ndim != 2) fail(PNP_ERR_UNSUPPORTED, "autotuning covers 2D plans");
  const std::string key = tune_key(p, L, tp != nullptr, s);
  out->row_coils = 0;
  out->row_coils_fwd = 0;
  for (double& t : out->time_us) t = 0.0;
  for (double& t : out->time_fwd_us) t = 0.0;
  out->from_cache = 0;
  for (double& t : out->time_spread_us) t = 0.0;
  out->spread_split = 0;
  out->spread_dense_min = 0;
  int c_adj = 0, c_fwd = 0, c_split = 0, c_dense = 0;
  if (cache_lookup(cache_path, key, &c_adj, &c_fwd, &c_split, &c_dense)) {
    p->row_coils = c_adj;
    p->row_coils_fwd = c_fwd;
    adj_build_items(p, c_split, c_dense, s);
    out->row_coils = c_adj;
    out->row_coils_fwd = c_fwd;
    out->spread_split = c_split;
    out->spread_dense_min = c_dense;
    out->from_cache = 1;
    return;
  }
  const long long N = image_size(p);
  void *x = nullptr, *o = nullptr, *ws = nullptr, *yk = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  const int keep = p->row_coils, keep_fwd = p->row_coils_fwd;
  const int keep_split = p->adj_split, keep_dense = p->adj_dense_min;
  auto release = [&] {
    if (x) (void)hipFree(x);
    if (o) (void)hipFree(o);
    if (ws) (void)hipFree(ws);
    if (yk) (void)hipFree(yk);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  };
  try {
    const size_t wb = op_workspace_bytes(p, L);
    PNP_HIP(hipMalloc(&x, sizeof(float2) * N));
    PNP_HIP(hipMalloc(&o, sizeof(float2) * N));
    PNP_HIP(hipMalloc(&ws, wb));
    PNP_HIP(hipMemsetAsync(x, 0, sizeof(float2) * N, s));
    PNP_HIP(hipEventCreate(&a));
    PNP_HIP(hipEventCreate(&b));
    const OpWorkspace w = op_workspace(p, L, ws);
    auto run = [&] {
      if (tp)
        op_normal_toep(tp, (const float2*)x, smaps, L, (float2*)o, w, s);
      else
        op_normal(p, (const float2*)x, smaps, L, dcf, (float2*)o, w, s);
    };
    // one sweep: `slot` takes each candidate in interleaved rounds (each
    // candidate's best round counts); returns the default (4) unless
    // another choice is more than 2% faster
    auto sweep = [&](int* slot, double* us) {
      const int reps = 20, rounds = 3;
      for (int c = 0; c < 3; ++c) us[c] = 1e30;
      for (int round = 0; round < rounds; ++round) {
        for (int c = 0; c < 3; ++c) {
          *slot = kCandidates[c];
          for (int r = 0; r < 3; ++r) run();
          PNP_HIP(hipEventRecord(a, s));
          for (int r = 0; r < reps; ++r) run();
          PNP_HIP(hipEventRecord(b, s));
          PNP_HIP(hipEventSynchronize(b));
          float ms = 0.f;
          PNP_HIP(hipEventElapsedTime(&ms, a, b));
          us[c] = std::min(us[c], 1e3 * ms / reps);
        }
      }
      int best_rc = 4;
      double best = us[1];
      for (int c = 0; c < 3; ++c)
        if (us[c] < 0.98 * best) {
          best = us[c];
          best_rc = kCandidates[c];
        }
      *slot = best_rc;
      return best_rc;
    };
    // warm-up (clocks, caches), then the adjoint pass's choice with the
    // forward pass at the default, then the forward pass's choice
    p->row_coils = 4;
    p->row_coils_fwd = 4;
    for (int r = 0; r < 50; ++r) run();
    out->row_coils = sweep(&p->row_coils, out->time_us);
    out->row_coils_fwd = sweep(&p->row_coils_fwd, out->time_fwd_us);
    // the spread's split level and dense threshold, on the gridded adjoint
    PNP_HIP(hipMalloc(&yk, sizeof(float2) * (size_t)L * p->M));
    PNP_HIP(hipMemsetAsync(yk, 0, sizeof(float2) * (size_t)L * p->M, s));
    auto run_adj = [&] { op_adjoint(p, (const float2*)yk, smaps, L, dcf, (float2*)o, w, s); };
    {
      const int reps = 10, rounds = 3;
      double* us = out->time_spread_us;
      for (int c = 0; c < 12; ++c) us[c] = 1e30;
      for (int round = 0; round < rounds; ++round) {
        for (int c = 0; c < 12; ++c) {
          adj_build_items(p, kSplits[c / 3], kDenseMins[c % 3], s);
          for (int r = 0; r < 3; ++r) run_adj();
          PNP_HIP(hipEventRecord(a, s));
          for (int r = 0; r < reps; ++r) run_adj();
          PNP_HIP(hipEventRecord(b, s));
          PNP_HIP(hipEventSynchronize(b));
          float ms = 0.f;
          PNP_HIP(hipEventElapsedTime(&ms, a, b));
          us[c] = std::min(us[c], 1e3 * ms / reps);
        }
      }
      int best_c = 3;                                  // split 1, 128: the default
      double best = us[best_c];
      for (int c = 0; c < 12; ++c)
        if (us[c] < 0.98 * best) {
          best = us[c];
          best_c = c;
        }
      out->spread_split = kSplits[best_c / 3];
      out->spread_dense_min = kDenseMins[best_c % 3];
      adj_build_items(p, out->spread_split, out->spread_dense_min, s);
    }
    release();
  } catch (...) {
    p->row_coils = keep;
    p->row_coils_fwd = keep_fwd;
    release();
    try {
      adj_build_items(p, keep_split, keep_dense, s);
    } catch (...) {
    }
    throw;
  }
  cache_append(cache_path, key, *out);
}

void plan_set_spread(pnp_plan* p, int split, int dense_min, hipStream_t s) {
  if (p->ndim != 2) fail(PNP_ERR_UNSUPPORTED, "the spread split applies to 2D plans");
  if (!valid_split(split) || dense_min < 1) fail(PNP_ERR_ARG, "split must be 0..3 and dense_min >= 1");
  adj_build_items(p, split, dense_min, s);
}

void plan_set_row_coils(pnp_plan* p, int fwd, int adj) {
  if (!valid_rc(fwd) || !valid_rc(adj)) fail(PNP_ERR_ARG, "row_coils must be 2, 4 or 8");
  p->row_coils = adj;
  p->row_coils_fwd = fwd;
}

}  // namespace pnp
