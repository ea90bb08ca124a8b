// Internal definitions shared by the library's translation units.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pnpmri.h"

namespace pnp {

// ---------------------------------------------------------------- errors
// Internal failures are thrown as pnp::Failure and converted to a status at
// the C ABI (no exception crosses it).
struct Failure {
  pnp_status code;
};

[[noreturn]] void fail(pnp_status code, const char* fmt, ...);
[[noreturn]] void fail_hip(hipError_t e, const char* what, const char* file, int line);
void set_error_text(const std::string& s);

#define PNP_HIP(call)                                                  \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) ::pnp::fail_hip(e_, #call, __FILE__, __LINE__); \
  } while (0)

#define PNP_CHECK_LAUNCH() PNP_HIP(hipGetLastError())

// --------------------------------------------------------- complex helpers
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline float2 cfma(float s, float2 a, float2 acc) {
  return make_float2(fmaf(s, a.x, acc.x), fmaf(s, a.y, acc.y));
}

// ------------------------------------------------------ XCD-aware order
// The MI355X deals consecutive workgroups of a launch to its 8 XCDs in
// turn (workgroup b runs on XCD b % 8).  xcd_order(b, nb) renumbers them so
// that XCD j works through the contiguous range of logical indices
// [start_j, start_j + count_j): neighbouring logical workgroups then share
// cache lines (and read-only tables) in one XCD's L2.  Bijective on [0, nb).
constexpr int kXCDs = 8;
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int j = b % kXCDs, q = nb / kXCDs, r = nb % kXCDs;
  return j * q + (j < r ? j : r) + b / kXCDs;
}

// ------------------------------------------------------------ FFT plan
constexpr int kMaxRadices = 16;

// One 1D FFT length: its radix sequence (Stockham order) and the device
// table of the K-th roots of unity exp(-2*pi*i*t/K), t = 0..K-1, tabulated
// in FP64 and rounded to FP32.
struct FFTDesc {
  int K;
  int nrad;
  int rad[kMaxRadices];
  const float2* tw;
};

// Factor K into radices 8, 4, 2, 5, 3 (largest power-of-two radices first).
// Returns false when K has another prime factor.
bool fft_factor(int K, FFTDesc* d);

// ------------------------------------------------------------------- plan
struct Axis {
  int n;             // image size along the axis
  int K;             // oversampled grid size (2n)
  FFTDesc fft;       // length-K transform
  float* deapod;     // device [n]: I0(beta) / Phi((i - n/2)/K)
};

// One (sample, tile) entry, packed for a single 64-byte load in the 2D
// kernels: idx = (first x tap, first y tap, sample, 0), w0..w2 = the 6 x
// weights followed by the 6 y weights.
struct alignas(16) EntryRec {
  int4 idx;
  float4 w0, w1, w2;
};

}  // namespace pnp

// The opaque plan handle of the ABI.
struct pnp_plan {
  int ndim;
  pnp::Axis ax[3];          // internal axis order: 0 = x (fastest), 1 = y, 2 = z
  int64_t M;
  int W;                    // kernel width (6)
  double beta;              // Kaiser-Bessel shape
  int tile;                 // tile edge (grid columns) along the tiled axes
  int row_coils;            // coils per workgroup in the register-FFT adjoint row pass (2, 4 or 8);
                            // also the coil-group count of the partial images
  int row_coils_fwd;        // coils per workgroup in the register-FFT forward row pass (2, 4 or 8)
  int ntx, nty;             // tiles along x and y (nty = 1 in 2D)
  int ntiles;
  int slots;                // max tiles a sample touches (2 in 2D, 4 in 3D)
  int64_t E;                // number of (sample, tile) entries
  int max_tile_entries;
  int device;
  // device arrays (inside one allocation `block`)
  int4* j0;                 // [M] wrapped first tap index per axis (x, y, z)
  float* wts;               // [M][ndim][W] kernel weights phi(g - j) / I0(beta)
  float* deapod_yz;         // 3D: [nz][ny] deapodisation of the (z, y) image rows
  int32_t* tile_off;        // [ntiles + 1]
  int32_t* row_start;       // [ntiles][K_last + 1] first entry per first-tap row
  int32_t* tile_order;      // 2D: [ntiles] tiles by descending entry count (spread dispatch order)
  int32_t* ent_sample;      // [E] sample of each entry, grouped by tile
  int32_t* sample_ent;      // [M][slots] entry indices of a sample (-1: none)
  pnp::EntryRec* rec;       // [E] packed taps and weights, grouped by tile (2D)
  float* traj;              // [M][ndim] copy of the trajectory (radians)
  // 3D: samples sorted by the grid cell of their first tap (stable), for
  // the gather form of the spread
  int32_t* sorted_m;        // [M] sample index in sorted order
  int32_t* sorted_jx;       // [M] first x tap of each sorted sample
  float* sorted_w;          // [M][3][W] weights in sorted order
  int32_t* cell_off;        // [Kz*Ky*Kx + 1] first sorted index of each cell
  // 3D spread work list over 8^3 grid tiles: items (tile, first candidate,
  // end candidate, partial slot or -1), heaviest first; tiles whose
  // candidates are split over several items are summed from their slots by
  // the folds (tile, first slot, slot count, 0)
  int4* sp_items;
  int4* sp_folds;
  int n_sp_items, n_sp_folds, sp_slots;
  // 3D interpolation work list: items (tile, first, end, 0) over the
  // samples whose first-tap cell lies in the tile (its home samples, listed
  // row by row), in tile order, at most kInterpChunk3 samples an item
  int4* ip_items;
  int n_ip_items;
  // 2D adjoint spread work items (strip, part, parts, first slot or -1),
  // heaviest first, and the split strips (strip, first slot, parts, 0);
  // built from the per-(strip, row block) window entry counts adj_cost for
  // a split level and a dense-block threshold (tuned)
  int4* adj_items;
  int4* adj_splits;
  int n_adj_items, n_adj_splits;
  int adj_split, adj_dense_min;
  std::vector<int32_t> adj_cost;   // host [ntx][K_y / 8]
  void* block;
  size_t block_bytes;
  void* block3;             // 3D: the spread and interpolation work lists
};

struct pnp_unet;

struct pnp_prior {
  int kind;                 // 0 = Haar wavelet, 1 = UNet
  int levels;               // wavelet: 0 = default rule
  double kappa;             // wavelet: tau = kappa*sigma; UNet: conditioning level kappa*sigma
  const pnp_unet* net;      // UNet
  const pnp_prior* fallback;   // UNet: prior used where the residual rises (or nullptr)
  int batch, ny, nx;        // UNet: image shape the workspace was sized for
  void* ws;                 // UNet: forward workspace (owned)
};

// Toeplitz embedding of A^H D_w A for one (plan, DCF): the real transfer
// function T[Ky][Kx] on the 2n x 2n grid, pre-scaled by 1/(Kx Ky).
struct pnp_toeplitz {
  const pnp_plan* plan;
  float* T;
};

namespace pnp {

// -------------------------------------------------------- launchers (host)
// Workspace layout of the gridded operator for L coils.
struct OpWorkspace {
  float2* mid;     // [L][rows][Kx]  half-transformed grid (2D) / [L][nz][ny][Kx]... (3D)
  float2* ypart;   // [L][E]         per-entry partial interpolation sums
  float2* ytmp;    // [L][M]         k-space scratch for the normal operator
  float2* yent;    // [L][E]         weighted k-space values in entry order
  float2* part;    // [G][N]         per-coil-group partial images
  float2* g2;      // 3D: [L][nz][Ky][Kx] after the y pass
  float2* grid;    // 3D: [L][Kz][Ky][Kx] full oversampled grid
  float2* ysort;   // 3D: [M][L] k-space values in the plan's sorted sample order
  float2* spart;   // [L][slots][K_y][8] partial strips of the split 2D spread; 3D: [slots][L][512] partial tiles
  size_t bytes;
};
size_t op_workspace_bytes(const pnp_plan* p, int L);
OpWorkspace op_workspace(const pnp_plan* p, int L, void* ws);
// PNP_ERR_UNSUPPORTED when the 2D passes of plan p need more LDS than a
// workgroup has (checked when the plan is created)
void nufft2d_check_plan(const pnp_plan* p);
// 2D adjoint spread: heavy strips are split into parts (kMaxAdjSlots parts
// over all strips at most); adj_build_items rebuilds the plan's work items
// for a split level (0: no split; 1, 2, 3: parts of about 4, 2, 1 times the
// median strip's work) and the dense-block threshold, and waits for `s`
constexpr int kMaxAdjSlots = 32;
void adj_build_items(pnp_plan* p, int split, int dense_min, hipStream_t s);
void plan_set_spread(pnp_plan* p, int split, int dense_min, hipStream_t s);

void op_forward(const pnp_plan* p, const float2* x, const float2* smaps, int L, float2* y,
                const OpWorkspace& w, hipStream_t s);
void op_adjoint(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf,
                float2* x, const OpWorkspace& w, hipStream_t s);
void op_normal(const pnp_plan* p, const float2* x, const float2* smaps, int L, const float* dcf,
               float2* out, const OpWorkspace& w, hipStream_t s);
// Per-coil adjoint images with unit maps: out[l] = A_1^H D_w y_l for l < L
// (ones: the unit map [N]); 2D runs the column pass once for all L coils.
// Workspace: op_workspace(p, L).
void op_adjoint_coils(const pnp_plan* p, const float2* y, int L, const float* dcf, const float2* ones,
                      float2* out, const OpWorkspace& w, hipStream_t s);

// Normal operator as used inside the solver: the input is x, or (when r is
// given) the CG direction p' = r + (*beta) x, which is also stored to pnew;
// the result is left as op_groups(p, L) partial images in w.part ([G][N],
// summed by the consumer).
// Input of the normal operator: the image x, or (cg.r != nullptr) the
// Chronopoulos-Gear CG update, formed per pixel by the operator's first pass:
//   p' = r + beta p,  s' = w + beta s,  u' = u + alpha p',  r' = r - alpha s'
// reading (r, p, s, u, w) and writing (r2, p2, s2, u2); the operator is then
// applied to r'.  One workgroup per pixel writes, so the sets must differ.
struct DevScalars;
// The step sizes of the preceding CG step formed by the pass that consumes
// them, from that step's block sums, instead of by a kernel of their own:
// every wave of the consumer adds the sums in the same order and applies
// the same step rule, so all of them (and the separate finisher) obtain the
// same values; workgroup 0 stores the new state.  parts == nullptr: alpha
// and beta are read from CGUpdate::alpha / beta.
struct CGFinish {
  const double* parts;     // [nparts][2]: block sums of <r, r> and Re<w, r>
  int nparts, first;       // first: the step restarts (beta = 0)
  const DevScalars* prev;  // rr and alpha of the step before (unused when first)
  DevScalars* next;        // receives alpha, beta, rr, pq of this step
  int* bad;                // set to 1 on a non-positive or non-finite denominator
  // fused: the second sums are Re<N r, r> (FusedDots), and
  // Re<w, r> = c0 <r, r> + cg Re<N r, r> is formed here
  int fused;
  float c0, cg;
};
// CG inner products of a step formed by the Toeplitz operator's adjoint row
// pass instead of a pass of their own: its workgroup of image row iy and
// coil group g puts (sum over the row of |r|^2 for g = 0, else 0; sum over
// the row of Re<part_g, r>) into slot g ny + iy of `parts`.
struct FusedDots {
  double* parts;           // [G ny][2]; nullptr: not formed
  const float2* r;         // the operator's input r
  int ny;
};
struct CGUpdate {
  const float2 *r, *p, *s, *u, *w;
  float2 *r2, *p2, *s2, *u2;
  const double *alpha, *beta;
  CGFinish fin;
  // w == nullptr: w = c0 r + cg sum_g part[g N + i] is formed on the fly
  // from the previous operator's coil-group partial images
  const float2* part;
  int G;
  long long N;
  float c0, cg;
  // b0 != nullptr: the CG start instead of a step, r = gamma (b0 - sum_g
  // part[g N + i]) for the image held in u; stores u2 = u, r2 = r and
  // p2 = s2 = 0, and the operator is applied to r (r, p, s, w, fin unused)
  const float2* b0;
  float gamma;
};
struct NormalIn {
  const float2* x;
  CGUpdate cg;
  FusedDots fd;
};
inline NormalIn plain_input(const float2* x) { return NormalIn{x, CGUpdate{}}; }
// Coil groups of the row passes: partial images left in w.part by the
// adjoint and normal operators (ceil(L / coils per workgroup)).
int op_groups(const pnp_plan* p, int L);
// Largest group count any tuning can produce (workspace sizing).
int op_groups_max(int L);
// Coil groups of the batched operator (fixed four coils per workgroup).
int batch_groups(int L);

// ------------------------------------------------ batched Toeplitz operator
// One slice of a batched Toeplitz normal operator (device table entry).
// Supported grids: the register-FFT sizes K = 2n in {128, 192, 256, 512,
// 640, 768, 1024}.
struct BatchSlice {
  int nx, ny, K, L;
  long long N;
  const float2* S;      // [L][N] coil maps
  float2* mid;          // [L][ny][K] half-transformed grid
  float2* part;         // [G][N] coil-group partial images
  const float* T;       // [K][K] transfer function
  const float2* tw;     // K-point twiddles of the slice's plan
};
bool batch_grid_supported(int K);
// Stage launches over the work items int4 {slice, a, b, 0} of all slices
// with grid size K (one workgroup per item):
//   rows passes: a = image row, b = coil group;  column pass: a = strip, b = coil.
// `ins` (device, one per slice) is each slice's operator input.
void batch_rows_fwd(int K, const BatchSlice* sl, const NormalIn* ins, const int4* items, int n_items,
                    hipStream_t s);
void batch_cols_toep(int K, const BatchSlice* sl, const int4* items, int n_items, hipStream_t s);
void batch_rows_adj(int K, const BatchSlice* sl, const int4* items, int n_items, hipStream_t s);
void op_normal_parts(const pnp_plan* p, const NormalIn& in, const float2* smaps, int L,
                     const float* dcf, const OpWorkspace& w, hipStream_t s);

// Toeplitz normal operator (2D, register-FFT grid sizes): same contract as
// op_normal_parts / op_normal, with D_w folded into T.
bool toeplitz_supported(const pnp_plan* p);
pnp_toeplitz* toeplitz_create(const pnp_plan* p, const float* traj, const float* dcf, hipStream_t s);
void toeplitz_destroy(pnp_toeplitz* tp);
// The 2D Toeplitz operator on the register-FFT passes forms a CG step's
// inner products in its row passes when NormalIn::fd asks for them.
bool toep_fused_dots(const pnp_toeplitz* tp);
void op_normal_toep_parts(const pnp_toeplitz* tp, const NormalIn& in, const float2* smaps, int L,
                          const OpWorkspace& w, hipStream_t s);
void op_normal_toep(const pnp_toeplitz* tp, const float2* x, const float2* smaps, int L, float2* out,
                    const OpWorkspace& w, hipStream_t s);

int64_t image_size(const pnp_plan* p);

// Haar prior
void wavelet_apply(int ndim, const int* n_xyz, int levels, float tau, const float2* in, float2* out,
                   hipStream_t s);
// The same prior applied to the last CG update u + alpha (r + beta p), with
// alpha and beta formed from the step's block sums (fin)
void wavelet_apply_cg(int ndim, const int* n_xyz, int levels, float tau, const float2* r, const float2* p,
                      const float2* u, const CGFinish& fin, float2* out, hipStream_t s);
int wavelet_default_levels(int nmin);
// Batched 2D Haar prior over slices (device table, ordered by block0; the
// slices' blocks 0 .. nx*ny/4^J - 1 are numbered from block0 on).
struct HaarSlice {
  const float2* in;
  float2* out;
  int nx, ny;
  int block0;
};
void wavelet_apply_batched(const HaarSlice* sl, int n_slices, int total_blocks, int levels, float tau,
                           hipStream_t s);

// UNet (learned prior)
long long unet_param_count();
long long unet_real_param_count();
int unet_layer_count();
void unet_layer_info(int i, pnp_unet_layer* out);
size_t unet_ws_bytes(int B, int H, int W, bool train);
pnp_unet* unet_create(const float* params, hipStream_t s);
void unet_destroy(pnp_unet* net);
void unet_set(pnp_unet* net, int which, const float* src, hipStream_t s);
void unet_get(pnp_unet* net, int which, float* dst, hipStream_t s);
long long& unet_step(pnp_unet* net);
// out = u + UNet(u, sigma) for a batch of B images H x W; sigma: device [B]
// or nullptr (then sigma_c for every image); out may be nullptr (training).
void unet_forward(const pnp_unet* net, const float2* u, const float* sigma, float sigma_c, int B, int H, int W,
                  float2* out, void* ws, hipStream_t s);
void unet_backward(pnp_unet* net, const float2* u, const float2* target, int B, int H, int W, double* loss,
                   void* ws, hipStream_t s);
void unet_adam(pnp_unet* net, double lr, double b1, double b2, double eps, hipStream_t s);
size_t unet_n2n_ws_bytes(int B, int H, int W);
void unet_n2n_backward(pnp_unet* net, const float2* x, const uint8_t* codes, double eta, int B, int H, int W,
                       double* loss, void* ws, hipStream_t s);
void unet_tensor(int B, int H, int W, bool train, void* ws, int id, void** ptr, int32_t dims[4]);
// 3D operator (register-FFT grid sizes on every axis)
bool plan3_supported(const pnp_plan* p);
int op3_groups(int L);
size_t op3_workspace_bytes(const pnp_plan* p, int L);
OpWorkspace op3_workspace(const pnp_plan* p, int L, void* ws);
void op3_forward(const pnp_plan* p, const float2* x, const float2* smaps, int L, float2* y, const OpWorkspace& w,
                 hipStream_t s);
void op3_adjoint(const pnp_plan* p, const float2* y, const float2* smaps, int L, const float* dcf, float2* x,
                 const OpWorkspace& w, hipStream_t s);
void op3_normal_parts(const pnp_plan* p, const NormalIn& in, const float2* smaps, int L, const float* dcf,
                      const OpWorkspace& w, hipStream_t s);
void op3_normal_toep_parts(const pnp_toeplitz* tp, const NormalIn& in, const float2* smaps, int L,
                           const OpWorkspace& w, hipStream_t s);

// autotuning
void autotune(pnp_plan* p, const float2* smaps, int L, const float* dcf, const pnp_toeplitz* tp,
              const char* cache_path, pnp_tuning* out, hipStream_t s);
void plan_set_row_coils(pnp_plan* p, int fwd, int adj);

// batched slices
pnp_batch* batch_create(int B, const pnp_slice* sl, hipStream_t s);
void batch_destroy(pnp_batch* b);
void batch_normal(pnp_batch* b, const float2* const* x, float2* const* out, hipStream_t s);
size_t batch_unet_ws_bytes(const pnp_batch* b);
void batch_hqs_solve(pnp_batch* b, const pnp_prior* prior, const double* sigmas, int n_out, int precond, int n_cg,
                     void* unet_ws, double* rho_host, int* bad_host, hipStream_t s);
// Apply any prior to an image of the plan's shape (u and x may alias for the wavelet only).
void prior_apply(const pnp_prior* prior, int ndim, const int* n_xyz, const float2* u, float2* x, double sigma,
                 hipStream_t s);

// plan
pnp_plan* plan_create(int ndim, const int32_t* shape, int64_t M, const float* traj, hipStream_t s);
void plan_destroy(pnp_plan* p);

// solver
size_t hqs_workspace_bytes(const pnp_plan* p, int L);
size_t opnorm_workspace_bytes(const pnp_plan* p, int L);
double power_iteration(const pnp_plan* p, const pnp_toeplitz* tp, const float2* smaps, int L,
                       const float* dcf, int iters, uint64_t seed, void* ws, hipStream_t s);

struct HQSArgs {
  const float2* y;
  const float2* smaps;
  int L;
  const float* dcf;
  const pnp_prior* prior;
  const double* sigmas;   // host [n_out]
  int n_out;
  int precond;
  int n_cg;
  double lambda;
  double opnorm;
  const float2* x0;
  float2* x_out;
  const pnp_toeplitz* toep;   // nullptr: gridded normal operator
  double rise_tol;            // fallback test of a prior that has a fallback
};
// Runs the loop; when rho_host is given, also the final residual, and waits.
// fb_host [n_out] (or nullptr) receives 1 where the fallback prior ran.
void hqs_solve(const pnp_plan* p, const HQSArgs& a, void* ws, hipStream_t s, double* rho_host,
               int* bad_host, int* fb_host);

// coil sensitivity maps from the k-space centre
size_t smaps_workspace_bytes(const pnp_plan* p);
void smaps_estimate(const pnp_plan* p, const float2* y, int L, const float* dcf, double width, double threshold,
                    float2* out, void* ws, hipStream_t s);

// PnP-PGD (Sec. 3.3): u = x - gamma P (N x - b0), x = D_{sigma_k}(u)
struct PGDArgs {
  const float2* y;
  const float2* smaps;
  int L;
  const float* dcf;
  const pnp_prior* prior;
  const double* sigmas;   // host [n_iter]
  int n_iter;
  int precond;
  double gamma;
  double opnorm;
  const float2* x0;
  float2* x_out;
  const pnp_toeplitz* toep;
};
void pgd_solve(const pnp_plan* p, const PGDArgs& a, void* ws, hipStream_t s);

// FISTA on f + lam ||detail(Psi x)||_1 (orthonormal Haar)
struct FISTAArgs {
  const float2* y;
  const float2* smaps;
  int L;
  const float* dcf;
  int levels;       // 0: the default rule
  double lam;
  double gamma;
  int n_iter;
  const float2* x0;
  float2* x_out;
  const pnp_toeplitz* toep;
};
void fista_wavelet(const pnp_plan* p, const FISTAArgs& a, void* ws, hipStream_t s);

}  // namespace pnp
