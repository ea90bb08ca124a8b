/*
 * pnpmri.h -- C ABI of the MI355X (gfx950) non-Cartesian MRI PnP-HQS library.
 *
 * The library computes the multicoil non-Cartesian forward model of the
 * paper "Robust Plug-and-Play Methods for Highly Accelerated Non-Cartesian
 * MRI Reconstruction" (Sec. 2.1, Eq. 1: y_l = F_Omega S_l x + e_l), its
 * adjoint, the normal operator of the (density-weighted) data term
 * (Sec. 2.2), the F-1 / Chebyshev / identity preconditioned proximal step
 * solved by conjugate gradients (Sec. 3.4) and the annealed PnP-HQS loop
 * (Sec. 3.3) with a Haar soft-threshold prior.
 *
 * Conventions (every entry point)
 *   - Complex data is complex64, interleaved (re, im): pnp_c64, the same
 *     memory layout as torch.complex64.
 *   - Images are row-major with x fastest: [ny][nx] or [nz][ny][nx].  The
 *     shape arrays below list the sizes SLOWEST FIRST (ny, nx) / (nz, ny, nx).
 *     Pixel index i along an axis of size n is the centred coordinate
 *     r = i - n/2.
 *   - Coil maps are [L][image]; k-space data is [L][M] (coil-major).
 *   - The trajectory is float32 [M][d] ordered (kx, ky[, kz]) in radians per
 *     pixel; the operator is 2*pi periodic in k, any finite value is valid.
 *   - Forward operator:  y_l[m] = N^{-1/2} sum_r S_l[r] x[r] exp(-i <k_m, r>)
 *     Adjoint with DCF:  x[r]  = N^{-1/2} sum_l conj(S_l[r]) sum_m w_m y_l[m] exp(+i <k_m, r>)
 *     (orthonormal scaling; w = 1 when dcf is NULL).  Both are evaluated by
 *     Kaiser-Bessel gridding (kernel width 6, oversampling 2, Beatty's beta)
 *     in FP32 with FP64-tabulated coordinates, kernel weights, twiddles and
 *     deapodisation; the relative L2 error against the exact NDFT is about
 *     1e-5 (KB alias error plus FP32 rounding).
 *   - Every pointer argument named *_dev / data array is DEVICE memory owned
 *     by the caller, unless marked "host".  The library never frees or keeps
 *     caller memory beyond the call.  The opaque handles (pnp_plan,
 *     pnp_toeplitz, pnp_prior, pnp_unet, pnp_batch) allocate and own their
 *     device tables -- the plan's sorted sample tables and twiddles, the
 *     transfer function, the UNet weights, moments and the UNet prior's
 *     forward buffers, the batch's work lists -- for the handle's lifetime,
 *     released by the matching destroy.  These are built once per
 *     trajectory, network or slice set; every per-call scratch buffer is the
 *     caller's workspace (or, for pnp_normal_toeplitz_noalloc, the library's
 *     static array).
 *   - The gridding kernel is fixed: Kaiser-Bessel of width 6 at
 *     oversampling 2 with Beatty's beta (13.855); there is no options
 *     struct for it.
 *   - Every compute call is asynchronous on the given HIP stream and enqueues
 *     nothing when it returns an error.  Calls that return host scalars
 *     (pnp_opnorm, pnp_hqs_solve with a report or a computed norm) wait for
 *     the stream before returning; pnp_hqs_solve with a prior that has a
 *     fallback also waits inside its loop (see pnp_prior_unet).
 *   - Workspace: the caller passes device scratch memory of at least the
 *     size the matching *_workspace_bytes query reports (256-byte aligned).
 *   - Errors: every call returns a pnp_status; pnp_last_error() gives a
 *     message for the calling thread's last failure.  Arguments are checked
 *     before anything is enqueued; no C++ exception crosses this ABI.
 *   - Calls on one plan from several streams at once must use separate
 *     workspaces.  A plan is read-only after creation except for its launch
 *     settings (pnp_autotune, pnp_plan_set_row_coils*, pnp_plan_set_spread),
 *     which must not be changed while a call on the plan may still run.
 */
#ifndef PNPMRI_H
#define PNPMRI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } pnp_c64;

typedef int32_t pnp_status;
#define PNP_OK                 0
#define PNP_ERR_ARG           -1   /* NULL pointer or invalid scalar argument  */
#define PNP_ERR_SHAPE         -2   /* unsupported or inconsistent sizes        */
#define PNP_ERR_UNSUPPORTED   -3   /* valid request the library does not serve */
#define PNP_ERR_DEVICE        -4   /* HIP runtime error (text in last_error)   */
#define PNP_ERR_WORKSPACE     -5   /* workspace smaller than required          */
#define PNP_ERR_NUMERIC       -6   /* non-finite input or CG/norm breakdown    */

#define PNP_PRECOND_ID    0        /* P = Id                                  */
#define PNP_PRECOND_F1    1        /* P = 2 - alpha A^H D_w A                 */
#define PNP_PRECOND_CHEB  2        /* P = 4 - (10/3) alpha A^H D_w A          */

/* Message describing the calling thread's most recent failure ("" if none).
 * Valid until the thread's next call into the library. */
const char* pnp_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t pnp_version(void);

/* Kernel tracing (instrumentation, not part of the method).  While enabled
 * (on != 0), every kernel the library launches is bracketed by two HIP
 * events recorded on the kernel's own stream.  pnp_trace_read waits for the
 * recorded events, writes a NUL-terminated JSON object
 *   {"kernel_name": [launch_count, total_milliseconds], ...}
 * into buf (host, len bytes), stores the size needed (including the NUL) in
 * *needed when needed is not NULL, and clears the totals.  buf may be NULL
 * to query the size only (the totals are then lost: query with a large
 * buffer instead).  PNP_ERR_ARG when buf is too small. */
pnp_status pnp_trace_enable(int32_t on);
pnp_status pnp_trace_read(char* buf, size_t len, size_t* needed);

/* ------------------------------------------------------------------ plan */
typedef struct pnp_plan pnp_plan;

/* Plan the gridded operator for one trajectory (Sec. 2.1: F_Omega depends
 * only on the sampling trajectory Omega, so it is planned once and reused by
 * every coil, iteration and slice with that trajectory).
 *   out      host: receives the new handle
 *   ndim     2 or 3
 *   shape    host int32[ndim], slowest first; every size even, 4..1024, and
 *            2*size may only have prime factors 2, 3 and 5 (PNP_ERR_SHAPE
 *            otherwise); 2D grids outside the register-FFT sizes also need
 *            their column strips in LDS, 16 * tile * (2*ny + 1) bytes <= 160 KB
 *            with tile = 8 where it divides 2*nx (sides up to 600 at 8-column
 *            tiles; PNP_ERR_UNSUPPORTED otherwise)
 *   M        number of samples (>= 1)
 *   traj     device float32 [M][ndim], (kx, ky[, kz]) radians per pixel,
 *            all finite (checked; PNP_ERR_NUMERIC otherwise)
 *   stream   stream the set-up kernels run on; the call waits for it.
 * Set-up converts the coordinates to grid units in FP64, tabulates the
 * 6 kernel weights per sample and axis, bins samples into oversampled-grid
 * tiles and builds FFT twiddle and deapodisation tables. */
pnp_status pnp_plan_create(pnp_plan** out, int32_t ndim, const int32_t* shape, int64_t M,
                           const float* traj, hipStream_t stream);
pnp_status pnp_plan_destroy(pnp_plan* plan);

/* Plan facts (host): oversampled grid size per axis (slowest first), number
 * of tiles and tile entries (sample-tile pairs). */
pnp_status pnp_plan_info(const pnp_plan* plan, int32_t* grid_shape, int32_t* n_tiles,
                         int64_t* n_entries);

/* Workspace bytes needed by pnp_forward / pnp_adjoint / pnp_normal /
 * pnp_opnorm for L coils. */
pnp_status pnp_workspace_bytes(const pnp_plan* plan, int32_t L, size_t* bytes);

/* Forward operator A (Eq. 1 without noise): y[L][M] = F_Omega S_l x.
 *   x      device pnp_c64 [N] image;  smaps device pnp_c64 [L][N]
 *   y      device pnp_c64 [L][M] output (fully overwritten) */
pnp_status pnp_forward(const pnp_plan* plan, const pnp_c64* x, const pnp_c64* smaps, int32_t L,
                       pnp_c64* y, void* ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint with density weighting A^H D_w (Sec. 3.4 notation A^H):
 *   y      device pnp_c64 [L][M];  dcf device float [M] or NULL (w = 1)
 *   x      device pnp_c64 [N] output (fully overwritten) */
pnp_status pnp_adjoint(const pnp_plan* plan, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                       const float* dcf, pnp_c64* x, void* ws, size_t ws_bytes, hipStream_t stream);

/* Normal operator of the weighted data term, out = A^H D_w A x (Sec. 3.4).
 * x and out may not alias. */
pnp_status pnp_normal(const pnp_plan* plan, const pnp_c64* x, const pnp_c64* smaps, int32_t L,
                      const float* dcf, pnp_c64* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Operator norm ||A^H D_w A||_2 by `iters` power iterations from a seeded
 * complex Gaussian start (Sec. 3.4: alpha = 1/norm normalises the F-1 and
 * Chebyshev preconditioners).  Norms and Rayleigh quotients in FP64.
 *   norm_out  host double; the call waits for the stream. */
pnp_status pnp_opnorm(const pnp_plan* plan, const pnp_c64* smaps, int32_t L, const float* dcf,
                      int32_t iters, uint64_t seed, double* norm_out, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* ------------------------------------------------------------- Toeplitz */
typedef struct pnp_toeplitz pnp_toeplitz;

/* Toeplitz embedding of the normal operator A^H D_w A (2D and 3D; grid
 * sides in {128, 192, 256, 512, 640, 768, 1024}, i.e. image sides 64, 96,
 * 128, 256, 320, 384, 512).  The normal operator of Sec. 3.4 is a
 * convolution with the point-spread function
 * psf[d] = N^{-1} sum_m w_m exp(+i <k_m, d>); embedded in the 2n x 2n
 * (x 2n) grid it is crop(IFFT(T * FFT(pad(z)))) per coil with a real
 * transfer function T = N^{-1} sum_m w_m prod_axis D(k_m,a - 2 pi j_a/K_a),
 * D the symmetric Dirichlet kernel of the n_a pixel offsets.  T is formed
 * once here, exactly in FP64 (per-axis tables contracted over the samples:
 * (2n)^d * M multiply-adds, about 1.8e13 for a 128^3 volume with 2^20
 * samples), from the plan's trajectory and `dcf` (device float [M] or
 * NULL), then rounded to FP32.  Applying it needs no interpolation and no
 * Kaiser-Bessel approximation.  Allocates the table scratch
 * (8 (Kx+Ky[+Kz]) M bytes) for the duration of the call.  The handle keeps
 * a pointer to `plan`: destroy it first.  The call waits for `stream`. */
pnp_status pnp_toeplitz_create(pnp_toeplitz** out, const pnp_plan* plan, const float* dcf,
                               hipStream_t stream);
pnp_status pnp_toeplitz_destroy(pnp_toeplitz* tp);

/* out = A^H D_w A x through the Toeplitz embedding (same layouts and
 * workspace size as pnp_normal; x and out may not alias). */
pnp_status pnp_normal_toeplitz(const pnp_toeplitz* tp, const pnp_c64* x, const pnp_c64* smaps,
                               int32_t L, pnp_c64* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * Toeplitz normal operator of pnp_normal_toeplitz (same arguments, results
 * bit-identical) without a workspace argument.  Its scratch is a static
 * device array inside the library of pnp_noalloc_scratch_bytes() bytes
 * (64 MiB), one per device, held until the process ends; its address is
 * looked up once per device (at pnp_toeplitz_create, or the first call on a
 * device).  The call allocates nothing.  Requests whose workspace
 * (pnp_workspace_bytes for this plan and L) exceeds the array return
 * PNP_ERR_WORKSPACE before anything is enqueued (a 320 x 320 plan takes up
 * to 16 coils at the clinical sampling; 3D plans rarely fit).  All calls on
 * one device share the array: calls that overlap in time on one device
 * (several streams or host threads) race and give wrong results.  Nothing
 * in the array needs to start at zero. */
pnp_status pnp_noalloc_scratch_bytes(size_t* bytes);
pnp_status pnp_normal_toeplitz_noalloc(const pnp_toeplitz* tp, const pnp_c64* x, const pnp_c64* smaps,
                                       int32_t L, pnp_c64* out, hipStream_t stream);

/* ----------------------------------------------------------------- prior */
typedef struct pnp_prior pnp_prior;

/* Haar soft-threshold prior D_sigma(u): orthonormal Haar analysis with
 * `levels` levels (0: min(4, floor(log2 n) - 3)), complex soft threshold
 * c*max(0, 1 - tau/|c|) of every detail coefficient with tau = kappa*sigma,
 * synthesis.  It is the proximal operator of tau*||details||_1 (Sec. 2.2,
 * Eq. 3's prox definition) and the plug-in denoiser of the plain method. */
pnp_status pnp_prior_wavelet(pnp_prior** out, int32_t levels, double kappa);
pnp_status pnp_prior_destroy(pnp_prior* prior);

/* Apply a prior once: out = D_sigma(in), image of the given shape (slowest
 * first).  in and out may alias.  Image sides must be divisible by
 * 2^levels. */
pnp_status pnp_prior_apply(const pnp_prior* prior, int32_t ndim, const int32_t* shape,
                           const pnp_c64* in, pnp_c64* out, double sigma, hipStream_t stream);

/* ------------------------------------------------------------------ UNet
 * The learned denoiser D_sigma of the plug-and-play prior (Sec. 2.3: a
 * denoiser acting on complex images through their real and imaginary parts
 * as two channels, conditioned on the noise level; Sec. 4.2: trained with a
 * supervised l1 loss and Adam).  Fixed architecture, widths 32/64/128/256:
 *   encoder  per scale two 3x3 convolutions + ReLU, 2x2 max-pool between
 *   decoder  2x2 stride-2 transposed convolution, concatenation [skip, up],
 *            two 3x3 convolutions + ReLU
 *   output   1x1 convolution to 2 channels;  D_sigma(u) = u + output
 * Input channels: Re u, Im u, sigma (a constant map).  Convolutions pad with
 * zeros ('same').  Weights and activations BF16 (round to nearest even),
 * products accumulated in FP32 on the matrix cores, master weights and Adam
 * moments FP32.
 *
 * Parameters are one flat FP32 array of pnp_unet_param_count() floats; layer
 * i (pnp_unet_layer_info) stores its weights at w_offset as
 *   3x3 / 1x1 convolution   W[cout][taps][cin_padded]   (tap = 3*(dy+1)+(dx+1))
 *   transposed convolution  W[cout][4][cin]             (tap = 2*a + b, output
 *                                                          pixel (2i+a, 2j+b))
 * and its bias [cout] at b_offset.  Only the first layer is padded (3 input
 * channels stored as 8); its padding weights must be zero and stay zero.
 * Images are complex64 [B][H][W]; H and W must be multiples of 8. */
typedef struct pnp_unet pnp_unet;

enum { PNP_UNET_CONV3 = 0, PNP_UNET_CONV1 = 1, PNP_UNET_UP = 2 };
enum { PNP_UNET_PARAMS = 0, PNP_UNET_GRAD = 1, PNP_UNET_ADAM_M = 2, PNP_UNET_ADAM_V = 3 };

typedef struct {
  int32_t kind;              /* PNP_UNET_CONV3 / CONV1 / UP                   */
  int32_t cin, cin_padded, cout, taps;
  int64_t w_offset, b_offset;   /* floats into the flat parameter array       */
} pnp_unet_layer;

int32_t pnp_unet_layer_count(void);
int64_t pnp_unet_param_count(void);
pnp_status pnp_unet_layer_info(int32_t i, pnp_unet_layer* out);

/* Create a network on the current device from `params` (device FP32
 * [pnp_unet_param_count()], copied).  Adam moments start at zero, step 0.
 * The network owns its parameter, gradient, moment and BF16 buffers. */
pnp_status pnp_unet_create(pnp_unet** out, const float* params, hipStream_t stream);
pnp_status pnp_unet_destroy(pnp_unet* net);

/* Copy one of the network's FP32 arrays (PNP_UNET_PARAMS / GRAD / ADAM_M /
 * ADAM_V) to or from device memory (gradients can only be read).  Setting
 * the parameters refreshes the BF16 copies.  Used for checkpoint / resume
 * together with the Adam step counter. */
pnp_status pnp_unet_set(pnp_unet* net, int32_t which, const float* src, hipStream_t stream);
pnp_status pnp_unet_get(pnp_unet* net, int32_t which, float* dst, hipStream_t stream);
pnp_status pnp_unet_get_step(const pnp_unet* net, int64_t* step);
pnp_status pnp_unet_set_step(pnp_unet* net, int64_t step);

/* Workspace for a batch of B images H x W; train != 0 adds the gradient
 * buffers needed by pnp_unet_backward. */
pnp_status pnp_unet_workspace_bytes(int32_t B, int32_t H, int32_t W, int32_t train, size_t* bytes);

/* out[b] = D_{sigma[b]}(u[b]) for b < B.  u, out: device complex64
 * [B][H][W] (may not alias); sigma: device float [B].  The activations
 * stay in `ws` for a following pnp_unet_backward on the same inputs. */
pnp_status pnp_unet_forward(const pnp_unet* net, const pnp_c64* u, const float* sigma, int32_t B, int32_t H,
                            int32_t W, pnp_c64* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* l1 training loss of the preceding pnp_unet_forward (same net, inputs and a
 * train-sized ws): loss = mean over the 2BHW real values of
 * |D(u) - target| (device double, overwritten); the gradient of the loss
 * with respect to every parameter replaces the network's gradient array
 * (sign(0) = 0; ReLU'(0) = 0; a max-pool routes to the first maximum in the
 * window order (0,0), (0,1), (1,0), (1,1)). */
pnp_status pnp_unet_backward(pnp_unet* net, const pnp_c64* u, const pnp_c64* target, int32_t B, int32_t H,
                             int32_t W, double* loss, void* ws, size_t ws_bytes, hipStream_t stream);

/* Neighbor2Neighbor training of the network as a restoration model f
 * without noise conditioning (Sec. 3.1; the conditioning channel is 0).
 * For noisy images x [B][H][W] (H, W divisible by 16) and one pair code per
 * 2 x 2 cell (codes device uint8 [B][H/2][W/2], values 0..7, drawn by the
 * caller) the sub-images take, in cell (i, j), the ordered pair of
 * 4-adjacent pixels (offsets (dy, dx) in the cell)
 *   0 (0,0)(0,1)  1 (0,0)(1,0)  2 (0,1)(0,0)  3 (0,1)(1,1)
 *   4 (1,0)(0,0)  5 (1,0)(1,1)  6 (1,1)(0,1)  7 (1,1)(1,0)
 * the first into g1(x), the second into g2(x).  loss (device double) =
 * mean over the 2B(H/2)(W/2) real values of d^2 + eta (d - e)^2 with
 * d = f(g1(x)) - g2(x), e = g1(f(x)) - g2(f(x)), f(x) held constant (no
 * gradient through it); its gradient replaces the network's gradient array
 * (then pnp_unet_adam_step).  ws: pnp_n2n_workspace_bytes. */
pnp_status pnp_n2n_workspace_bytes(int32_t B, int32_t H, int32_t W, size_t* bytes);
pnp_status pnp_n2n_backward(pnp_unet* net, const pnp_c64* x, const uint8_t* codes, double eta, int32_t B,
                            int32_t H, int32_t W, double* loss, void* ws, size_t ws_bytes, hipStream_t stream);

/* One Adam step on the FP32 master weights with the current gradients
 * (bias-corrected moments: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * w -= lr/(1-b1^t) * m / (sqrt(v/(1-b2^t)) + eps)), then the BF16 copies
 * are refreshed.  Increments the step counter t. */
pnp_status pnp_unet_adam_step(pnp_unet* net, double lr, double beta1, double beta2, double eps,
                              hipStream_t stream);

/* Inspection: device address and [B][H][W][C] shape of activation `id` in a
 * workspace sized for (B, H, W, train).  Forward ids 0..18: x0 e1a c1 d1a
 * d1b p1 e2a c2 d2a d2b p2 e3a c3 d3a d3b p3 ba bb out (c* hold [skip, up];
 * out is FP32 [2]); with train, 19..36: the gradients gout gd1b gd1a gc1 gd2b
 * gd2a gc2 gd3b gd3a gc3 gbb gba gp3 ge3a gp2 ge2a gp1 ge1a (BF16). */
pnp_status pnp_unet_tensor(int32_t B, int32_t H, int32_t W, int32_t train, void* ws, int32_t id, void** ptr,
                           int32_t* dims);

/* Learned prior D_sigma(u) = UNet(u, kappa*sigma) for images of `shape`
 * (2D [ny][nx]; 3D [nz][ny][nx] is denoised slice by slice).  With a
 * `fallback` (a wavelet prior), pnp_hqs_solve replaces the UNet output by
 * the fallback's whenever it is not finite or its data-consistency residual
 * rho_k exceeds (1 + opts.rise_tol) rho_{k-1}.  The check reads rho_k on
 * the host from a small pinned buffer (one per host thread, allocated on
 * first use and kept) while the next iteration's CG already runs; a
 * rejection discards that CG and starts it again from the fallback image.
 * Allocates its forward workspace; keeps pointers to `net` and `fallback`
 * (destroy them last). */
pnp_status pnp_prior_unet(pnp_prior** out, const pnp_unet* net, int32_t ndim, const int32_t* shape, double kappa,
                          const pnp_prior* fallback);

/* ------------------------------------------------------------------- HQS */
typedef struct {
  uint32_t struct_size;      /* sizeof(pnp_hqs_opts)                          */
  int32_t precond;           /* PNP_PRECOND_*                                 */
  int32_t n_cg;              /* CG steps per proximal step (>= 1)             */
  int32_t opnorm_iters;      /* power iterations when opnorm <= 0             */
  double lambda;             /* gamma_k = lambda * sigma_k  (> 0)             */
  double opnorm;             /* ||A^H D_w A|| if > 0, else computed           */
  uint64_t opnorm_seed;      /* seed of the power-iteration start vector      */
  const pnp_c64* x0;         /* device [N] start image, NULL: x0 = A^H D_w y  */
  double rise_tol;           /* fallback when rho_k > (1+rise_tol) rho_{k-1}  */
  const pnp_toeplitz* toeplitz;  /* NULL: gridded normal operator; else the
                                    Toeplitz one (built with the same dcf)   */
  int32_t k_start;           /* first outer iteration to run (0 <= k_start <
                                n_out): resume a schedule from x0, e.g. the
                                x_out of an earlier call that stopped at
                                k_start; 0 when struct_size ends before it  */
} pnp_hqs_opts;

typedef struct {
  uint32_t struct_size;      /* sizeof(pnp_hqs_report)                        */
  int32_t capacity;          /* length of the host arrays below (>= n_out)    */
  double* rho;               /* host [n_out]: ||D_w^{1/2}(A x_k - y)||^2      */
  int32_t* fallback;         /* host [n_out]: 1 where the fallback prior ran  */
  double opnorm_used;        /* out: the operator norm used                   */
} pnp_hqs_report;

/* Workspace bytes for pnp_hqs_solve. */
pnp_status pnp_hqs_workspace_bytes(const pnp_plan* plan, int32_t L, size_t* bytes);

/* Annealed preconditioned PnP-HQS (Sec. 3.3-3.4):
 *   b0 = A^H D_w y;  x = x0 (or b0)
 *   for k = k_start..n_out-1:  gamma = lambda*sigma[k]
 *       u = prox^P_{gamma f}(x) by exactly n_cg CG steps on
 *           (gamma A^H D_w A + P) u = P x + gamma b0, started at u = x
 *       x = D_{sigma[k]}(u)
 * with P = c0 - c1 alpha A^H D_w A (Id: 1,0; F-1: 2,1; Chebyshev: 4,10/3),
 * alpha = 1/opnorm.  CG inner products, step sizes and residual norms are
 * FP64 and stay on the device (no host synchronisation inside the loop,
 * except the residual check of a prior with a fallback: the host waits for
 * each rho_k while the next iteration's CG already runs).
 *   y       device pnp_c64 [L][M];  smaps device [L][N];  dcf device [M]|NULL
 *   sigmas  host double [n_out] (positive from k_start on): the whole
 *           schedule; a call with k_start > 0 runs its tail, so splitting a
 *           schedule over several calls (each resuming from the previous
 *           x_out) gives the same iterates as one call
 *   x_out   device pnp_c64 [N]: x_{n_out}
 *   report  host or NULL (its arrays are indexed by the outer iteration k;
 *           entries below k_start are left as they are); when given the
 *           call waits for the stream and
 *           returns PNP_ERR_NUMERIC after a CG breakdown (non-finite or
 *           non-positive <p, Mp>, e.g. from non-finite data).  Without a
 *           report the call stays asynchronous and does not detect a
 *           breakdown: it returns PNP_OK and the breakdown shows only as
 *           non-finite values in x_out. */
pnp_status pnp_hqs_solve(const pnp_plan* plan, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                         const float* dcf, const pnp_prior* prior, const double* sigmas,
                         int32_t n_out, const pnp_hqs_opts* opts, pnp_c64* x_out,
                         pnp_hqs_report* report, void* ws, size_t ws_bytes, hipStream_t stream);

/* Coil sensitivity maps estimated from the centre of k-space (Sec. 4.1: a
 * 20 x 20 Hamming window on the k-space centre, brought to the image domain
 * and masked).  Each sample m is weighted by dcf[m] * prod_axis h(kappa_a),
 * kappa_a = k_a n_a / (2 pi) its frequency in grid units and
 * h(kappa) = 0.54 + 0.46 cos(pi kappa / c) for |kappa| <= c = width/2, else
 * 0; z_l = the adjoint of coil l's weighted data with a unit map;
 * s = sqrt(sum_l |z_l|^2); smaps_out[l] = z_l / s where s > threshold * max s,
 * 0 elsewhere.
 *   y          device pnp_c64 [L][M];  dcf device float [M] or NULL
 *   width      window width in grid units (> 0; 20 for the paper's window)
 *   threshold  mask level as a fraction of max s, in [0, 1) (0: no mask)
 *   smaps_out  device pnp_c64 [L][N] (written, also used as scratch)
 *   ws         pnp_smaps_workspace_bytes bytes.  Asynchronous on `stream`. */
pnp_status pnp_smaps_workspace_bytes(const pnp_plan* plan, size_t* bytes);
pnp_status pnp_smaps_estimate(const pnp_plan* plan, const pnp_c64* y, int32_t L, const float* dcf, double width,
                              double threshold, pnp_c64* smaps_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* PnP-PGD (Sec. 3.3, the preconditioned plug-and-play proximal gradient
 * scheme), one noise level per iteration:
 *   b0 = A^H D_w y;  x = x0 (or b0)
 *   for k = 0..n_iter-1:  u = x - gamma P (A^H D_w A x - b0);  x = D_{sigma[k]}(u)
 * with P = c0 - c1 alpha A^H D_w A as in pnp_hqs_solve (alpha = 1/opnorm,
 * opnorm > 0 required unless precond is PNP_PRECOND_ID).  One normal
 * operator per iteration with P = Id, two otherwise.  A UNet prior is
 * applied without its fallback.
 *   y, smaps, dcf, x0, x_out as in pnp_hqs_solve;  sigmas host double [n_iter]
 *   toeplitz  NULL: gridded normal operator; else the Toeplitz one
 *   ws        the pnp_hqs_workspace_bytes workspace.  Asynchronous on `stream`. */
pnp_status pnp_pgd_solve(const pnp_plan* plan, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                         const float* dcf, const pnp_prior* prior, const double* sigmas, int32_t n_iter,
                         double gamma, int32_t precond, double opnorm, const pnp_toeplitz* toeplitz,
                         const pnp_c64* x0, pnp_c64* x_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* FISTA-Wavelet (the wavelet baseline of Table 1): FISTA (Beck and Teboulle
 * 2009) on f(x) + lam ||detail(Psi x)||_1, Psi the orthonormal Haar
 * transform with `levels` levels (0: the default rule), only detail bands
 * penalised:
 *   z = x = x0 (or b0), t = 1
 *   for k: x' = soft_{gamma lam}(z - gamma (A^H D_w A z - b0))
 *          t' = (1 + sqrt(1 + 4 t^2)) / 2;  z = x' + ((t - 1)/t') (x' - x);  x = x', t = t'
 * gamma > 0 is the step (convergent for gamma <= 1/||A^H D_w A||), lam >= 0.
 * Arguments and workspace as in pnp_pgd_solve; x_out receives x_{n_iter}. */
pnp_status pnp_fista_wavelet(const pnp_plan* plan, const pnp_c64* y, const pnp_c64* smaps, int32_t L,
                             const float* dcf, int32_t levels, double lam, double gamma, int32_t n_iter,
                             const pnp_toeplitz* toeplitz, const pnp_c64* x0, pnp_c64* x_out, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ autotuning
 * The register-FFT row passes of a 2D plan handle 2, 4 or 8 coils per
 * workgroup, chosen separately for the forward (image -> grid) and the
 * adjoint (grid -> image) pass; both default to 4.  pnp_autotune times the
 * normal operator the caller will run -- Toeplitz when `toeplitz` is given,
 * else the gridded one with `dcf` -- on this device (after a warm-up, in
 * interleaved rounds): first each adjoint choice with the forward one at 4,
 * then each forward choice with the adjoint one fixed.  Each keeps the
 * default 4 unless another choice is more than 2% faster.  It then times
 * the gridded adjoint (with `dcf`) for the 12 spread settings of
 * pnp_plan_set_spread and keeps the default unless another is more than 2%
 * faster.  The choices are
 * stored in the plan and appended to the JSON-lines file `cache_path`
 * (NULL: no cache), keyed by device, image shape, L, M, a hash of the
 * histogram of gridding entries per column strip, and the operator kind.  A
 * cached key is applied without timing.  Allocates and frees temporary
 * device memory; waits for `stream`.  Workspaces sized by the query
 * functions fit every choice.  2D plans only (PNP_ERR_UNSUPPORTED else).
 *
 * pnp_plan_set_row_coils sets both passes to one value;
 * pnp_plan_get_row_coils returns the adjoint pass's value (which also sets
 * the number of coil groups of the partial images); the _pair forms set and
 * get the two separately.  Values other than 2, 4, 8: PNP_ERR_ARG.  Every
 * choice gives the same results up to floating-point summation order. */
typedef struct {
  uint32_t struct_size;      /* sizeof(pnp_tuning)                            */
  int32_t row_coils;         /* out: chosen coils per workgroup, adjoint pass */
  double time_us[3];         /* out: operator time, adjoint 2, 4, 8 (0 if cached) */
  int32_t from_cache;        /* out: 1 when the choice came from the cache    */
  int32_t row_coils_fwd;     /* out: chosen coils per workgroup, forward pass */
  double time_fwd_us[3];     /* out: operator time, forward 2, 4, 8 (0 if cached) */
  int32_t spread_split;      /* out: chosen split level of the adjoint spread */
  int32_t spread_dense_min;  /* out: chosen dense-block threshold            */
  double time_spread_us[12]; /* out: gridded adjoint time for split 0..3 x
                                threshold 128, 256, 512 (0 if cached)        */
} pnp_tuning;

pnp_status pnp_autotune(pnp_plan* plan, const pnp_c64* smaps, int32_t L, const float* dcf,
                        const pnp_toeplitz* toeplitz, const char* cache_path, pnp_tuning* out,
                        hipStream_t stream);
/* The type-1 spread of the 2D adjoint (the column pass that gathers the
 * weighted samples into each 8-column strip of the oversampled grid before
 * its inverse FFT) runs one workgroup per strip, except that the strips
 * with the most work (the k-space centre; 32 parts in all at most) are
 * split into up to 8 parts, part p taking every P-th chunk of the strip's
 * entries; each part is a workgroup of its own, and the parts' partial
 * strips are added in part order before the strip's inverse FFT.  `split`
 * 0 never splits; 1, 2, 3 aim at parts of about 4, 2 and 1 times the median
 * strip's work.  Row blocks whose window holds
 * `dense_min` or more entries are shared by all waves of their workgroup.
 * Defaults: split 1, dense_min 128; pnp_autotune sweeps split 0..3 x
 * dense_min 128, 256, 512 on the gridded adjoint.  Every choice gives the
 * same results up to floating-point summation order.  2D plans only;
 * pnp_plan_set_spread waits for `stream`. */
pnp_status pnp_plan_set_spread(pnp_plan* plan, int32_t split, int32_t dense_min, hipStream_t stream);
pnp_status pnp_plan_get_spread(const pnp_plan* plan, int32_t* split, int32_t* dense_min);
pnp_status pnp_plan_set_row_coils(pnp_plan* plan, int32_t row_coils);
pnp_status pnp_plan_get_row_coils(const pnp_plan* plan, int32_t* row_coils);
pnp_status pnp_plan_set_row_coils_pair(pnp_plan* plan, int32_t forward, int32_t adjoint);
pnp_status pnp_plan_get_row_coils_pair(const pnp_plan* plan, int32_t* forward, int32_t* adjoint);

/* ------------------------------------------------------- batched slices
 * Many independent 2D slices (different sizes, coil counts and trajectories)
 * reconstructed together with the same schedule (Sec. 3.3-3.4 per slice).
 * Each stage of the Toeplitz normal operator runs as one launch per image
 * size over the work items of all slices of that size; CG
 * reductions are per slice (FP64, on the device); the Haar prior is one
 * launch over all slices and the UNet prior one batched forward per image
 * size.  Supported: square images with n in {64, 96, 128, 256, 320, 384,
 * 512} and one Haar depth for all slices. */
typedef struct {
  const pnp_plan* plan;          /* the slice's plan (2D, square)              */
  const pnp_toeplitz* toeplitz;  /* its Toeplitz embedding (built with `dcf`)  */
  const pnp_c64* y;              /* device [L][M] k-space data                 */
  const pnp_c64* smaps;          /* device [L][n][n]                           */
  int32_t L;
  const float* dcf;              /* device [M] or NULL                         */
  double opnorm;                 /* ||A^H D_w A|| of the slice (> 0)           */
  double lambda;                 /* gamma_k = lambda * sigma_k (> 0)           */
  pnp_c64* x_out;                /* device [n][n] result                       */
} pnp_slice;

typedef struct pnp_batch pnp_batch;

/* Build the batch (work lists, per-slice tables, workspace; one device
 * allocation owned by the batch).  Keeps the slices' pointers: the plans,
 * Toeplitz handles and arrays must outlive the batch.  Waits for `stream`. */
pnp_status pnp_batch_create(pnp_batch** out, int32_t B, const pnp_slice* slices, hipStream_t stream);
pnp_status pnp_batch_destroy(pnp_batch* batch);

/* out[i] = A_i^H D_w A_i x[i] for every slice (Toeplitz operator, three
 * launches per image size plus one coil-group sum).  x, out: host arrays of B
 * device pointers (each [n_i][n_i]).  Waits for `stream`. */
pnp_status pnp_batch_normal(pnp_batch* batch, const pnp_c64* const* x, pnp_c64* const* out, hipStream_t stream);

/* Workspace bytes pnp_hqs_solve_batched needs for `prior` (0 for a wavelet prior). */
pnp_status pnp_batch_workspace_bytes(const pnp_batch* batch, const pnp_prior* prior, size_t* bytes);

/* Annealed PnP-HQS of every slice (pnp_hqs_solve per slice, started at
 * x0 = A^H D_w y, fallback not available): sigmas host [n_out], precond
 * PNP_PRECOND_*, n_cg >= 1.  prior: a wavelet prior (its depth must be the
 * slices' default) or a UNet prior (its network and kappa are used; its
 * shape is ignored).  rho: host [B][n_out] residuals of x_k, or NULL (the
 * call then returns without waiting). */
pnp_status pnp_hqs_solve_batched(pnp_batch* batch, const pnp_prior* prior, const double* sigmas, int32_t n_out,
                                 int32_t precond, int32_t n_cg, double* rho, void* ws, size_t ws_bytes,
                                 hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PNPMRI_H */
