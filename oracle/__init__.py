"""FP64 CPU oracle for the non-Cartesian PnP-HQS reconstruction hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously
correct reference that the GPU library is checked against.  Only the test
suite, the entry point's smoke check and the benchmark's CPU-baseline leg may
import it.  The product path (the HIP library and its Python binding) never
imports, links or calls anything here, and this package never imports the
product.  The two share only the seeded input generators in ``synth``, which
hold none of the method's arithmetic.

Modules (each function cites the passage of the paper it follows):
* ``ndft``     exact multicoil non-uniform DFT  A, A^H and A^H D_w A  (Eq. 1)
* ``gridding`` independent FP64 Kaiser-Bessel gridding reference and the
               exact per-sample alias response (used only to pin ``ndft`` and
               to predict the approximation error of any KB-gridded operator)
* ``wavelet``  orthonormal Haar transform and complex soft-threshold prior
* ``solver``   power iteration, the F-1 / Chebyshev / identity
               preconditioners, the fixed-step CG prox, annealed PnP-HQS,
               PnP-PGD, the data-consistency residual
* ``metrics``  PSNR (magnitude, ROI) and SSIM
* ``unet``     FP64 UNet reference with the GPU's BF16 rounding points

Numerics: float64 / complex128 throughout.  Inputs given as float32 or
complex64 are promoted without rounding.
"""
