// Device-resident scalar state of the CG proximal solver and power
// iteration, and the scalar updates that close a CG reduction.
#pragma once

#include "common.hpp"

namespace pnp {

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
};

// Chronopoulos-Gear step sizes from g = <r,r> and d = Re<M r, r>:
//   first step:  beta = 0, alpha = g / d
//   later steps: beta = g / rr, alpha = g / (d - beta g / alpha)
// then rr = g.  A zero residual gives alpha = beta = 0; a non-positive or
// non-finite denominator sets `bad` and alpha = beta = 0 (u stops moving).
__device__ inline void cg_finish_dots(DevScalars* sc, double g, double d, int first) {
  double alpha = 0.0, beta = 0.0;
  if (g > 0.0 && isfinite(g)) {
    const bool restart = first || !(sc->alpha != 0.0) || !(sc->rr > 0.0);
    beta = restart ? 0.0 : g / sc->rr;
    const double den = restart ? d : d - beta * g / sc->alpha;
    if (den > 0.0 && isfinite(den)) {
      alpha = g / den;
    } else {
      beta = 0.0;
      sc->bad = 1;
    }
  } else if (!isfinite(g)) {
    sc->bad = 1;
  }
  sc->pq = d;
  sc->alpha = alpha;
  sc->beta = beta;
  sc->rr = g;
}

// CG start: rr = <r0,r0>; rho(x) = <x,Nx> - 2 Re<x,b0> + ||y||_w^2.
__device__ inline void cg_finish_init(DevScalars* sc, double rr, double xnx, double xb0, double* rho_out) {
  sc->rr = rr;
  if (rho_out) *rho_out = xnx - 2.0 * xb0 + sc->yw2;
}

}  // namespace pnp
