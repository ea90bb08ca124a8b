// Prints the sizes and field offsets of the ABI structs as the C header
// lays them out, for comparison with the ctypes binding (host build only).
#include <cstddef>
#include <cstdio>

#include "pnpmri.h"

#define OFF(T, f) std::printf(#T "." #f " %zu\n", offsetof(T, f))

int main() {
  std::printf("pnp_hqs_opts %zu\n", sizeof(pnp_hqs_opts));
  OFF(pnp_hqs_opts, precond);
  OFF(pnp_hqs_opts, lambda);
  OFF(pnp_hqs_opts, opnorm_seed);
  OFF(pnp_hqs_opts, x0);
  OFF(pnp_hqs_opts, rise_tol);
  OFF(pnp_hqs_opts, toeplitz);
  OFF(pnp_hqs_opts, k_start);
  std::printf("pnp_hqs_report %zu\n", sizeof(pnp_hqs_report));
  OFF(pnp_hqs_report, rho);
  OFF(pnp_hqs_report, fallback);
  OFF(pnp_hqs_report, opnorm_used);
  std::printf("pnp_slice %zu\n", sizeof(pnp_slice));
  OFF(pnp_slice, L);
  OFF(pnp_slice, opnorm);
  OFF(pnp_slice, x_out);
  std::printf("pnp_tuning %zu\n", sizeof(pnp_tuning));
  OFF(pnp_tuning, time_us);
  OFF(pnp_tuning, row_coils_fwd);
  OFF(pnp_tuning, time_fwd_us);
  OFF(pnp_tuning, spread_split);
  OFF(pnp_tuning, time_spread_us);
  return 0;
}
