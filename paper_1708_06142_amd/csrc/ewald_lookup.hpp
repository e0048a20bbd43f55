// Ewald correction from the FP64 table (Sec. 2.2.4, second approach): the
// value and gradient at the nearest grid point of the folded domain plus the
// first-order Taylor term, with the stored Hessian for the acceleration.
#pragma once
#include "kernels.hpp"

namespace ot {

// u: folded offset (all components >= 0).  phic = phi_c(u), a = A_c(u) in the
// positive octant; the caller restores the signs of the components.
__device__ inline void table_taylor64(const EwaldP &E, const double u[3], double &phic, double a[3]) {
  int g[3];
  double dl[3];
  for (int k = 0; k < 3; ++k) {
    int gi = (int)floor(u[k] / E.step[k] + 0.5);
    gi = gi > E.n - 1 ? E.n - 1 : gi;
    g[k] = gi;
    dl[k] = u[k] - gi * E.step[k];
  }
  const double *T = E.tab64 + 10 * (((int64_t)g[2] * E.n + g[1]) * E.n + g[0]);
  phic = T[0] - (T[1] * dl[0] + T[2] * dl[1] + T[3] * dl[2]);
  a[0] = T[1] - (T[4] * dl[0] + T[7] * dl[1] + T[8] * dl[2]);
  a[1] = T[2] - (T[7] * dl[0] + T[5] * dl[1] + T[9] * dl[2]);
  a[2] = T[3] - (T[8] * dl[0] + T[9] * dl[1] + T[6] * dl[2]);
}

}  // namespace ot
