// Ewald correction from the FP64 table (Sec. 2.2.5, second approach): the
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

// The stored second derivatives of phi_c at the grid point nearest to the
// folded offset u (xx, yy, zz, xy, xz, yz; the positive octant's signs).
__device__ inline void table_hessian64(const EwaldP &E, const double u[3], double h[6]) {
  int g[3];
  for (int k = 0; k < 3; ++k) {
    int gi = (int)floor(u[k] / E.step[k] + 0.5);
    g[k] = gi > E.n - 1 ? E.n - 1 : gi;
  }
  const double *T = E.tab64 + 10 * (((int64_t)g[2] * E.n + g[1]) * E.n + g[0]);
  for (int c = 0; c < 6; ++c) h[c] = T[4 + c];
}

// Beyond the far-field switch (2P1I |dz| > zfar, 1P2I sqrt(dy^2 + dz^2) >
// zfar) the correction is the analytic limit minus the Newtonian kernel, whose
// second derivatives are (3 d_j d_k - r^2 delta_jk) / r^5: writes the ten
// channels (phi_c, A_c, H_c; signed) to o and returns true, else false.
__device__ inline bool far_field10(const EwaldP &E, double dx, double dy, double dz, double o[10]) {
  const bool far2 = E.bctype == 2 && fabs(dz) > E.zfar;
  const bool far3 = E.bctype == 3 && dy * dy + dz * dz > E.zfar * E.zfar;
  if (!far2 && !far3) return false;
  const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2), r3 = r2 * r, r5 = r3 * r2;
  const double v[3] = {dx, dy, dz};
  double N[6];
  const int jj[6] = {0, 1, 2, 0, 0, 1}, kk[6] = {0, 1, 2, 1, 2, 2};
  for (int c = 0; c < 6; ++c) N[c] = (3.0 * v[jj[c]] * v[kk[c]] - (jj[c] == kk[c] ? r2 : 0.0)) / r5;
  if (far2) {
    // phi = a |dz| + b: linear, no second derivatives
    o[0] = E.far_phi_a * fabs(dz) + E.far_phi_b - 1.0 / r;
    o[1] = -dx / r3;
    o[2] = -dy / r3;
    o[3] = (dz < 0 ? -E.far_az : E.far_az) - dz / r3;
    for (int c = 0; c < 6; ++c) o[4 + c] = -N[c];
  } else {
    // phi = a ln(rho^2) + b: d^2/dy^2 = 2a (rho^2 - 2 y^2) / rho^4, d^2/dydz = -4a y z / rho^4
    const double rho2 = dy * dy + dz * dz, rho4 = rho2 * rho2, fa = E.far_phi_a;
    o[0] = fa * log(rho2) + E.far_phi_b - 1.0 / r;
    o[1] = -dx / r3;
    o[2] = E.far_az * dy / rho2 - dy / r3;
    o[3] = E.far_az * dz / rho2 - dz / r3;
    o[4] = -N[0];
    o[5] = 2.0 * fa * (rho2 - 2.0 * dy * dy) / rho4 - N[1];
    o[6] = 2.0 * fa * (rho2 - 2.0 * dz * dz) / rho4 - N[2];
    o[7] = -N[3];
    o[8] = -N[4];
    o[9] = -4.0 * fa * dy * dz / rho4 - N[5];
  }
  return true;
}

}  // namespace ot
