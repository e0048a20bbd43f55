// Ewald correction table, FP64 on the device (Sec. 2.2.3-2.2.5, App. A).
//
// For every point u of a uniform grid over the folded domain the kernel sums
// the series of phi (3P: Eq. 9 with the cut-offs of Eq. 10; 2P1I: Eq. 15 in
// the code form of its footnote) with the Newtonian 1/r removed from the
// central image, and their analytic first and second derivatives:
//   channel 0: phi_c = phi - 1/r
//   1..3     : A_c = -grad phi_c
//   4..9     : H = grad grad phi_c (xx, yy, zz, xy, xz, yz)
// The 2P1I z-integral uses Itilde = pi/(2s) [exp(-g^2/4z - z s^2) erfcx(A+)
// + exp(-g s) erfc(A-)] with A+- = sqrt(z) s +- g/(2 sqrt(z)), evaluated at
// |gamma| (even; the first derivative is odd), and the regularised l = 0 term
// I(0,0) of Eq. 14.
// 1P2I (periodic along x): the images along x in real space and, in Fourier
// space, 2/Lx sum_l exp(-zeta l^2) cos(kappa l dx) K(l, eta), eta = kappa rho,
// rho = sqrt(dy^2 + dz^2) (Sec. 2.2.4; App. A for the acceleration).
#include "common.hpp"
#include "ewald_lookup.hpp"
#include "kernels.hpp"

namespace ot {

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double SQRTPI = 1.7724538509055160273;

struct Radial {
  double f, D1, D2;  // value, f'/r, (f'/r)'/r
};

// erfc(alpha r)/r
__device__ inline Radial erfc_term(double a, double r) {
  const double r2 = r * r;
  const double ex = (2.0 * a / SQRTPI) * exp(-a * a * r2);
  const double ec = erfc(a * r);
  Radial R;
  R.f = ec / r;
  R.D1 = -(ex / r2 + ec / (r2 * r));
  R.D2 = ex * (2.0 * a * a / r2 + 3.0 / (r2 * r2)) + 3.0 * ec / (r2 * r2 * r);
  return R;
}

// -erf(alpha r)/r, the central image with 1/r removed; Taylor series of
// erf(x)/x below x = 0.5 (smooth through r = 0)
__device__ inline Radial erf_corr_term(double a, double r) {
  const double x = a * r;
  Radial R;
  if (x < 0.5) {
    const double c = 2.0 * a / SQRTPI;
    const double x2 = x * x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    double p0 = 1.0, p1 = 0.0, p2 = 0.0;  // x^(2n), x^(2n-2), x^(2n-4)
    double inv_fact = 1.0;
    for (int n = 0; n < 18; ++n) {
      if (n > 0) inv_fact /= n;
      const double an = ((n & 1) ? -inv_fact : inv_fact) / (2 * n + 1);
      s0 += an * p0;
      if (n >= 1) s1 += 2.0 * n * an * p1;
      if (n >= 2) s2 += 2.0 * n * (2.0 * n - 2.0) * an * p2;
      p2 = n >= 1 ? p1 : 0.0;
      p1 = p0;
      p0 *= x2;
    }
    R.f = -c * s0;
    R.D1 = -c * a * a * s1;
    R.D2 = -c * a * a * a * a * s2;
    return R;
  }
  const double r2 = r * r;
  const double ex = (2.0 * a / SQRTPI) * exp(-a * a * r2);
  const double ef = erf(x);
  R.f = -ef / r;
  R.D1 = -ex / r2 + ef / (r2 * r);
  R.D2 = ex * (2.0 * a * a / r2 + 3.0 / (r2 * r2)) - 3.0 * ef / (r2 * r2 * r);
  return R;
}

// 1P2I: K(l, eta), M = -dK/deta, dM/deta and M/eta (dM/deta at eta = 0).
// For l != 0, writing 1/(l^2 + q^2) as int_0^inf exp(-t (l^2 + q^2)) dt and
// using int_0^inf J0(eta q) exp(-p q^2) q dq = exp(-eta^2/(4p))/(2p) turns
// the Bessel integral into
//   K = 1/2 int_0^inf exp(-zeta l^2 (e^s - 1) - b e^-s) ds,  b = eta^2/(4 zeta),
// with M and dM/deta by differentiation under the integral.  The integral is
// taken by the trapezoidal rule after s = e^t, t in [-45, 3] with step 1/32:
// the transformed integrand decays at both ends and is analytic in a strip,
// so the rule converges geometrically.  For l = 0 the regularised closed
// forms: K = -Ein(b)/2, M = (1 - e^-b)/eta, with Ein(b) = E1(b) + ln b + gamma
// (its series below b = 1; above, E1(b) = int_0^inf exp(-b e^w) dw by the same
// rule after w = e^t).
struct KFun {
  double K, M, Mp, Mq;
};

constexpr double EULER_GAMMA = 0.57721566490153286061;
constexpr double DE_T0 = -45.0, DE_H = 1.0 / 32.0;
constexpr int DE_N = 1537;  // t = -45 ... 3

__device__ inline double ein(double b) {
  if (b < 1.0) {
    double term = 1.0, sum = 0.0;
    for (int k = 1; k <= 30; ++k) {
      term *= b / k;
      sum += ((k & 1) ? term : -term) / k;
    }
    return sum;
  }
  double e1 = 0.0;
  for (int i = 0; i < DE_N; ++i) {
    const double w = exp(DE_T0 + i * DE_H);
    e1 += exp(-b * exp(w)) * w;
  }
  return DE_H * e1 + log(b) + EULER_GAMMA;
}

__device__ inline KFun kfun(int l, double eta, double zeta) {
  KFun F;
  const double b = eta * eta / (4.0 * zeta);
  if (l == 0) {
    const double om = -expm1(-b);
    F.K = -0.5 * ein(b);
    F.M = eta > 0.0 ? om / eta : 0.0;
    F.Mq = b > 0.0 ? om / b / (4.0 * zeta) : 1.0 / (4.0 * zeta);
    F.Mp = exp(-b) / (2.0 * zeta) - F.Mq;
    return F;
  }
  const double a = zeta * l * l, c = eta / (2.0 * zeta), c0 = 1.0 / (2.0 * zeta);
  double sk = 0.0, sm = 0.0, sp = 0.0;
  for (int i = 0; i < DE_N; ++i) {
    const double sg = exp(DE_T0 + i * DE_H);
    const double em = exp(-sg);
    const double f = exp(-a * expm1(sg) - b * em) * sg;
    sk += f;
    sm += f * em;
    sp += f * em * (c0 - c * c * em);
  }
  F.K = 0.5 * DE_H * sk;
  F.M = 0.5 * DE_H * c * sm;
  F.Mp = 0.5 * DE_H * sp;
  F.Mq = eta > 0.0 ? F.M / eta : F.Mp;
  return F;
}

struct Acc10 {
  double v[10];
};

__device__ inline void add_radial(const Radial &R, double x, double y, double z, Acc10 &o) {
  o.v[0] += R.f;
  o.v[1] -= R.D1 * x;
  o.v[2] -= R.D1 * y;
  o.v[3] -= R.D1 * z;
  o.v[4] += R.D2 * x * x + R.D1;
  o.v[5] += R.D2 * y * y + R.D1;
  o.v[6] += R.D2 * z * z + R.D1;
  o.v[7] += R.D2 * x * y;
  o.v[8] += R.D2 * x * z;
  o.v[9] += R.D2 * y * z;
}

// phi_c, A_c and the Hessian of phi_c at folded offset u (all components >= 0)
__device__ inline void ewald_point(const EwaldP &E, double alpha, int rcut2, int fcut2, const double u[3],
                                   Acc10 &o) {
  const double Lx = E.L[0], b = E.L[1] / E.L[0], c = E.L[2] / E.L[0];
  const double zeta = (PI * PI) / ((alpha * Lx) * (alpha * Lx));
  const bool three = E.bctype == 1, onep = E.bctype == 3;
  for (int k = 0; k < 10; ++k) o.v[k] = 0.0;

  const double rr = sqrt((double)rcut2);
  const int R1 = (int)ceil(rr) + 1, R2 = onep ? 0 : (int)ceil(rr / b) + 1, R3 = three ? (int)ceil(rr / c) + 1 : 0;
  for (int i3 = -R3; i3 <= R3; ++i3)
    for (int i2 = -R2; i2 <= R2; ++i2)
      for (int i1 = -R1; i1 <= R1; ++i1) {
        const double qq = (double)(i1 * i1) + (b * i2) * (b * i2) + (c * i3) * (c * i3);
        if (qq > rcut2) continue;
        const double x = u[0] - i1 * Lx, y = u[1] - i2 * b * Lx, z = u[2] - i3 * c * Lx;
        const double r = sqrt(x * x + y * y + z * z);
        if (i1 == 0 && i2 == 0 && i3 == 0) {
          add_radial(erf_corr_term(alpha, r), x, y, z, o);
        } else {
          add_radial(erfc_term(alpha, r), x, y, z, o);
        }
      }

  const double fr = sqrt((double)fcut2);
  const int F1 = (int)ceil(fr) + 1, F2 = (int)ceil(fr * b) + 1, F3 = (int)ceil(fr * c) + 1;
  const double kap = 2.0 * PI / Lx;
  if (three) {
    const double pre = 1.0 / (PI * b * c * Lx);
    for (int l3 = -F3; l3 <= F3; ++l3)
      for (int l2 = -F2; l2 <= F2; ++l2)
        for (int l1 = -F1; l1 <= F1; ++l1) {
          if (l1 == 0 && l2 == 0 && l3 == 0) continue;
          const double q0 = l1, q1 = l2 / b, q2 = l3 / c;
          const double Q = q0 * q0 + q1 * q1 + q2 * q2;
          if (Q > fcut2) continue;
          const double Ew = exp(-zeta * Q) / Q;
          double sv, cv;
          sincos(kap * (q0 * u[0] + q1 * u[1] + q2 * u[2]), &sv, &cv);
          const double hk = -pre * kap * kap * Ew * cv;
          o.v[0] += pre * Ew * cv;
          o.v[1] += pre * kap * q0 * Ew * sv;
          o.v[2] += pre * kap * q1 * Ew * sv;
          o.v[3] += pre * kap * q2 * Ew * sv;
          o.v[4] += hk * q0 * q0;
          o.v[5] += hk * q1 * q1;
          o.v[6] += hk * q2 * q2;
          o.v[7] += hk * q0 * q1;
          o.v[8] += hk * q0 * q2;
          o.v[9] += hk * q1 * q2;
        }
  } else if (onep) {
    const double pre = 2.0 / Lx;
    const double rho = sqrt(u[1] * u[1] + u[2] * u[2]);
    const double uy = rho > 0.0 ? u[1] / rho : 0.0, uz = rho > 0.0 ? u[2] / rho : 0.0;
    const double eta = kap * rho;
    for (int l = 0; l * l <= fcut2; ++l) {
      const KFun F = kfun(l, eta, zeta);
      // the terms of l and -l: cos doubles, sin l cancels with the sign of l
      const double w = (l == 0 ? 1.0 : 2.0) * pre * exp(-zeta * l * l);
      double sv, cv;
      sincos(kap * l * u[0], &sv, &cv);
      const double k2 = w * kap * kap;
      const double ar = w * kap * cv * F.M;  // radial component of A
      o.v[0] += w * cv * F.K;
      o.v[1] += w * kap * l * sv * F.K;
      o.v[2] += ar * uy;
      o.v[3] += ar * uz;
      o.v[4] -= k2 * l * l * cv * F.K;
      o.v[5] -= k2 * cv * (F.Mp * uy * uy + F.Mq * (1.0 - uy * uy));
      o.v[6] -= k2 * cv * (F.Mp * uz * uz + F.Mq * (1.0 - uz * uz));
      o.v[7] += k2 * l * sv * F.M * uy;
      o.v[8] += k2 * l * sv * F.M * uz;
      o.v[9] -= k2 * cv * (F.Mp - F.Mq) * uy * uz;
    }
  } else {
    const double pre = 1.0 / (PI * Lx * b);
    const double gam = kap * u[2];  // u[2] >= 0 on the folded grid
    const double sz = sqrt(zeta);
    for (int l2 = -F2; l2 <= F2; ++l2)
      for (int l1 = -F1; l1 <= F1; ++l1) {
        const double q0 = l1, q1 = l2 / b;
        const double Q = q0 * q0 + q1 * q1;
        if (Q > fcut2) continue;
        double I0, I1, I2;
        if (l1 == 0 && l2 == 0) {
          const double e = erf(gam / (2.0 * sz));
          const double gs = exp(-gam * gam / (4.0 * zeta));
          I0 = -PI * (gam * e + 2.0 * sqrt(zeta / PI) * gs) + 2.0 * sqrt(PI * zeta);
          I1 = -PI * e;
          I2 = -(SQRTPI / sz) * gs;
        } else {
          const double s = sqrt(Q);
          const double Ap = sz * s + gam / (2.0 * sz);
          const double Am = sz * s - gam / (2.0 * sz);
          const double gauss = exp(-gam * gam / (4.0 * zeta) - zeta * Q);
          const double E1 = gauss * erfcx(Ap);
          const double E2 = exp(-gam * s) * erfc(Am);
          I0 = PI / (2.0 * s) * (E1 + E2);
          I1 = (PI / 2.0) * (E1 - E2);
          I2 = (PI / 2.0) * (s * (E1 + E2) - 2.0 / sqrt(PI * zeta) * gauss);
        }
        double sv, cv;
        sincos(kap * (q0 * u[0] + q1 * u[1]), &sv, &cv);
        const double k2 = pre * kap * kap;
        o.v[0] += pre * cv * I0;
        o.v[1] += pre * kap * q0 * sv * I0;
        o.v[2] += pre * kap * q1 * sv * I0;
        o.v[3] -= pre * kap * cv * I1;
        o.v[4] -= k2 * q0 * q0 * cv * I0;
        o.v[5] -= k2 * q1 * q1 * cv * I0;
        o.v[6] += k2 * cv * I2;
        o.v[7] -= k2 * q0 * q1 * cv * I0;
        o.v[8] -= k2 * q0 * sv * I1;
        o.v[9] -= k2 * q1 * sv * I1;
      }
  }
}

__global__ __launch_bounds__(128) void k_ewald_table(EwaldP E, double alpha, int rcut2, int fcut2,
                                                     double *__restrict__ tab64,
                                                     float4 *__restrict__ tab32) {
  const int64_t n = E.n;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * n * n) return;
  const int ix = (int)(q % n), iy = (int)((q / n) % n), iz = (int)(q / (n * n));
  const double u[3] = {ix * E.step[0], iy * E.step[1], iz * E.step[2]};
  Acc10 o;
  ewald_point(E, alpha, rcut2, fcut2, u, o);
  double *t = tab64 + 10 * q;
  for (int k = 0; k < 10; ++k) t[k] = o.v[k];
  tab32[3 * q + 0] = make_float4((float)o.v[0], (float)o.v[1], (float)o.v[2], (float)o.v[3]);
  tab32[3 * q + 1] = make_float4((float)o.v[4], (float)o.v[5], (float)o.v[6], (float)o.v[7]);
  tab32[3 * q + 2] = make_float4((float)o.v[8], (float)o.v[9], 0.0f, 0.0f);
}

// FP32 copy of an FP64 table (a table read from a cache file)
__global__ __launch_bounds__(128) void k_ewald_pack32(int64_t np, const double *__restrict__ tab64,
                                                      float4 *__restrict__ tab32) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const double *v = tab64 + 10 * q;
  tab32[3 * q + 0] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  tab32[3 * q + 1] = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
  tab32[3 * q + 2] = make_float4((float)v[8], (float)v[9], 0.0f, 0.0f);
}

// the same series at arbitrary folded offsets u [n][3] -> out [n][10]
__global__ __launch_bounds__(128) void k_ewald_points(EwaldP E, double alpha, int rcut2, int fcut2, int64_t n,
                                                      const double *__restrict__ u, double *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double uq[3] = {fabs(u[3 * q]), fabs(u[3 * q + 1]), fabs(u[3 * q + 2])};
  Acc10 o;
  ewald_point(E, alpha, rcut2, fcut2, uq, o);
  for (int k = 0; k < 10; ++k) out[10 * q + k] = o.v[k];
}

// correction (phi_c, signed A_c, H_c) at offsets d [n][3] -> out [n][10]:
// method 1 = FP64 series, 0 = FP64 table (Taylor term for phi_c and A_c, the
// nearest grid point's second derivatives); beyond the far-field switch
// (2P1I |dz| > zfar, 1P2I sqrt(dy^2 + dz^2) > zfar) the analytic limit minus
// the Newtonian kernel, whose second derivatives are (3 d_j d_k - r^2
// delta_jk) / r^5
__global__ __launch_bounds__(128) void k_ewald_points10(int method, EwaldP E, double alpha, int rcut2, int fcut2,
                                                        int64_t n, const double *__restrict__ d,
                                                        double *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double dx = d[3 * q], dy = d[3 * q + 1], dz = d[3 * q + 2];
  double *o = out + 10 * q;
  if (far_field10(E, dx, dy, dz, o)) return;
  const double u[3] = {fabs(dx), fabs(dy), fabs(dz)};
  double v[10];
  if (method == 1) {
    Acc10 s;
    ewald_point(E, alpha, rcut2, fcut2, u, s);
    for (int k = 0; k < 10; ++k) v[k] = s.v[k];
  } else {
    table_taylor64(E, u, v[0], v + 1);
    table_hessian64(E, u, v + 4);
  }
  // unfold: phi_c and the diagonal second derivatives are even in every
  // component, A_c,k odd in d_k, H_jk (j != k) odd in d_j and in d_k
  const double sx = dx < 0 ? -1.0 : 1.0, sy = dy < 0 ? -1.0 : 1.0, sz = dz < 0 ? -1.0 : 1.0;
  o[0] = v[0];
  o[1] = sx * v[1];
  o[2] = sy * v[2];
  o[3] = sz * v[3];
  o[4] = v[4];
  o[5] = v[5];
  o[6] = v[6];
  o[7] = sx * sy * v[7];
  o[8] = sx * sz * v[8];
  o[9] = sy * sz * v[9];
}

}  // namespace

hipError_t launch_ewald_pack32(const EwaldP &E, const double *tab64, float4 *tab32, hipStream_t st) {
  const int64_t np = (int64_t)E.n * E.n * E.n;
  hipLaunchKernelGGL(k_ewald_pack32, dim3((unsigned)((np + 127) / 128)), dim3(128), 0, st, np, tab64, tab32);
  return hipGetLastError();
}

hipError_t launch_ewald_points10(int method, const EwaldP &E, double alpha, int rcut2, int fcut2, int64_t n,
                                 const double *d, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_ewald_points10, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, method, E, alpha,
                     rcut2, fcut2, n, d, out);
  return hipGetLastError();
}

hipError_t launch_ewald_points(const EwaldP &E, double alpha, int rcut2, int fcut2, int64_t n, const double *u,
                               double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_ewald_points, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, E, alpha, rcut2, fcut2,
                     n, u, out);
  return hipGetLastError();
}

hipError_t launch_ewald_table(const EwaldP &E, double alpha, int rcut2, int fcut2, double *tab64,
                              float4 *tab32, hipStream_t st) {
  int64_t np = (int64_t)E.n * E.n * E.n;
  hipLaunchKernelGGL(k_ewald_table, dim3((unsigned)((np + 127) / 128)), dim3(128), 0, st, E, alpha,
                     rcut2, fcut2, tab64, tab32);
  return hipGetLastError();
}

}  // namespace ot
