// Column densities (OpticalDepth module, Sec. 2.3) on the device.
//
// 1. HEALPix NESTED pixel of a direction (Gorski et al. 2005 construction:
//    12 base pixels, polar caps above |z| = 2/3, equatorial belt between).
// 2. Node-ray intersection table: for each (theta, phi, psi) bin centre, a
//    uniform sphere of angular radius psi is sampled on nr radii x nazi
//    azimuths (weight sqrt(1 - (b/psi)^2) sin b); each sample is assigned at
//    Nside_f = 2 Nside (the paper's oversampling) and coarsened to its NESTED
//    parent; per-pixel weights are normalised to 1 and stored as compressed
//    rows (pixels ascending).  One wave per entry: lanes fill the sample pixels
//    into LDS, then each lane sums its own pixels over the samples in order,
//    so the sums are deterministic.
// 3. Column walk: like the gravity walk, plus for every (cell, node) pair the
//    direction bins (FP64; for cells of the block's own size on a dyadic grid
//    a precomputed lattice row), the table row's four-slot record, and
//    N_p += w M / (Omega_pix d^2) in a per-cell pixel map held in LDS as
//    [pixel][cell] (each thread owns its cell's column: plain
//    read-modify-write, no atomics, no bank conflicts), or in place in the
//    output when the maps are too large for LDS.  The record loads run two
//    pairs ahead of the map updates; rows of more than four pixels finish
//    from a per-thread queue at the end of each list tile.  At the end each
//    cell's map and tau_avg = -ln(mean_p exp(-kappa N_p)) are written out.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "mlp_infer.hpp"

namespace ot {

namespace {

constexpr double PI = 3.14159265358979323846;

__device__ inline int64_t spread2(int64_t v) {
  int64_t r = 0;
  for (int b = 0; b < 16; ++b) r |= ((v >> b) & 1) << (2 * b);
  return r;
}

// NESTED pixel of direction (x, y, z), any positive length
__device__ inline int vec2pix_nest(int nside, double x, double y, double z) {
  const double s2 = x * x + y * y;
  const double r = sqrt(s2 + z * z);
  const double zn = z / r;
  const double za = fabs(zn);
  double phi = atan2(y, x);
  if (phi < 0.0) phi += 2.0 * PI;
  double tt = phi / (0.5 * PI);
  if (tt >= 4.0) tt = 0.0;
  int face, ix, iy;
  if (za <= 2.0 / 3.0) {
    const double t1 = (double)nside * (0.5 + tt);
    const double t2 = (double)nside * (zn * 0.75);
    const int jp = (int)(t1 - t2), jm = (int)(t1 + t2);
    const int ifp = jp / nside, ifm = jm / nside;
    face = ifp == ifm ? (ifp & 3) + 4 : (ifp < ifm ? (ifp & 3) : (ifm & 3) + 8);
    ix = jm & (nside - 1);
    iy = nside - (jp & (nside - 1)) - 1;
  } else {
    int ntt = (int)tt;
    ntt = ntt > 3 ? 3 : ntt;
    const double tp = tt - (double)ntt;
    const double one_minus = s2 / (r * (r + fabs(z)));  // 1 - |z| without cancellation
    const double tmp = (double)nside * sqrt(3.0 * one_minus);
    int jp = (int)(tp * tmp), jm = (int)((1.0 - tp) * tmp);
    jp = jp > nside - 1 ? nside - 1 : jp;
    jm = jm > nside - 1 ? nside - 1 : jm;
    if (zn >= 0) {
      face = ntt;
      ix = nside - jm - 1;
      iy = nside - jp - 1;
    } else {
      face = ntt + 8;
      ix = jp;
      iy = jm;
    }
  }
  return face * nside * nside + (int)(spread2(ix) | (spread2(iy) << 1));
}

constexpr int RT_MAXS = 8192;  // samples per entry
constexpr int RT_MAXR = 256;   // radii
constexpr int RT_MAXP = 768;   // pixels (Nside <= 8)

__global__ __launch_bounds__(64) void k_raytable_dense(RayTableP P, double *__restrict__ dense) {
  __shared__ short spix[RT_MAXS];
  __shared__ double swr[RT_MAXR];
  __shared__ double sw[RT_MAXP];
  __shared__ double stot;
  const int e = blockIdx.x, lane = threadIdx.x;
  const int it = e / (P.nphi * P.npsi), ip = (e / P.npsi) % P.nphi, is = e % P.npsi;
  const double th = ((double)it + 0.5) * P.dtheta;
  const double ph = ((double)ip + 0.5) * P.dphi;
  const double ps = ((double)is + 0.5) * P.dpsi;
  const double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
  const double c[3] = {st * cp, st * sp, ct};
  const double et[3] = {ct * cp, ct * sp, -st};
  const double ep[3] = {-sp, cp, 0.0};
  const int ns = P.nr * P.nazi;
  const double dal = (2.0 * PI) / (double)P.nazi;
  for (int j = lane; j < ns; j += 64) {
    const int r = j / P.nazi, a = j % P.nazi;
    const double u = ((double)r + 0.5) / (double)P.nr;
    const double b = u * ps;
    const double cb = cos(b), sb = sin(b);
    const double al = ((double)a + 0.5) * dal;
    const double ca = cos(al), sa = sin(al);
    double n[3];
    for (int k = 0; k < 3; ++k) n[k] = cb * c[k] + sb * (ca * et[k] + sa * ep[k]);
    spix[j] = (short)(vec2pix_nest(2 * P.nside, n[0], n[1], n[2]) >> 2);
  }
  for (int r = lane; r < P.nr; r += 64) {
    const double u = ((double)r + 0.5) / (double)P.nr;
    swr[r] = sqrt(1.0 - u * u) * sin(u * ps);
  }
  __syncthreads();
  for (int p = lane; p < P.npix; p += 64) {
    double acc = 0.0;
    for (int r = 0; r < P.nr; ++r) {
      const double w = swr[r];
      for (int a = 0; a < P.nazi; ++a)
        if (spix[r * P.nazi + a] == p) acc += w;
    }
    sw[p] = acc;
  }
  __syncthreads();
  if (lane == 0) {
    double tot = 0.0;
    for (int p = 0; p < P.npix; ++p) tot += sw[p];
    stot = tot;
  }
  __syncthreads();
  for (int p = lane; p < P.npix; p += 64) dense[(int64_t)e * P.npix + p] = sw[p] / stot;
}

__global__ void k_raytable_count(RayTableP P, const double *__restrict__ dense, int32_t *__restrict__ cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.nentries) return;
  int n = 0;
  for (int p = 0; p < P.npix; ++p) n += dense[(int64_t)e * P.npix + p] > 0.0;
  cnt[e] = n;
}

__global__ void k_raytable_fill(RayTableP P, const double *__restrict__ dense, const int64_t *__restrict__ off,
                                uint16_t *__restrict__ pix, double *__restrict__ w64) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.nentries) return;
  int64_t o = off[e];
  for (int p = 0; p < P.npix; ++p) {
    const double v = dense[(int64_t)e * P.npix + p];
    if (v > 0.0) {
      pix[o] = (uint16_t)p;
      w64[o] = v;
      ++o;
    }
  }
}

// ------------------------------------------------------------- column walk
// a list record in the LDS tile: centre of mass and mass, (R_eq h)^2, and
// R_eq h (times the psi table's scale) and the mass in FP32.  A record of the
// lattice table (negative rhs) holds, in place of (R_eq h)^2, its entry for
// the block's first cell; a cell's entry adds the cell's own lattice index.
struct __align__(16) ColRec {
  double x, y, z, w;
  union {
    double rh2;
    int lat;
  };
  float rhs, m;
};

// list records per LDS tile (small: the maps need the LDS; with 48-pixel
// FP32 maps of 256 cells three workgroups then fit in a compute unit's LDS)
constexpr int TILE = 60;

// Largest k in [0, n-1] with pred(k), pred monotone (true up to some k) and
// pred(0) taken as true; branch-free binary search for n <= 64.
template <typename Pred>
__device__ inline int last_true(int n, Pred pred) {
  int k = 0;
  for (int step = 32; step > 0; step >>= 1) {
    const int c = k + step;
    if (c <= n - 1 && pred(c)) k = c;
  }
  return k;
}

// Table row of a node at offset d = r - r_a from the target cell (the node
// seen from the cell along v = -d; |d|^2 = r2, node size h, R_eq h).  The bins
// are those of floor(theta / dtheta), floor(phi / dphi) and floor(psi / dpsi)
// of v, decided without inverse trigonometric functions or square roots:
//   theta >= k dtheta  <=>  v_z <= cos(k dtheta) |v|
//                      <=>  v_z |v_z| <= cos(k dtheta) |cos(k dtheta)| r2
//   psi   >= k dpsi    <=>  (R_eq h)^2 >= sin^2(k dpsi) r2
//   phi   >= k dphi    <=>  cos(k dphi) v_y - sin(k dphi) v_x >= 0   (0 < phi < pi)
// (x -> x |x| is increasing, so the squared forms are the same inequalities),
// with phi in (pi, 2 pi) mapped to the upper half-plane by v -> -v; on the x
// axis (v_y = +-0) phi is that of atan2: 0, or pi (bin ip_pi) when v_x has its
// sign bit set.  The comparisons are FP64.
// Which k to compare: three byte tables in LDS, indexed by FP32 values that
// are monotone in the angles (cos theta, sin psi, and t = u_x / (|u_x| + u_y)
// for phi in [0, pi]), hold for each cell the lowest bin over the cell
// widened by a guard band larger than the FP32 rounding.  A widened cell
// spans at most one threshold (cells are at most half as wide as the closest
// two), so the bin is k0 or k0 + 1: one FP64 comparison at k0 + 1 decides
// (each threshold list ends in a sentinel its test never passes).  Binary
// searches remain for offsets too small for FP32 and when the tables would
// not fit (C.estimate = 0).
// dxf, dyf, dzf: d in FP32; rd = 1 / sqrt(max(f2, 1e-30)) for f2 = r2 in FP32;
// rhs = R_eq h times the psi table's scale.
__device__ inline int table_row(const ColP &C, const double *thr, const uint8_t *lut, double dx, double dy,
                                double dz, float dxf, float dyf, float dzf, double r2, float f2, float rd,
                                double rh2, float rhs) {
  const double *cth = thr;                       // [ntheta + 1] c |c|, sentinel -inf
  const double *sps = cth + C.ntheta + 1;        // [npsi + 1] sin^2, sentinel +inf
  const double *cs = sps + C.npsi + 1;           // [nphi/2 + 1] (cos, sin), the last (-1, 0)
  const double vzz = -dz * fabs(dz);             // v_z |v_z|
  const int half = C.nphi / 2;
  const bool lower = dy > 0.0;                   // v_y < 0
  // v -> -v on the lower half-plane: u = (v_x or -v_x, |v_y|)
  const double ux = dx * (lower ? 1.0 : -1.0);
  auto pth = [&](int k) { return vzz <= cth[k] * r2; };
  auto pps = [&](int k) { return rh2 >= sps[k] * r2; };
  auto pph = [&](int q) { return cs[2 * q] * fabs(dy) - cs[2 * q + 1] * ux >= 0.0; };
  const float den = fabsf(dxf) + fabsf(dyf);     // |u_x| + u_y
  // Every index is inside its table: |cos theta| <= 1 and |t| <= 1 up to
  // rounding, sin psi is clamped to 1, and each table has one cell to spare.
  // The estimates run on every lane; lanes outside their range are redone by
  // the binary search under a wave-uniform branch, which keeps the common path
  // free of divergent control flow.  (On the x axis, v_y = 0, phi comes from
  // the atan2 rule below and its estimate is not used: a node straight above
  // or below the cell is safe.)
  // (den + 1e-30 below keeps the reciprocal finite; it is den to ten digits
  // only for den > 1e-20, so smaller den take the exact path)
  const bool safe = C.estimate && f2 > 1e-30f && (den > 1e-20f || dy == 0.0);
  const int k0t = lut[(int)fmaf(-dzf * rd, C.lut_th, C.lut_th)];
  // (rhs rd >= 0: the median with 0 and the table size is the clamp; (float)ux
  // is +-dxf exactly)
  const int k0s = lut[LUT_TH + (int)__builtin_amdgcn_fmed3f(rhs * rd, 0.0f, C.lut_ps)];
  const float t = (lower ? dxf : -dxf) * __builtin_amdgcn_rcpf(den + 1e-30f);
  const int k0p = lut[LUT_TH + LUT_PS + (int)fmaf(t, C.lut_ph, C.lut_ph)];
  int it = k0t + (int)pth(k0t + 1);
  int is = k0s + (int)pps(k0s + 1);
  int k = k0p + (int)pph(k0p + 1);
  if (__ballot(!safe)) {
    if (!safe) {
      it = last_true(C.ntheta, pth);
      is = last_true(C.npsi, pps);
      k = last_true(half, pph);
    }
  }
  // atan2(+-0, x) is pi (bin ip_pi) whenever the sign bit of v_x = -d_x is
  // set, -0 included (a node straight above the cell, d_x = +0), else 0;
  // k <= half - 1, so the lower half-plane stays below nphi
  const int ip = dy == 0.0 ? (signbit(dx) ? 0 : C.ip_pi) : (lower ? half : 0) + k;
  return (int)__umul24(__umul24(it, C.nphi) + ip, C.npsi) + is;  // < 2^24 entries
}

template <int BC>
__device__ inline void wrap3(const EwaldP &E, double &dx, double &dy, double &dz) {
  if (BC != 0) {
    dx = wrap_axis(dx, E.L[0], E.inv_L[0], 1);
    if (BC != 3) dy = wrap_axis(dy, E.L[1], E.inv_L[1], 1);
    if (BC == 1) dz = wrap_axis(dz, E.L[2], E.inv_L[2], 1);
  }
}

// gravity kernel of one pair in FP64 (isolated or table Ewald); returns false
// for the target cell itself
template <int BC>
__device__ inline bool grav64(const EwaldP &E, double dx, double dy, double dz, double r2, double &phi,
                              double &A0, double &A1, double &A2) {
  const double inv = 1.0 / sqrt(r2);
  const double inv3 = inv * inv * inv;
  if (BC == 0) {
    phi = inv;
    A0 = dx * inv3;
    A1 = dy * inv3;
    A2 = dz * inv3;
    return true;
  }
  if (BC == 2 && fabs(dz) > E.zfar) {
    phi = E.far_phi_a * fabs(dz) + E.far_phi_b;
    A0 = 0.0;
    A1 = 0.0;
    A2 = dz < 0 ? -E.far_az : E.far_az;
    return true;
  }
  if (BC == 3 && dy * dy + dz * dz > E.zfar * E.zfar) {
    const double rho2 = dy * dy + dz * dz;
    phi = E.far_phi_a * log(rho2) + E.far_phi_b;
    A0 = 0.0;
    A1 = E.far_az * dy / rho2;
    A2 = E.far_az * dz / rho2;
    return true;
  }
  const double u[3] = {fabs(dx), fabs(dy), fabs(dz)};
  int g[3];
  double dl[3];
  for (int k = 0; k < 3; ++k) {
    int gi = (int)floor(u[k] / E.step[k] + 0.5);
    gi = gi > E.n - 1 ? E.n - 1 : gi;
    g[k] = gi;
    dl[k] = u[k] - gi * E.step[k];
  }
  const double *T = E.tab64 + 10 * (((int64_t)g[2] * E.n + g[1]) * E.n + g[0]);
  const double phic = T[0] - (T[1] * dl[0] + T[2] * dl[1] + T[3] * dl[2]);
  const double a0 = T[1] - (T[4] * dl[0] + T[7] * dl[1] + T[8] * dl[2]);
  const double a1 = T[2] - (T[7] * dl[0] + T[5] * dl[1] + T[9] * dl[2]);
  const double a2 = T[3] - (T[8] * dl[0] + T[9] * dl[1] + T[6] * dl[2]);
  phi = inv + phic;
  A0 = dx * inv3 + (dx < 0 ? -a0 : a0);
  A1 = dy * inv3 + (dy < 0 ? -a1 : a1);
  A2 = dz * inv3 + (dz < 0 ? -a2 : a2);
  return true;
}

// FP32 gravity of one pair (same forms as the FP32 walk)
// (inv = 1 / |d|, 0 for the target cell itself)
template <int BC>
__device__ inline void grav32(const EwaldP &E, float dx, float dy, float dz, float inv, float &phi, float &A0,
                              float &A1, float &A2) {
  const float inv3 = inv * inv * inv;
  if (BC == 0) {
    phi = inv;
    A0 = dx * inv3;
    A1 = dy * inv3;
    A2 = dz * inv3;
    return;
  }
  if (BC == 2 && fabsf(dz) > (float)E.zfar) {
    phi = (float)E.far_phi_a * fabsf(dz) + (float)E.far_phi_b;
    A0 = 0.0f;
    A1 = 0.0f;
    A2 = dz < 0 ? -(float)E.far_az : (float)E.far_az;
    return;
  }
  if (BC == 3 && dy * dy + dz * dz > (float)(E.zfar * E.zfar)) {
    const float rho2 = dy * dy + dz * dz, fa = (float)E.far_az / rho2;
    phi = (float)E.far_phi_a * logf(rho2) + (float)E.far_phi_b;
    A0 = 0.0f;
    A1 = fa * dy;
    A2 = fa * dz;
    return;
  }
  const float u0 = fabsf(dx), u1 = fabsf(dy), u2 = fabsf(dz);
  const int g0 = min((int)(u0 * (float)E.inv_step[0] + 0.5f), E.n - 1);
  const int g1 = min((int)(u1 * (float)E.inv_step[1] + 0.5f), E.n - 1);
  const int g2 = min((int)(u2 * (float)E.inv_step[2] + 0.5f), E.n - 1);
  const float d0 = u0 - g0 * (float)E.step[0];
  const float d1 = u1 - g1 * (float)E.step[1];
  const float d2 = u2 - g2 * (float)E.step[2];
  const float4 *p = E.tab32 + 3 * (((int64_t)g2 * E.n + g1) * E.n + g0);
  const float4 q0 = p[0], q1 = p[1], q2 = p[2];
  const float phic = q0.x - (q0.y * d0 + q0.z * d1 + q0.w * d2);
  const float a0 = q0.y - (q1.x * d0 + q1.w * d1 + q2.x * d2);
  const float a1 = q0.z - (q1.w * d0 + q1.y * d1 + q2.y * d2);
  const float a2 = q0.w - (q2.x * d0 + q2.y * d1 + q1.z * d2);
  phi = inv + phic;
  A0 = dx * inv3 + (dx < 0 ? -a0 : a0);
  A1 = dy * inv3 + (dy < 0 ? -a1 : a1);
  A2 = dz * inv3 + (dz < 0 ? -a2 : a2);
}

// One workgroup handles cpw cells (one per thread) of one leaf block.
// LDS: the bin look-up tables and the list tile at fixed addresses (static),
// then the thresholds and (GMAP = false) the maps (dynamic).  With GMAP the
// maps are accumulated in place in npix (each thread owns its cell's column,
// a wave's 64 cells are adjacent): for maps too large for LDS at a useful
// occupancy (192 pixels take 768 bytes per cell in FP32).
// NOGRAV (FP32): the columns only; phi and acc are left to another kernel (the
// walk with the learned correction).
template <typename Real, int BC, bool NOGRAV, bool GMAP, bool LATTICE = !GMAP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_eval_cols(DevTree T, EwaldP E, ColP C, const int64_t *__restrict__ off,
                                                   const double4 *__restrict__ rec,
                                                   const int32_t *__restrict__ ids, const double *__restrict__ lh,
                                                   Real *__restrict__ phi, Real *__restrict__ acc,
                                                   Real *__restrict__ npix, Real *__restrict__ tau, double negG,
                                                   int cpw, int lcpw, const int32_t *__restrict__ blist) {
  __shared__ uint8_t lut[LUT_BYTES];
  __shared__ ColRec tile[TILE];
  extern __shared__ __align__(16) unsigned char smem[];
  double *thr = reinterpret_cast<double *>(smem);
  Real *map = reinterpret_cast<Real *>(thr + C.nthr);
  const int nchunk = 512 / cpw;
  // blist (optional): the leaf blocks to evaluate, else all of them in order
  const int64_t b = blist ? (int64_t)blist[blockIdx.x / nchunk] : (int64_t)(blockIdx.x / nchunk);
  const int tid = threadIdx.x;
  const int ci = (int)(blockIdx.x % nchunk) * cpw + tid;
  const int64_t ncell = T.nb * 512;
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  // absolute cell centre, the same expression as the records' cell centres
  const double cx = centre_coord(T.org[0], 8 * (int64_t)T.bcoord[3 * b] + (ci & 7), h);
  const double cy = centre_coord(T.org[1], 8 * (int64_t)T.bcoord[3 * b + 1] + ((ci >> 3) & 7), h);
  const double cz = centre_coord(T.org[2], 8 * (int64_t)T.bcoord[3 * b + 2] + (ci >> 6), h);
  for (int q = tid; q < LUT_BYTES; q += cpw) lut[q] = C.lut[q];
  for (int q = tid; q < C.nthr; q += cpw) thr[q] = C.thr[q];
  // byte address of this cell's entry of pixel 0; pixel p is (p << lmap) on
  char *const mcell = GMAP ? reinterpret_cast<char *>(npix + b * C.npix * 512 + ci)
                           : reinterpret_cast<char *>(map + tid);
  const int lmap = (GMAP ? 9 : lcpw) + (sizeof(Real) == 8 ? 3 : 2);
  for (int p = 0; p < C.npix; ++p) *reinterpret_cast<Real *>(mcell + (p << lmap)) = (Real)0;
  const float inv_omega = (float)(1.0 / C.omega);
  // Cells of this block's size at lattice offsets take their table row from
  // the lattice table (exact: the grid is dyadic when lat_r > 0, so such
  // offsets are exact multiples of h, and the bins do not change under
  // power-of-two scaling).  A record qualifies when the offsets of all 512
  // cells of the block lie in the table and no periodic image is involved;
  // the entry of cell (i, j, k) is then the record's entry for cell 0 plus
  // (k W + j) W + i.
  const int64_t cell0 = T.na + 72 * T.nb;
  const int lat_w = 2 * C.lat_r + 1;
  const int lat_lane = ((ci >> 6) * lat_w + ((ci >> 3) & 7)) * lat_w + (ci & 7);
  const double inv_h = 1.0 / h;  // exact: h is a power of two on a dyadic grid
  const double bx0 = centre_coord(T.org[0], 8 * (int64_t)T.bcoord[3 * b], h);
  const double by0 = centre_coord(T.org[1], 8 * (int64_t)T.bcoord[3 * b + 1], h);
  const double bz0 = centre_coord(T.org[2], 8 * (int64_t)T.bcoord[3 * b + 2], h);
  // lattice offset (in cells) of a node from the block's first cell, or a
  // value outside [-lat_r, lat_r - 7] if the block's offsets leave the table
  // or may wrap on a periodic axis
  auto lat_axis = [&](double d0, int ax) {
    const bool per = BC == 1 || (BC == 2 && ax < 2) || (BC == 3 && ax == 0);
    if (per && !(d0 > -0.5 * E.L[ax] + h && d0 + 8.0 * h < 0.5 * E.L[ax])) return 1 << 20;
    const double n0 = d0 * inv_h;
    return fabs(n0) < (double)(1 << 20) && n0 == rint(n0) ? (int)n0 : 1 << 20;
  };
  // potential: FP64 sum (FP64 walk) or Kahan-compensated FP32 sum and its
  // compensation (FP32 walk)
  double s = 0.0;
  float ks = 0.0f, kc = 0.0f;
  auto kahan = [&](float x) {
    const float y = x - kc;
    const float t = ks + y;
    kc = (t - ks) - y;
    ks = t;
  };
  Real ax = 0, ay = 0, az = 0;
  const int64_t start = off[b], n = off[b + 1] - start;
  for (int64_t t0 = 0; t0 < n; t0 += TILE) {
    __syncthreads();
    for (int q = tid; q < TILE && t0 + q < n; q += cpw) {
      const double4 rq = rec[start + t0 + q];
      const double rh = C.req * lh[start + t0 + q];  // radius of the equal-volume sphere
      tile[q].x = rq.x;
      tile[q].y = rq.y;
      tile[q].z = rq.z;
      tile[q].w = rq.w;
      // rhs carries the lattice flag in its sign
      bool lat = LATTICE && C.lat_r > 0 && ids[start + t0 + q] >= cell0 && lh[start + t0 + q] == h;
      if (lat) {
        const int nx = lat_axis(bx0 - rq.x, 0), ny = lat_axis(by0 - rq.y, 1), nz = lat_axis(bz0 - rq.z, 2);
        const int lo = -C.lat_r, hi = C.lat_r - 7;
        lat = nx >= lo && nx <= hi && ny >= lo && ny <= hi && nz >= lo && nz <= hi;
        if (lat) tile[q].lat = C.lat0 + ((nz + C.lat_r) * lat_w + (ny + C.lat_r)) * lat_w + (nx + C.lat_r);
      }
      if (!lat) tile[q].rh2 = rh * rh;
      tile[q].rhs = (lat ? -1.0f : 1.0f) * ((float)rh * C.lut_ps);
      tile[q].m = (float)rq.w;
    }
    __syncthreads();
    const int m = (int)(n - t0 < TILE ? n - t0 : TILE);
    // the acceleration is summed per tile, then the tile sums are added
    // (blocked summation: the rounding grows with the tile and tile count,
    // not with the list length)
    Real tx = 0, ty = 0, tz = 0;
    // offsets of a pair (minimum image, FP64) and their FP32 copies
    struct Geo {
      double dx, dy, dz, r2;
      float r2f, rd, dxf, dyf, dzf;
      bool valid, col;
    };
    auto geometry = [&](const ColRec &r) {
      Geo q;
      q.dx = cx - r.x;
      q.dy = cy - r.y;
      q.dz = cz - r.z;
      wrap3<BC>(E, q.dx, q.dy, q.dz);
      q.r2 = q.dx * q.dx + q.dy * q.dy + q.dz * q.dz;
      q.valid = q.r2 != 0.0;  // the target cell itself contributes nothing
      q.col = q.valid && q.r2 <= C.max_dist2;
      q.r2f = (float)q.r2;
      q.rd = __builtin_amdgcn_rsqf(fmaxf(q.r2f, 1e-30f));
      q.dxf = (float)q.dx;
      q.dyf = (float)q.dy;
      q.dzf = (float)q.dz;
      return q;
    };
    // the row of a pair in the node-ray table (0 outside the column radius,
    // where the pair's weight base is zero)
    auto row_of = [&](const ColRec &r, const Geo &q) {
      // a cell of this block's size, in the lattice rows for every cell of
      // the block (the record is the same for the whole wave)
      if (LATTICE && r.rhs < 0.0f) return r.lat + lat_lane;
      return q.col ? table_row(C, thr, lut, q.dx, q.dy, q.dz, q.dxf, q.dyf, q.dzf, q.r2, q.r2f, q.rd, r.rh2,
                               fabsf(r.rhs))
                   : 0;
    };
    // A two-stage pipeline over the tile: stage A of pair j + 2 (offsets,
    // gravity, bins, and the load of its row record) runs before stage B of
    // pair j (the map update), so each record load is in flight while the
    // next two pairs' bins are computed (with the maps in memory one stage
    // follows the other).  Both stages keep list order (the remainders of
    // long rows follow at the tile's end).  The record: four pixels, and their
    // weights in FP32 (the FP32 walk) or FP64.
    struct W64 {
      double2 a, b;
    };
    using WQ = typename std::conditional<sizeof(Real) == 8, W64, uint4>::type;
    struct Pend {
      uint4 pq;
      WQ wq;
      Real base;
      int e;
      bool col;
    };
    // stage A of a pair past the tile's end (jj >= m: the pipeline issues its
    // loads unconditionally, so that the waits for each record can count the
    // loads issued after it) repeats the last record with zero mass and no
    // columns: it adds exact zeros
    auto stage_a = [&](int jj) {
      const bool live = jj < m;
      const ColRec r = tile[live ? jj : m - 1];
      const Geo q = geometry(r);
      Pend p;
      p.e = row_of(r, q);
      // pixels and weights at one 32-bit byte offset from uniform bases
      const uint32_t ro = (uint32_t)p.e << 5;
      const char *const rq = reinterpret_cast<const char *>(C.rows8) + ro;
      p.pq = *reinterpret_cast<const uint4 *>(rq);
      p.col = q.col && live;
      if constexpr (sizeof(Real) == 8) {
        const char *const wq = reinterpret_cast<const char *>(C.quad_w64) + ro;
        p.wq.a = *reinterpret_cast<const double2 *>(wq);
        p.wq.b = *reinterpret_cast<const double2 *>(wq + 16);
        // FP64 gravity; the target cell (and a repeat) adds exact zeros
        const double m64 = q.valid && live ? r.w : 0.0;
        double ph, A0, A1, A2;
        grav64<BC>(E, q.dx, q.dy, q.dz, q.valid ? q.r2 : 1.0, ph, A0, A1, A2);
        s += m64 * ph;
        tx += m64 * A0;
        ty += m64 * A1;
        tz += m64 * A2;
        // N_p += w M / (Omega d^2): the weight base of the pair
        p.base = p.col ? r.w / (C.omega * q.r2) : 0.0;
      } else {
        p.wq = *reinterpret_cast<const uint4 *>(rq + 16);
        // FP32 gravity from the FP64 offset (already the minimum image); the
        // target cell's terms are exact zeros (zero mass; 1/r stays finite; a
        // Kahan step with a zero only moves the compensation into the sum)
        const float m32 = q.valid && live ? r.m : 0.0f;
        const float mr = m32 * q.rd, mr2 = mr * q.rd;  // M / r, M / r^2
        if (NOGRAV) {
        } else if (BC == 0) {
          const float mr3 = mr2 * q.rd;
          kahan(mr);
          tx = fmaf(q.dxf, mr3, (float)tx);
          ty = fmaf(q.dyf, mr3, (float)ty);
          tz = fmaf(q.dzf, mr3, (float)tz);
        } else {
          float ph, A0, A1, A2;
          grav32<BC>(E, q.dxf, q.dyf, q.dzf, q.valid ? q.rd : 0.0f, ph, A0, A1, A2);
          kahan(m32 * ph);
          tx += (Real)(m32 * A0);
          ty += (Real)(m32 * A1);
          tz += (Real)(m32 * A2);
        }
        // N_p += w M / (Omega d^2): the weight base of the pair
        p.base = p.col ? (Real)(mr2 * inv_omega) : (Real)0;
      }
      return p;
    };
    // Rows of more than four pixels: the rest of the row (further loads that
    // would stall the pipeline) is added at the tile's end, from a per-thread
    // queue of up to DQ rows; a thread whose queue is full adds its oldest row
    // at once.
    constexpr int DQ = GMAP ? 4 : 8;
    uint32_t dq_code[DQ] = {};  // count << 26 | offset
    Real dq_base[DQ] = {};
    int dq_n = 0;
    auto long_row = [&](uint32_t code, Real base) {
      const int o0 = (int)(code & 0x3ffffffu), o1 = o0 + (int)(code >> 26);
      if constexpr (sizeof(Real) == 8) {
        for (int o = o0 + 4; o < o1; ++o)
          *reinterpret_cast<double *>(mcell + ((uint32_t)C.pix[o] << lmap)) += C.w64[o] * base;
      } else {
        const float base24 = base * (1.0f / 16777216.0f);
        // two packed entries at a time (a zero entry adds zero to pixel 0)
        for (int o = o0 + 4; o < o1; o += 2) {
          const uint32_t v = C.ent[o], u = o + 1 < o1 ? C.ent[o + 1] : 0u;
          float *const qv = reinterpret_cast<float *>(mcell + ((v >> 24) << lmap));
          *qv += (float)(v & 0xffffffu) * base24;
          float *const qu = reinterpret_cast<float *>(mcell + ((u >> 24) << lmap));
          *qu += (float)(u & 0xffffffu) * base24;
        }
      }
    };
    // four of the row's pixels come with its record (distinct pixels, weight
    // 0 past the count), so the four read-modify-writes are independent; the
    // column is the thread's own (plain read-modify-write: LDS atomic adds
    // measured 2.5x slower)
    struct MapV {
      Real v0, v1, v2, v3;
    };
    // the map values of a pending pair's slots (maps in memory: the padding
    // slots, weight 0, are not read)
    auto map_read = [&](const Pend &p) {
      MapV m;
      m.v1 = m.v2 = m.v3 = (Real)0;
      const uint4 pq = p.pq;
      Real w1, w2, w3;
      if constexpr (sizeof(Real) == 8) {
        w1 = p.wq.a.y;
        w2 = p.wq.b.x;
        w3 = p.wq.b.y;
      } else {
        w1 = __uint_as_float(p.wq.y);
        w2 = __uint_as_float(p.wq.z);
        w3 = __uint_as_float(p.wq.w);
      }
      m.v0 = *reinterpret_cast<const Real *>(mcell + (pq.x << lmap));
      if (w1 != (Real)0) m.v1 = *reinterpret_cast<const Real *>(mcell + (pq.y << lmap));
      if (w2 != (Real)0) m.v2 = *reinterpret_cast<const Real *>(mcell + (pq.z << lmap));
      if (w3 != (Real)0) m.v3 = *reinterpret_cast<const Real *>(mcell + (pq.w << lmap));
      return m;
    };
    auto stage_b = [&](const Pend &p, const MapV *pre = nullptr) {
      const Real base = p.base;
      const uint4 pq = p.pq;
      Real w[4];
      if constexpr (sizeof(Real) == 8) {
        w[0] = p.wq.a.x;
        w[1] = p.wq.a.y;
        w[2] = p.wq.b.x;
        w[3] = p.wq.b.y;
      } else {
        w[0] = __uint_as_float(p.wq.x);
        w[1] = __uint_as_float(p.wq.y);
        w[2] = __uint_as_float(p.wq.z);
        w[3] = __uint_as_float(p.wq.w);
      }
      // bit 31 of the first pixel (more than four) and the bits from 23 up
      // are shifted out here
      Real *const q0 = reinterpret_cast<Real *>(mcell + (pq.x << lmap));
      Real *const q1 = reinterpret_cast<Real *>(mcell + (pq.y << lmap));
      Real *const q2 = reinterpret_cast<Real *>(mcell + (pq.z << lmap));
      Real *const q3 = reinterpret_cast<Real *>(mcell + (pq.w << lmap));
      if (GMAP) {
        // in memory the padding slots would cost traffic: they are skipped
        const bool u1 = w[1] != (Real)0, u2 = w[2] != (Real)0, u3 = w[3] != (Real)0;
        Real v0, v1 = 0, v2 = 0, v3 = 0;
        if (pre) {
          v0 = pre->v0;
          v1 = pre->v1;
          v2 = pre->v2;
          v3 = pre->v3;
        } else {
          v0 = *q0;
          if (u1) v1 = *q1;
          if (u2) v2 = *q2;
          if (u3) v3 = *q3;
        }
        *q0 = fma(w[0], base, v0);
        if (u1) *q1 = fma(w[1], base, v1);
        if (u2) *q2 = fma(w[2], base, v2);
        if (u3) *q3 = fma(w[3], base, v3);
      } else {
        const Real v0 = *q0, v1 = *q1, v2 = *q2, v3 = *q3;
        *q0 = fma(w[0], base, v0);
        *q1 = fma(w[1], base, v1);
        *q2 = fma(w[2], base, v2);
        *q3 = fma(w[3], base, v3);
      }
      if ((int)pq.x < 0 && p.col) {
        // the row's count and offset ride in the pixels' high bits; the row
        // joins the queue
        const uint32_t cnt = (pq.x >> 23) & 63u;
        const uint32_t o0 = (pq.y >> 23) | ((pq.z >> 23) << 9) | ((pq.w >> 23) << 18);
        if (dq_n == DQ) {
          long_row(dq_code[DQ - 1], dq_base[DQ - 1]);
          --dq_n;
        }
        for (int k = DQ - 1; k > 0; --k) {
          dq_code[k] = dq_code[k - 1];
          dq_base[k] = dq_base[k - 1];
        }
        dq_code[0] = (cnt << 26) | o0;
        dq_base[0] = base;
        ++dq_n;
      }
    };
    if (GMAP && sizeof(Real) == 8) {
      // maps in memory, FP64: each pair's map reads, then the next pair's
      // stage A, then the map writes, so the reads' latency overlaps that
      // arithmetic (4.13 -> 3.98 s on the large grid, at three workgroups per
      // CU instead of four)
      Pend cur = stage_a(0);
      for (int j = 0; j < m; ++j) {
        const MapV mv = map_read(cur);
        const Pend nxt = j + 1 < m ? stage_a(j + 1) : cur;
        stage_b(cur, &mv);
        cur = nxt;
      }
    } else if (GMAP) {
      // maps in memory, FP32: no pipeline (its registers would cost a fifth
      // workgroup per CU: 2.30 instead of 2.26 s on the large grid)
      for (int j = 0; j < m; ++j) stage_b(stage_a(j));
    } else {
      // two pairs ahead, unrolled by three with the pending state in rotating
      // registers (no copy of the state between iterations)
      Pend p0 = stage_a(0), p1 = stage_a(1), p2;
      for (int j = 0; j < m; j += 3) {
        p2 = stage_a(j + 2);
        stage_b(p0);
        p0 = stage_a(j + 3);
        if (j + 1 < m) stage_b(p1);
        p1 = stage_a(j + 4);
        if (j + 2 < m) stage_b(p2);
      }
    }
    for (int k = 0; k < DQ; ++k)
      if (k < dq_n) long_row(dq_code[k], dq_base[k]);
    ax += tx;
    ay += ty;
    az += tz;
  }
  const int64_t o = b * 512 + ci;
  if (!NOGRAV) {
    phi[o] = (Real)(negG * (sizeof(Real) == 8 ? s : (double)(ks - kc)));
    acc[o] = (Real)(negG * (double)ax);
    acc[ncell + o] = (Real)(negG * (double)ay);
    acc[2 * ncell + o] = (Real)(negG * (double)az);
  }
  double se = 0.0;
  for (int p = 0; p < C.npix; ++p) {
    const Real v = *reinterpret_cast<const Real *>(mcell + (p << lmap));
    if (!GMAP) npix[(b * C.npix + p) * 512 + ci] = v;
    se += exp(-C.kappa * (double)v);
  }
  tau[o] = (Real)(-log(se / (double)C.npix));
}

// Adaptive block update with columns (Sec. 2.2.6 names the optical depth
// among the quantities compared at the corner cells): the maps of the eight
// corner cells (i, j, k in {0, 7}) of every leaf block, summed in FP64 over
// the block's list with the FP64 walk's bins and weights.  One workgroup of
// eight waves per block, wave w takes corner w: its lanes bin 64 list entries
// at a time and add each entry's pixels to the corner's map in LDS (FP64 adds
// that only this wave makes, in list order per lane, so the sum is the same
// run to run).  flags[b] = 1 when at one corner the optical depth kappa N_p
// of a direction moved from the previous map by tol_tau or more (which also
// bounds the change of tau_avg); the flags are only ever set here.
template <int BC, typename Real>
__global__ __launch_bounds__(512) void k_abu_corner_cols(DevTree T, EwaldP E, ColP C,
                                                         const int64_t *__restrict__ off,
                                                         const double4 *__restrict__ rec,
                                                         const double *__restrict__ lh,
                                                         const Real *__restrict__ prev_npix, double tol_tau,
                                                         int32_t *__restrict__ flags) {
  __shared__ uint8_t lut[LUT_BYTES];
  extern __shared__ __align__(16) unsigned char smem[];
  double *const thr = reinterpret_cast<double *>(smem);
  double *const maps = thr + ((C.nthr + 1) & ~1);  // [8][npix]
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int q = tid; q < LUT_BYTES; q += 512) lut[q] = C.lut[q];
  for (int q = tid; q < C.nthr; q += 512) thr[q] = C.thr[q];
  for (int q = tid; q < 8 * C.npix; q += 512) maps[q] = 0.0;
  __syncthreads();
  double *const map = maps + w * C.npix;
  const int ci = 7 * (w & 1) + 56 * ((w >> 1) & 1) + 448 * ((w >> 2) & 1);
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const double cx = centre_coord(T.org[0], 8 * (int64_t)T.bcoord[3 * b] + (ci & 7), h);
  const double cy = centre_coord(T.org[1], 8 * (int64_t)T.bcoord[3 * b + 1] + ((ci >> 3) & 7), h);
  const double cz = centre_coord(T.org[2], 8 * (int64_t)T.bcoord[3 * b + 2] + (ci >> 6), h);
  const int64_t start = off[b], end = off[b + 1];
  for (int64_t j0 = start; j0 < end; j0 += 64) {
    const int64_t j = j0 + l < end ? j0 + l : end - 1;
    const double4 r = rec[j];
    double dx = cx - r.x, dy = cy - r.y, dz = cz - r.z;
    wrap3<BC>(E, dx, dy, dz);
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool col = j0 + l < end && r2 != 0.0 && r2 <= C.max_dist2;
    const float r2f = (float)r2;
    const float rd = __builtin_amdgcn_rsqf(fmaxf(r2f, 1e-30f));
    const double rh = C.req * lh[j];
    const int e = col ? table_row(C, thr, lut, dx, dy, dz, (float)dx, (float)dy, (float)dz, r2, r2f, rd, rh * rh,
                                  (float)rh * C.lut_ps)
                      : 0;
    if (col) {
      // the row: four pixels with their FP64 weights (zero past the count),
      // the rest of a longer row in pix / w64
      const double base = r.w / (C.omega * r2);
      const uint4 pq = C.rows8[2 * (int64_t)e];
      const double *const wq = C.quad_w64 + 4 * (int64_t)e;
      unsafeAtomicAdd(&map[pq.x & 0x7fffffu], wq[0] * base);
      unsafeAtomicAdd(&map[pq.y & 0x7fffffu], wq[1] * base);
      unsafeAtomicAdd(&map[pq.z & 0x7fffffu], wq[2] * base);
      unsafeAtomicAdd(&map[pq.w & 0x7fffffu], wq[3] * base);
      if ((int)pq.x < 0) {
        const int cnt = (int)((pq.x >> 23) & 63u);
        const int o0 = (int)((pq.y >> 23) | ((pq.z >> 23) << 9) | ((pq.w >> 23) << 18));
        for (int o = o0 + 4; o < o0 + cnt; ++o) unsafeAtomicAdd(&map[C.pix[o]], C.w64[o] * base);
      }
    }
  }
  __syncthreads();
  bool moved = false;
  for (int p = l; p < C.npix; p += 64)
    moved = moved || !(C.kappa * fabs(map[p] - (double)prev_npix[(b * C.npix + p) * 512 + ci]) < tol_tau);
  if (__any(moved) && l == 0) flags[b] = 1;
}

// Lattice row of every list entry for the walk with the learned surrogate:
// the row of the table that a cell of the target's own size at a lattice
// offset takes for the target's first cell (the walk adds each cell's own
// index), or -1 (not such a cell, offsets of the target's cells outside the
// table, or a periodic image possible).  One workgroup per list target: a
// leaf block, or with sub set a 4^3 octant of one (list b, block b / 8,
// octant b % 8).
template <int BC>
__global__ __launch_bounds__(256) void k_lattice_index(DevTree T, EwaldP E, ColP C, const int64_t *__restrict__ off,
                                                      const double4 *__restrict__ rec,
                                                      const int32_t *__restrict__ ids,
                                                      const double *__restrict__ lh, int32_t *__restrict__ llat,
                                                      int sub) {
  const int64_t tgt = blockIdx.x;
  const int64_t b = sub ? tgt >> 3 : tgt;
  const int so = sub ? (int)(tgt & 7) : 0;
  const int ext = sub ? 4 : 8;  // cells per axis of the target
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const double inv_h = 1.0 / h;  // exact: h is a power of two on a dyadic grid
  const double b0[3] = {centre_coord(T.org[0], 8 * (int64_t)T.bcoord[3 * b] + 4 * (so & 1), h),
                        centre_coord(T.org[1], 8 * (int64_t)T.bcoord[3 * b + 1] + 4 * ((so >> 1) & 1), h),
                        centre_coord(T.org[2], 8 * (int64_t)T.bcoord[3 * b + 2] + 4 * (so >> 2), h)};
  const int64_t cell0 = T.na + 72 * T.nb;
  const int lat_w = 2 * C.lat_r + 1;
  auto lat_axis = [&](double d0, int ax) {
    const bool per = BC == 1 || (BC == 2 && ax < 2) || (BC == 3 && ax == 0);
    if (per && !(d0 > -0.5 * E.L[ax] + h && d0 + (double)ext * h < 0.5 * E.L[ax])) return 1 << 20;
    const double n0 = d0 * inv_h;
    return fabs(n0) < (double)(1 << 20) && n0 == rint(n0) ? (int)n0 : 1 << 20;
  };
  const int64_t start = off[tgt], n = off[tgt + 1] - start;
  for (int64_t q = threadIdx.x; q < n; q += 256) {
    int32_t v = -1;
    if (C.lat_r > 0 && ids[start + q] >= cell0 && lh[start + q] == h) {
      const double4 r = rec[start + q];
      const int nx = lat_axis(b0[0] - r.x, 0), ny = lat_axis(b0[1] - r.y, 1), nz = lat_axis(b0[2] - r.z, 2);
      const int lo = -C.lat_r, hi = C.lat_r - (ext - 1);
      if (nx >= lo && nx <= hi && ny >= lo && ny <= hi && nz >= lo && nz <= hi)
        v = C.lat0 + ((nz + C.lat_r) * lat_w + (ny + C.lat_r)) * lat_w + (nx + C.lat_r);
    }
    llat[start + q] = v;
  }
}

// FP32 column walk with the learned surrogate's gravity, maps in memory (the
// 192-pixel walk): one workgroup of 512 threads per leaf block, thread t owns
// cell t, the block's list streams through LDS once.  Per chunk of list
// entries each wave first runs its batch of 32 (cell group, entry) pairs
// through the network on the matrix cores (the groups and the Taylor step of
// the surrogate walk: the ten channels at the group centre, unfolded, left in
// LDS), then every thread takes, for each entry of the chunk, the gravity
// from its group's channels and the column binning and map update of the
// column walk.  Waves in their network phase and waves waiting on map
// traffic share each compute unit.
// list entries per LDS tile: the column walk's, so that the rows of more than
// four pixels finish at the same points of the list and the maps agree bit
// for bit with the table walk's
constexpr int FTILE = TILE;

template <int BC>
__global__ __launch_bounds__(512) void k_eval_cols_mlp(DevTree T, EwaldP E, ColP C, const void *__restrict__ pk,
                                                       const int64_t *__restrict__ off,
                                                       const double4 *__restrict__ rec,
                                                       const int32_t *__restrict__ llat,
                                                       const double *__restrict__ lh, float *__restrict__ phi,
                                                       float *__restrict__ acc, float *__restrict__ npix,
                                                       float *__restrict__ tau, float negG, double tmax) {
  using namespace mlpdef;
  __shared__ uint8_t lut[LUT_BYTES];
  __shared__ f16x8 wl[64 * NPK];
  __shared__ ColRec tile[FTILE];
  extern __shared__ __align__(16) unsigned char smem[];
  double *thr = reinterpret_cast<double *>(smem);
  float *slot = reinterpret_cast<float *>(thr + ((C.nthr + 1) & ~1));  // 16-byte aligned
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, m = l & 31;
  const int ci = tid, ii = ci & 7, jj = (ci >> 3) & 7, kk = ci >> 6;
  const int64_t ncell = T.nb * 512;
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const int64_t bx = T.bcoord[3 * b], by = T.bcoord[3 * b + 1], bz = T.bcoord[3 * b + 2];
  const double cx = centre_coord(T.org[0], 8 * bx + ii, h);
  const double cy = centre_coord(T.org[1], 8 * by + jj, h);
  const double cz = centre_coord(T.org[2], 8 * bz + kk, h);
  for (int q = tid; q < LUT_BYTES; q += 512) lut[q] = C.lut[q];
  for (int q = tid; q < C.nthr; q += 512) thr[q] = C.thr[q];
  const mlpinf::Ops W = mlpinf::load_ops(pk, wl);  // ends with a barrier
  const f16x8 one = mlpinf::ones();
  // this cell's map in the output (a wave's 64 cells are adjacent)
  char *const mcell = reinterpret_cast<char *>(npix + b * C.npix * 512 + ci);
  constexpr int lmap = 11;  // pixel p of the cell at byte offset p << 11 (512 floats per pixel)
  for (int p = 0; p < C.npix; ++p) *reinterpret_cast<float *>(mcell + (p << lmap)) = 0.0f;
  const float inv_omega = (float)(1.0 / C.omega);
  // groups of the surrogate walk
  const int gl = mlp_group_level(h, tmax);
  const int gs = 1 << gl, ga = 8 >> gl, G = ga * ga * ga;
  const int P = taylor_pairs(gl), CH = P / G;
  const double gsz = h * (double)gs;
  auto gcentre = [&](int g, double c[3]) {
    const int gx = g % ga, gy = (g / ga) % ga, gz = g / (ga * ga);
    c[0] = centre_coord(T.org[0], ga * bx + gx, gsz);
    c[1] = centre_coord(T.org[1], ga * by + gy, gsz);
    c[2] = centre_coord(T.org[2], ga * bz + gz, gsz);
  };
  const int mg = (ii >> gl) + ga * ((jj >> gl) + ga * (kk >> gl));
  float dlx, dly, dlz;
  {
    double gc[3];
    gcentre(mg, gc);
    dlx = (float)(cx - gc[0]);
    dly = (float)(cy - gc[1]);
    dlz = (float)(cz - gc[2]);
  }
  const float fa = (float)E.far_phi_a, fb = (float)E.far_phi_b, faz = (float)E.far_az;
  float ks = 0.f, kc = 0.f, ax = 0.f, ay = 0.f, az = 0.f;
  // Cells of this block's size at lattice offsets take their table row from
  // the lattice rows (their entries' rows for the block's first cell come
  // with the list, llat >= 0), as in the column walk with its maps in LDS
  const int lat_w = 2 * C.lat_r + 1;
  const int lat_lane = (kk * lat_w + jj) * lat_w + ii;
  // rows of more than four pixels finish from a per-thread queue at the
  // tile's end (as in the column walk)
  constexpr int DQ = 4;
  uint32_t dq_code[DQ] = {};
  float dq_base[DQ] = {};
  int dq_n = 0;
  auto long_row = [&](uint32_t code, float base) {
    const int o0 = (int)(code & 0x3ffffffu), o1 = o0 + (int)(code >> 26);
    const float base24 = base * (1.0f / 16777216.0f);
    for (int o = o0 + 4; o < o1; o += 2) {
      const uint32_t v = C.ent[o], u = o + 1 < o1 ? C.ent[o + 1] : 0u;
      float *const qv = reinterpret_cast<float *>(mcell + ((v >> 24) << lmap));
      *qv += (float)(v & 0xffffffu) * base24;
      float *const qu = reinterpret_cast<float *>(mcell + ((u >> 24) << lmap));
      *qu += (float)(u & 0xffffffu) * base24;
    }
  };
  const int64_t start = off[b], n = off[b + 1] - start;
  for (int64_t t0 = 0; t0 < n; t0 += FTILE) {
    const int mt = (int)(n - t0 < FTILE ? n - t0 : FTILE);
    __syncthreads();  // the previous tile is consumed
    if (tid < mt) {
      const double4 rq = rec[start + t0 + tid];
      const double hn = lh[start + t0 + tid];
      const double rh = C.req * hn;  // radius of the equal-volume sphere
      tile[tid].x = rq.x;
      tile[tid].y = rq.y;
      tile[tid].z = rq.z;
      tile[tid].w = rq.w;
      // rhs carries the lattice flag in its sign
      const int32_t li = llat[start + t0 + tid];
      const bool lat = li >= 0;
      if (lat) tile[tid].lat = li;
      else tile[tid].rh2 = rh * rh;
      tile[tid].rhs = (lat ? -1.0f : 1.0f) * ((float)rh * C.lut_ps);
      tile[tid].m = (float)rq.w;
    }
    float tx = 0.f, ty = 0.f, tz = 0.f;
    for (int j0 = 0; j0 < mt; j0 += CH) {
      __syncthreads();  // tile loaded; the previous chunk's channels are consumed
      // network phase: pairs 32 (w + 8 q) + m, entry p / G, group p % G;
      // entries past the tile's end repeat its last (their channels are never read)
      for (int q = 0; q < P / 256; ++q) {
        const int p = 32 * (w + 8 * q) + m;
        const int j = j0 + p / G < mt ? j0 + p / G : mt - 1;
        double gc[3];
        gcentre(p % G, gc);
        const ColRec &r = tile[j];
        const double ex = wrap_axis(gc[0] - r.x, E.L[0], E.inv_L[0], 1);
        const double ey = wrap_axis(gc[1] - r.y, E.L[1], E.inv_L[1], 1);
        const double ez = wrap_axis(gc[2] - r.z, E.L[2], E.inv_L[2], BC == 1);
        const float dx = (float)ex, dy = (float)ey, dz = (float)ez;
        float y[NO];
        mlpinf::forward(W, mlpinf::input(fabsf(dx), fabsf(dy), fabsf(dz)), one, y);
        const float sx = ex < 0 ? -1.f : 1.f, sy = ey < 0 ? -1.f : 1.f, sz = ez < 0 ? -1.f : 1.f;
        const bool far = BC == 2 && fabs(ez) > E.zfar;
        float4 *o = reinterpret_cast<float4 *>(slot + TSLOT * (32 * (w + 8 * q) + m));
        if (l < 32) {
          o[0] = make_float4(y[0], sx * y[1], sy * y[2], sz * y[3]);
          o[1] = make_float4(y[4], y[5], y[6], sx * sy * y[7]);
        } else {
          o[2] = make_float4(sx * sz * y[8], sy * sz * y[9], dx, dy);
          o[3] = make_float4(dz, far ? 1.f : 0.f, 0.f, 0.f);
        }
      }
      __syncthreads();
      // cell phase, software-pipelined by one entry: entry j's map reads are
      // issued, then entry j + 1's gravity, bins and row-record load, then
      // entry j's map writes, so the map reads' latency overlaps the next
      // entry's arithmetic and the record's the map writes (the order of every
      // sum is that of the plain loop)
      const int mc = mt - j0 < CH ? mt - j0 : CH;
      struct PendingRow {
        uint4 pq, wq;  // the row's four-slot record
        float base;    // M / (r^2 omega), 0 outside the column reach
        bool col;
      };
      auto row_stage = [&](int jj) {
        const ColRec r = tile[j0 + jj];
        // gravity: Newtonian part and the Taylor step from the group's channels
        float r2, inv;
        {
          const float4 *o = reinterpret_cast<const float4 *>(slot + TSLOT * (jj * G + mg));
          const float4 v0 = o[0], v1 = o[1], v2 = o[2], v3 = o[3];
          const float dx = v2.z + dlx, dy = v2.w + dly, dz = v3.x + dlz;
          r2 = dx * dx + dy * dy + dz * dz;
          const bool valid = r2 != 0.0f;
          inv = valid ? __builtin_amdgcn_rsqf(fmaxf(r2, 1e-30f)) : 0.0f;
          const float inv3 = inv * inv * inv;
          float ph, A0, A1, A2;
          if (BC == 2 && v3.y != 0.0f) {
            ph = fa * fabsf(dz) + fb;
            A0 = 0.0f;
            A1 = 0.0f;
            A2 = dz < 0 ? -faz : faz;
          } else {
            ph = inv + (v0.x - (v0.y * dlx + v0.z * dly + v0.w * dlz));
            A0 = dx * inv3 + (v0.y - (v1.x * dlx + v1.w * dly + v2.x * dlz));
            A1 = dy * inv3 + (v0.z - (v1.w * dlx + v1.y * dly + v2.y * dlz));
            A2 = dz * inv3 + (v0.w - (v2.x * dlx + v2.y * dly + v1.z * dlz));
          }
          const float mw = valid ? r.m : 0.0f;
          const float yk = mw * ph - kc, tk = ks + yk;
          kc = (tk - ks) - yk;
          ks = tk;
          tx += mw * A0;
          ty += mw * A1;
          tz += mw * A2;
        }
        // columns: the direction bins and the table row's four-slot record.
        // A lattice cell's row comes with the list; its offset from the group
        // centre and the cell's from it are whole multiples of h / 2, so the
        // gravity's FP32 r^2 is exact and equals the FP64 one: the column
        // weight uses it directly (the record is the workgroup's: a uniform
        // branch).  Other records take the FP64 minimum-image offset.
        bool col;
        float rd;
        int e;
        if (__builtin_amdgcn_readfirstlane(r.rhs < 0.0f ? 1 : 0)) {
          e = r.lat + lat_lane;
          col = r2 != 0.0f && (double)r2 <= C.max_dist2;
          rd = inv;
        } else {
          double qx = cx - r.x, qy = cy - r.y, qz = cz - r.z;
          wrap3<BC>(E, qx, qy, qz);
          const double q2 = qx * qx + qy * qy + qz * qz;
          col = q2 != 0.0 && q2 <= C.max_dist2;
          const float q2f = (float)q2;
          rd = __builtin_amdgcn_rsqf(fmaxf(q2f, 1e-30f));
          e = col ? table_row(C, thr, lut, qx, qy, qz, (float)qx, (float)qy, (float)qz, q2, q2f, rd, r.rh2, r.rhs) : 0;
        }
        const char *const rq8 = reinterpret_cast<const char *>(C.rows8) + ((uint32_t)e << 5);
        const uint4 pq = *reinterpret_cast<const uint4 *>(rq8);
        const uint4 wq = *reinterpret_cast<const uint4 *>(rq8 + 16);
        PendingRow p;
        p.pq = pq;
        p.wq = wq;
        p.base = (col ? r.m : 0.0f) * rd * rd * inv_omega;
        p.col = col;
        return p;
      };
      // map values of a pending row's four slots (the padding slots, weight 0,
      // are not read: they would cost traffic)
      struct MapVals {
        float v0, v1, v2, v3;
      };
      auto map_load = [&](const PendingRow &p) {
        MapVals m;
        m.v1 = m.v2 = m.v3 = 0.f;
        m.v0 = *reinterpret_cast<const float *>(mcell + (p.pq.x << lmap));
        if (__uint_as_float(p.wq.y) != 0.0f) m.v1 = *reinterpret_cast<const float *>(mcell + (p.pq.y << lmap));
        if (__uint_as_float(p.wq.z) != 0.0f) m.v2 = *reinterpret_cast<const float *>(mcell + (p.pq.z << lmap));
        if (__uint_as_float(p.wq.w) != 0.0f) m.v3 = *reinterpret_cast<const float *>(mcell + (p.pq.w << lmap));
        return m;
      };
      auto map_store = [&](const PendingRow &p, const MapVals &m) {
        const uint4 pq = p.pq, wq = p.wq;
        const float base = p.base;
        const bool col = p.col;
        const float w0 = __uint_as_float(wq.x), w1 = __uint_as_float(wq.y), w2 = __uint_as_float(wq.z),
                    w3 = __uint_as_float(wq.w);
        *reinterpret_cast<float *>(mcell + (pq.x << lmap)) = fmaf(w0, base, m.v0);
        if (w1 != 0.0f) *reinterpret_cast<float *>(mcell + (pq.y << lmap)) = fmaf(w1, base, m.v1);
        if (w2 != 0.0f) *reinterpret_cast<float *>(mcell + (pq.z << lmap)) = fmaf(w2, base, m.v2);
        if (w3 != 0.0f) *reinterpret_cast<float *>(mcell + (pq.w << lmap)) = fmaf(w3, base, m.v3);
        if ((int)pq.x < 0 && col) {
          const uint32_t cnt = (pq.x >> 23) & 63u;
          const uint32_t o0 = (pq.y >> 23) | ((pq.z >> 23) << 9) | ((pq.w >> 23) << 18);
          if (dq_n == DQ) {
            long_row(dq_code[DQ - 1], dq_base[DQ - 1]);
            --dq_n;
          }
          for (int k = DQ - 1; k > 0; --k) {
            dq_code[k] = dq_code[k - 1];
            dq_base[k] = dq_base[k - 1];
          }
          dq_code[0] = (cnt << 26) | o0;
          dq_base[0] = base;
          ++dq_n;
        }
      };
      PendingRow cur = row_stage(0);
      for (int j = 0; j < mc; ++j) {
        const MapVals mv = map_load(cur);
        PendingRow nxt = cur;
        if (j + 1 < mc) nxt = row_stage(j + 1);
        map_store(cur, mv);
        cur = nxt;
      }
    }
    for (int k = 0; k < DQ; ++k)
      if (k < dq_n) long_row(dq_code[k], dq_base[k]);
    dq_n = 0;
    ax += tx;
    ay += ty;
    az += tz;
  }
  const int64_t o = b * 512 + ci;
  phi[o] = negG * (ks - kc);
  acc[o] = negG * ax;
  acc[ncell + o] = negG * ay;
  acc[2 * ncell + o] = negG * az;
  double se = 0.0;
  for (int p = 0; p < C.npix; ++p) se += exp(-C.kappa * (double)*reinterpret_cast<const float *>(mcell + (p << lmap)));
  tau[o] = (float)(-log(se / (double)C.npix));
}

// LDS written by lanes of a wave, then read by other lanes of the same wave
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same walk with one list per 4^3 octant of the block (the group walk's
// MAC suite against the octant's box: shorter lists).  Wave w owns octant w
// (bit a: upper half of axis a) and walks its list alone: its own LDS tile of
// 32 entries, its own network batch (32 (cell group, entry) pairs, the cell
// groups of 2^3 or 4^3 cells lying inside the octant) and wave-level
// synchronisation only, so the eight waves of a workgroup never wait on each
// other inside the walk.  Lane l owns cell (l & 3, (l >> 2) & 3, l >> 4) of
// the octant.  A wave's 64 maps are accumulated in adjacent slots of each
// pixel row of npix (slot 64 w + l), and put in the cell order i + 8 j + 64 k
// at the end, eight pixel rows at a time between workgroup barriers.
// Occupancy: 4 waves per SIMD (two workgroups per compute unit) at up to 128
// registers.
template <int BC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_cols_mlp4(
    DevTree T, EwaldP E, ColP C, const void *__restrict__ pk, const int64_t *__restrict__ off,
    const double4 *__restrict__ rec, const int32_t *__restrict__ llat, const double *__restrict__ lh,
    float *__restrict__ phi, float *__restrict__ acc, float *__restrict__ npix, float *__restrict__ tau,
    float negG, double tmax) {
  using namespace mlpdef;
  __shared__ uint8_t lut[LUT_BYTES];
  __shared__ f16x8 wl[64 * NPK];
  constexpr int FT4 = 32;  // list entries per wave tile
  __shared__ ColRec tiles[8][FT4];
  extern __shared__ __align__(16) unsigned char smem[];
  double *thr = reinterpret_cast<double *>(smem);
  const int64_t b = blockIdx.x;
  // the wave index is uniform across the wave: kept in a scalar register, so
  // that each wave's list bounds and loops stay scalar
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, m = l & 31;
  float *slot = reinterpret_cast<float *>(thr + ((C.nthr + 1) & ~1)) + 32 * TSLOT * w;
  // wave w walks octant w (4^3 cells) with its own list; lane l its cell
  const int sx = w & 1, sy = (w >> 1) & 1, sz = w >> 2;
  const int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
  const int ii = 4 * sx + lx, jj = 4 * sy + ly, kk = 4 * sz + lz;
  const int ci = ii + 8 * jj + 64 * kk;
  ColRec *const tile = tiles[w];
  const int64_t ncell = T.nb * 512;
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const int64_t bx = T.bcoord[3 * b], by = T.bcoord[3 * b + 1], bz = T.bcoord[3 * b + 2];
  const double cx = centre_coord(T.org[0], 8 * bx + ii, h);
  const double cy = centre_coord(T.org[1], 8 * by + jj, h);
  const double cz = centre_coord(T.org[2], 8 * bz + kk, h);
  for (int q = tid; q < LUT_BYTES; q += 512) lut[q] = C.lut[q];
  for (int q = tid; q < C.nthr; q += 512) thr[q] = C.thr[q];
  const mlpinf::Ops W = mlpinf::load_ops(pk, wl);  // ends with a barrier
  const f16x8 one = mlpinf::ones();
  // this cell's map in the output while the walk runs: slot 64 w + l = tid
  // of each pixel row
  char *const mcell = reinterpret_cast<char *>(npix + b * C.npix * 512 + tid);
  constexpr int lmap = 11;  // pixel p of the cell at byte offset p << 11 (512 floats per pixel)
  for (int p = 0; p < C.npix; ++p) *reinterpret_cast<float *>(mcell + (p << lmap)) = 0.0f;
  const float inv_omega = (float)(1.0 / C.omega);
  // groups of the surrogate walk
  const int gl = mlp_group_level(h, tmax);  // 1 or 2: the host checks the largest cells
  const int gs = 1 << gl, ga = 8 >> gl, g4 = 4 >> gl, G = g4 * g4 * g4;
  const int CH = 32 / G;
  const double gsz = h * (double)gs;
  auto gcentre = [&](int g, double c[3]) {
    const int gx = g % g4, gy = (g / g4) % g4, gz = g / (g4 * g4);
    c[0] = centre_coord(T.org[0], ga * bx + g4 * sx + gx, gsz);
    c[1] = centre_coord(T.org[1], ga * by + g4 * sy + gy, gsz);
    c[2] = centre_coord(T.org[2], ga * bz + g4 * sz + gz, gsz);
  };
  const int mg = (lx >> gl) + g4 * ((ly >> gl) + g4 * (lz >> gl));
  float dlx, dly, dlz;
  {
    double gc[3];
    gcentre(mg, gc);
    dlx = (float)(cx - gc[0]);
    dly = (float)(cy - gc[1]);
    dlz = (float)(cz - gc[2]);
  }
  const float fa = (float)E.far_phi_a, fb = (float)E.far_phi_b, faz = (float)E.far_az;
  float ks = 0.f, kc = 0.f, ax = 0.f, ay = 0.f, az = 0.f;
  // Cells of this block's size at lattice offsets take their table row from
  // the lattice rows (their entries' rows for the octant's first cell come
  // with the list, llat >= 0), as in the column walk with its maps in LDS
  const int lat_w = 2 * C.lat_r + 1;
  const int lat_lane = (lz * lat_w + ly) * lat_w + lx;
  // rows of more than four pixels finish from a per-thread queue at the
  // tile's end (as in the column walk)
  constexpr int DQ = 4;
  uint32_t dq_code[DQ] = {};
  float dq_base[DQ] = {};
  int dq_n = 0;
  auto long_row = [&](uint32_t code, float base) {
    const int o0 = (int)(code & 0x3ffffffu), o1 = o0 + (int)(code >> 26);
    const float base24 = base * (1.0f / 16777216.0f);
    for (int o = o0 + 4; o < o1; o += 2) {
      const uint32_t v = C.ent[o], u = o + 1 < o1 ? C.ent[o + 1] : 0u;
      float *const qv = reinterpret_cast<float *>(mcell + ((v >> 24) << lmap));
      *qv += (float)(v & 0xffffffu) * base24;
      float *const qu = reinterpret_cast<float *>(mcell + ((u >> 24) << lmap));
      *qu += (float)(u & 0xffffffu) * base24;
    }
  };
  const int64_t start = off[8 * b + w], n = off[8 * b + w + 1] - start;
  for (int64_t t0 = 0; t0 < n; t0 += FT4) {
    const int mt = (int)(n - t0 < FT4 ? n - t0 : FT4);
    wave_sync();  // the previous tile is consumed
    if (l < mt) {
      const int tid = l;
      const double4 rq = rec[start + t0 + tid];
      const double hn = lh[start + t0 + tid];
      const double rh = C.req * hn;  // radius of the equal-volume sphere
      tile[tid].x = rq.x;
      tile[tid].y = rq.y;
      tile[tid].z = rq.z;
      tile[tid].w = rq.w;
      // rhs carries the lattice flag in its sign
      const int32_t li = llat[start + t0 + tid];
      const bool lat = li >= 0;
      if (lat) tile[tid].lat = li;
      else tile[tid].rh2 = rh * rh;
      tile[tid].rhs = (lat ? -1.0f : 1.0f) * ((float)rh * C.lut_ps);
      tile[tid].m = (float)rq.w;
    }
    float tx = 0.f, ty = 0.f, tz = 0.f;
    for (int j0 = 0; j0 < mt; j0 += CH) {
      wave_sync();  // tile loaded; the previous chunk's channels are consumed
      // network phase: pairs m, entry m / G, group m % G of this sub-block
      {
        const int p = m;
        const int j = j0 + p / G < mt ? j0 + p / G : mt - 1;
        double gc[3];
        gcentre(p % G, gc);
        const ColRec &r = tile[j];
        const double ex = wrap_axis(gc[0] - r.x, E.L[0], E.inv_L[0], 1);
        const double ey = wrap_axis(gc[1] - r.y, E.L[1], E.inv_L[1], 1);
        const double ez = wrap_axis(gc[2] - r.z, E.L[2], E.inv_L[2], BC == 1);
        const float dx = (float)ex, dy = (float)ey, dz = (float)ez;
        float y[NO];
        mlpinf::forward(W, mlpinf::input(fabsf(dx), fabsf(dy), fabsf(dz)), one, y);
        const float sx = ex < 0 ? -1.f : 1.f, sy = ey < 0 ? -1.f : 1.f, sz = ez < 0 ? -1.f : 1.f;
        const bool far = BC == 2 && fabs(ez) > E.zfar;
        float4 *o = reinterpret_cast<float4 *>(slot + TSLOT * p);
        if (l < 32) {
          o[0] = make_float4(y[0], sx * y[1], sy * y[2], sz * y[3]);
          o[1] = make_float4(y[4], y[5], y[6], sx * sy * y[7]);
        } else {
          o[2] = make_float4(sx * sz * y[8], sy * sz * y[9], dx, dy);
          o[3] = make_float4(dz, far ? 1.f : 0.f, 0.f, 0.f);
        }
      }
      wave_sync();
      // cell phase, software-pipelined by one entry: entry j's map reads are
      // issued, then entry j + 1's gravity, bins and row-record load, then
      // entry j's map writes, so the map reads' latency overlaps the next
      // entry's arithmetic and the record's the map writes (the order of every
      // sum is that of the plain loop)
      const int mc = mt - j0 < CH ? mt - j0 : CH;
      struct PendingRow {
        uint4 pq, wq;  // the row's four-slot record
        float base;    // M / (r^2 omega), 0 outside the column reach
        bool col;
      };
      auto row_stage = [&](int jj) {
        const ColRec r = tile[j0 + jj];
        // gravity: Newtonian part and the Taylor step from the group's channels
        float r2, inv;
        {
          const float4 *o = reinterpret_cast<const float4 *>(slot + TSLOT * (jj * G + mg));
          const float4 v0 = o[0], v1 = o[1], v2 = o[2], v3 = o[3];
          const float dx = v2.z + dlx, dy = v2.w + dly, dz = v3.x + dlz;
          r2 = dx * dx + dy * dy + dz * dz;
          const bool valid = r2 != 0.0f;
          inv = valid ? __builtin_amdgcn_rsqf(fmaxf(r2, 1e-30f)) : 0.0f;
          const float inv3 = inv * inv * inv;
          float ph, A0, A1, A2;
          if (BC == 2 && v3.y != 0.0f) {
            ph = fa * fabsf(dz) + fb;
            A0 = 0.0f;
            A1 = 0.0f;
            A2 = dz < 0 ? -faz : faz;
          } else {
            ph = inv + (v0.x - (v0.y * dlx + v0.z * dly + v0.w * dlz));
            A0 = dx * inv3 + (v0.y - (v1.x * dlx + v1.w * dly + v2.x * dlz));
            A1 = dy * inv3 + (v0.z - (v1.w * dlx + v1.y * dly + v2.y * dlz));
            A2 = dz * inv3 + (v0.w - (v2.x * dlx + v2.y * dly + v1.z * dlz));
          }
          const float mw = valid ? r.m : 0.0f;
          const float yk = mw * ph - kc, tk = ks + yk;
          kc = (tk - ks) - yk;
          ks = tk;
          tx += mw * A0;
          ty += mw * A1;
          tz += mw * A2;
        }
        // columns: the direction bins and the table row's four-slot record.
        // A lattice cell's row comes with the list; its offset from the group
        // centre and the cell's from it are whole multiples of h / 2, so the
        // gravity's FP32 r^2 is exact and equals the FP64 one: the column
        // weight uses it directly (the record is the workgroup's: a uniform
        // branch).  Other records take the FP64 minimum-image offset.
        bool col;
        float rd;
        int e;
        if (__builtin_amdgcn_readfirstlane(r.rhs < 0.0f ? 1 : 0)) {
          e = r.lat + lat_lane;
          col = r2 != 0.0f && (double)r2 <= C.max_dist2;
          rd = inv;
        } else {
          double qx = cx - r.x, qy = cy - r.y, qz = cz - r.z;
          wrap3<BC>(E, qx, qy, qz);
          const double q2 = qx * qx + qy * qy + qz * qz;
          col = q2 != 0.0 && q2 <= C.max_dist2;
          const float q2f = (float)q2;
          rd = __builtin_amdgcn_rsqf(fmaxf(q2f, 1e-30f));
          e = col ? table_row(C, thr, lut, qx, qy, qz, (float)qx, (float)qy, (float)qz, q2, q2f, rd, r.rh2, r.rhs) : 0;
        }
        const char *const rq8 = reinterpret_cast<const char *>(C.rows8) + ((uint32_t)e << 5);
        const uint4 pq = *reinterpret_cast<const uint4 *>(rq8);
        const uint4 wq = *reinterpret_cast<const uint4 *>(rq8 + 16);
        PendingRow p;
        p.pq = pq;
        p.wq = wq;
        p.base = (col ? r.m : 0.0f) * rd * rd * inv_omega;
        p.col = col;
        return p;
      };
      // map values of a pending row's four slots (the padding slots, weight 0,
      // are not read: they would cost traffic)
      struct MapVals {
        float v0, v1, v2, v3;
      };
      auto map_load = [&](const PendingRow &p) {
        MapVals m;
        m.v1 = m.v2 = m.v3 = 0.f;
        m.v0 = *reinterpret_cast<const float *>(mcell + (p.pq.x << lmap));
        if (__uint_as_float(p.wq.y) != 0.0f) m.v1 = *reinterpret_cast<const float *>(mcell + (p.pq.y << lmap));
        if (__uint_as_float(p.wq.z) != 0.0f) m.v2 = *reinterpret_cast<const float *>(mcell + (p.pq.z << lmap));
        if (__uint_as_float(p.wq.w) != 0.0f) m.v3 = *reinterpret_cast<const float *>(mcell + (p.pq.w << lmap));
        return m;
      };
      auto map_store = [&](const PendingRow &p, const MapVals &m) {
        const uint4 pq = p.pq, wq = p.wq;
        const float base = p.base;
        const bool col = p.col;
        const float w0 = __uint_as_float(wq.x), w1 = __uint_as_float(wq.y), w2 = __uint_as_float(wq.z),
                    w3 = __uint_as_float(wq.w);
        *reinterpret_cast<float *>(mcell + (pq.x << lmap)) = fmaf(w0, base, m.v0);
        if (w1 != 0.0f) *reinterpret_cast<float *>(mcell + (pq.y << lmap)) = fmaf(w1, base, m.v1);
        if (w2 != 0.0f) *reinterpret_cast<float *>(mcell + (pq.z << lmap)) = fmaf(w2, base, m.v2);
        if (w3 != 0.0f) *reinterpret_cast<float *>(mcell + (pq.w << lmap)) = fmaf(w3, base, m.v3);
        if ((int)pq.x < 0 && col) {
          const uint32_t cnt = (pq.x >> 23) & 63u;
          const uint32_t o0 = (pq.y >> 23) | ((pq.z >> 23) << 9) | ((pq.w >> 23) << 18);
          if (dq_n == DQ) {
            long_row(dq_code[DQ - 1], dq_base[DQ - 1]);
            --dq_n;
          }
          for (int k = DQ - 1; k > 0; --k) {
            dq_code[k] = dq_code[k - 1];
            dq_base[k] = dq_base[k - 1];
          }
          dq_code[0] = (cnt << 26) | o0;
          dq_base[0] = base;
          ++dq_n;
        }
      };
      PendingRow cur = row_stage(0);
      for (int j = 0; j < mc; ++j) {
        const MapVals mv = map_load(cur);
        PendingRow nxt = cur;
        if (j + 1 < mc) nxt = row_stage(j + 1);
        map_store(cur, mv);
        cur = nxt;
      }
    }
    for (int k = 0; k < DQ; ++k)
      if (k < dq_n) long_row(dq_code[k], dq_base[k]);
    dq_n = 0;
    ax += tx;
    ay += ty;
    az += tz;
  }
  const int64_t o = b * 512 + ci;
  phi[o] = negG * (ks - kc);
  acc[o] = negG * ax;
  acc[ncell + o] = negG * ay;
  acc[2 * ncell + o] = negG * az;
  double se = 0.0;
  for (int p = 0; p < C.npix; ++p) se += exp(-C.kappa * (double)*reinterpret_cast<const float *>(mcell + (p << lmap)));
  tau[o] = (float)(-log(se / (double)C.npix));
  // slot order -> cell order, eight pixel rows at a time (every slot of a
  // row is read before any is overwritten)
  float *const rows = npix + b * C.npix * 512;
  for (int p0 = 0; p0 < C.npix; p0 += 8) {
    float v[8];
    __syncthreads();
    for (int q = 0; q < 8; ++q) v[q] = p0 + q < C.npix ? rows[(p0 + q) * 512 + tid] : 0.0f;
    __syncthreads();
    for (int q = 0; q < 8; ++q)
      if (p0 + q < C.npix) rows[(p0 + q) * 512 + ci] = v[q];
  }
}


// table rows of arbitrary offsets d = cell - node with the walk's binning
// (thresholds and look-up tables in LDS as in the walk); -1 for d = 0
__global__ __launch_bounds__(256) void k_column_bins(ColP C, int64_t n, const double *__restrict__ d,
                                                     const double *__restrict__ hn, int32_t *__restrict__ row) {
  __shared__ uint8_t lut[LUT_BYTES];
  extern __shared__ __align__(16) unsigned char smem[];
  double *thr = reinterpret_cast<double *>(smem);
  for (int q = threadIdx.x; q < LUT_BYTES; q += 256) lut[q] = C.lut[q];
  for (int q = threadIdx.x; q < C.nthr; q += 256) thr[q] = C.thr[q];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = i < n;
  // every lane runs the binning (its fallback is decided by a wave vote)
  const double dx = in ? d[3 * i] : 1.0, dy = in ? d[3 * i + 1] : 0.0, dz = in ? d[3 * i + 2] : 0.0;
  const double h = in ? hn[i] : 0.0;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const float r2f = (float)r2;
  const float rd = __builtin_amdgcn_rsqf(fmaxf(r2f, 1e-30f));
  const double rh = C.req * h;
  const int e = r2 != 0.0 ? table_row(C, thr, lut, dx, dy, dz, (float)dx, (float)dy, (float)dz, r2, r2f, rd,
                                      rh * rh, (float)rh * C.lut_ps)
                          : -1;
  if (in) row[i] = e;
}

// rows of the lattice offsets d = (i, j, k) (in cell sizes, node size 1),
// copied from the table row that the walk's own binning gives (head and
// packed record); the origin gets an empty row
__global__ __launch_bounds__(256) void k_lattice_rows(ColP C, int R, uint32_t *__restrict__ out,
                                                      uint4 *__restrict__ out8, double *__restrict__ out_w64) {
  __shared__ uint8_t lut[LUT_BYTES];
  extern __shared__ __align__(16) unsigned char smem[];
  double *thr = reinterpret_cast<double *>(smem);
  for (int q = threadIdx.x; q < LUT_BYTES; q += 256) lut[q] = C.lut[q];
  for (int q = threadIdx.x; q < C.nthr; q += 256) thr[q] = C.thr[q];
  __syncthreads();
  const int W = 2 * R + 1;
  const int n = W * W * W;
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int tt = t < n ? t : 0;
  const double dz = (double)(tt / (W * W) - R), dy = (double)((tt / W) % W - R), dx = (double)(tt % W - R);
  const double r2 = dx * dx + dy * dy + dz * dz;
  const float r2f = (float)r2;
  const float rd = __builtin_amdgcn_rsqf(fmaxf(r2f, 1e-30f));
  const double rh = C.req;
  const int e = r2 != 0.0 ? table_row(C, thr, lut, dx, dy, dz, (float)dx, (float)dy, (float)dz, r2, r2f, rd,
                                      rh * rh, (float)rh * C.lut_ps)
                          : -1;
  if (t < n) {
    out[t] = e >= 0 ? C.rows[e] : 0u;
    out8[2 * t] = e >= 0 ? C.rows8[2 * e] : make_uint4(0, 1, 2, 3);
    out8[2 * t + 1] = e >= 0 ? C.rows8[2 * e + 1] : make_uint4(0, 0, 0, 0);
    for (int k = 0; k < 4; ++k) out_w64[4 * (int64_t)t + k] = e >= 0 ? C.quad_w64[4 * (int64_t)e + k] : 0.0;
  }
}

// packed rows for the walk: head = offset << 6 | count; entry = pixel << 24 |
// round(w 2^24) (w <= 1, clamped to 2^24 - 1); rows8 = the first four pixels
// and their FP32 weights, padded with the lowest pixels the row does not use
// (weight 0); a row of more than four has bit 31 of the first pixel set and
// its count and offset in the pixels' bits 23..30 / 23..31
__global__ void k_raytable_pack(RayTableP P, const int64_t *__restrict__ off, const uint16_t *__restrict__ pix,
                                const double *__restrict__ w, uint32_t *__restrict__ rows,
                                uint32_t *__restrict__ ent, uint4 *__restrict__ rows8,
                                double *__restrict__ quad_w64) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P.nentries) return;
  const int64_t o0 = off[e], o1 = off[e + 1];
  const uint32_t head = (uint32_t)(o0 << 6) | (uint32_t)(o1 - o0);
  rows[e] = head;
  uint32_t p4[4], w4[4];
  double d4[4];
  int nf = 0;
  for (int64_t o = o0; o < o1; ++o) {
    double q = rint(w[o] * 16777216.0);
    q = q > 16777215.0 ? 16777215.0 : q;
    ent[o] = ((uint32_t)pix[o] << 24) | (uint32_t)q;
    if (nf < 4) {
      p4[nf] = pix[o];
      w4[nf] = __float_as_uint((float)w[o]);
      d4[nf] = w[o];
      ++nf;
    }
  }
  // padding (rows of fewer than four): the lowest pixels not in the row
  uint32_t cand = 0;
  while (nf < 4) {
    bool used = false;
    for (int i = 0; i < nf; ++i) used |= p4[i] == cand;
    if (!used) {
      p4[nf] = cand;
      w4[nf] = 0u;
      d4[nf] = 0.0;
      ++nf;
    }
    ++cand;
  }
  if (o1 - o0 > 4) {
    // more than four: flag, count and offset (< 2^26) in bits 23..31 of the
    // pixels (the walks shift the pixels by at least 9 bits into 32-bit
    // addresses, which drops these bits)
    p4[0] |= 0x80000000u | ((uint32_t)(o1 - o0) << 23);
    p4[1] |= (uint32_t)(o0 & 511) << 23;
    p4[2] |= (uint32_t)((o0 >> 9) & 511) << 23;
    p4[3] |= (uint32_t)((o0 >> 18) & 511) << 23;
  }
  rows8[2 * e] = make_uint4(p4[0], p4[1], p4[2], p4[3]);
  rows8[2 * e + 1] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
  for (int k = 0; k < 4; ++k) quad_w64[4 * (int64_t)e + k] = d4[k];
}

}  // namespace

hipError_t launch_column_bins(const ColP &C, int64_t n, const double *d, const double *h, int32_t *row,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_column_bins, dim3((unsigned)((n + 255) / 256)), dim3(256), C.nthr * sizeof(double), st, C,
                     n, d, h, row);
  return hipGetLastError();
}

hipError_t launch_lattice_rows(const ColP &C, int R, uint32_t *rows, uint4 *rows8, double *quad_w64,
                               hipStream_t st) {
  const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
  hipLaunchKernelGGL(k_lattice_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), C.nthr * sizeof(double), st, C,
                     R, rows + C.lat0, rows8 + 2 * (int64_t)C.lat0, quad_w64 + 4 * (int64_t)C.lat0);
  return hipGetLastError();
}

hipError_t launch_raytable(const RayTableP &P, double *dense, int32_t *cnt, int64_t *off, uint16_t *pix,
                           double *w64, int64_t *total, hipStream_t st) {
  hipLaunchKernelGGL(k_raytable_dense, dim3((unsigned)P.nentries), dim3(64), 0, st, P, dense);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)((P.nentries + 255) / 256);
  hipLaunchKernelGGL(k_raytable_count, dim3(nb), dim3(256), 0, st, P, dense, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_scan(cnt, P.nentries, off, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(total, off + P.nentries, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (!pix) return hipSuccess;  // sizing pass
  hipLaunchKernelGGL(k_raytable_fill, dim3(nb), dim3(256), 0, st, P, dense, off, pix, w64);
  return hipGetLastError();
}

constexpr size_t COLS_STATIC_LDS = LUT_BYTES + TILE * sizeof(ColRec);
static_assert(sizeof(ColRec) == 48, "list record of the column walk");

size_t cols_smem_bytes(int npix, int cpw, bool fp64, int nthr) {
  return COLS_STATIC_LDS + (size_t)nthr * sizeof(double) + (size_t)npix * cpw * (fp64 ? 8 : 4);
}

int cols_lds_cpw(int npix, bool fp64, int nthr) {
  for (int cpw : {256, 128})
    if (cols_smem_bytes(npix, cpw, fp64, nthr) <= 65536) return cpw;
  return 0;
}

hipError_t launch_abu_corner_cols(bool fp64, const DevTree &T, const EwaldP &E, const ColP &C, const int64_t *off,
                                  const double4 *rec, const double *lh, const void *prev_npix, double tol_tau,
                                  int32_t *flags, hipStream_t st) {
  const size_t sm = (size_t)(((C.nthr + 1) & ~1) + 8 * C.npix) * sizeof(double);
  dim3 grid((unsigned)T.nb), blk(512);
#define OT_ABC(B, R)                                                                                       \
  hipLaunchKernelGGL((k_abu_corner_cols<B, R>), grid, blk, sm, st, T, E, C, off, rec, lh, (const R *)prev_npix, \
                     tol_tau, flags)
  if (fp64) {
    switch (E.bctype) {
      case 0: OT_ABC(0, double); break;
      case 1: OT_ABC(1, double); break;
      case 2: OT_ABC(2, double); break;
      default: OT_ABC(3, double); break;
    }
  } else {
    switch (E.bctype) {
      case 0: OT_ABC(0, float); break;
      case 1: OT_ABC(1, float); break;
      case 2: OT_ABC(2, float); break;
      default: OT_ABC(3, float); break;
    }
  }
#undef OT_ABC
  return hipGetLastError();
}

hipError_t launch_eval_cols_mlp(const DevTree &T, const EwaldP &E, const ColP &C, const void *pk, const int64_t *off,
                                const double4 *rec, const int32_t *ids, const double *lh, int32_t *llat, float *phi,
                                float *acc, float *npix, float *tau, double G, double tmax, double h_max,
                                int *wg_per_cu, hipStream_t st, int sub) {
  const size_t sm = (size_t)((C.nthr + 1) & ~1) * sizeof(double) +
                    (size_t)taylor_pairs(mlp_group_level(h_max, tmax)) * TSLOT * sizeof(float);
  // octant lists (sub): eight waves of 32 network pairs each; cell groups of
  // 2^3 or 4^3 cells, so that each octant holds whole groups
  const size_t sm4 = (size_t)((C.nthr + 1) & ~1) * sizeof(double) + (size_t)8 * 32 * TSLOT * sizeof(float);
  if (sub && mlp_group_level(h_max, tmax) < 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)T.nb), blk(512);
  const float ng = (float)(-G);
#define OT_LAUNCH_CM(B)                                                                                    \
  do {                                                                                                     \
    if (wg_per_cu &&                                                                                       \
        (sub ? hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_eval_cols_mlp4<B>, 512, sm4)     \
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_eval_cols_mlp<B>, 512, sm)) !=   \
            hipSuccess)                                                                                    \
      *wg_per_cu = 0;                                                                                      \
    hipLaunchKernelGGL((k_lattice_index<B>), dim3((unsigned)(sub ? 8 * T.nb : T.nb)), dim3(256), 0, st, T, E, \
                       C, off, rec, ids, lh, llat, sub);                                                    \
    if (sub)                                                                                               \
      hipLaunchKernelGGL((k_eval_cols_mlp4<B>), grid, blk, sm4, st, T, E, C, pk, off, rec, llat, lh, phi, acc, \
                         npix, tau, ng, tmax);                                                             \
    else                                                                                                   \
      hipLaunchKernelGGL((k_eval_cols_mlp<B>), grid, blk, sm, st, T, E, C, pk, off, rec, llat, lh, phi, acc,  \
                         npix, tau, ng, tmax);                                                             \
  } while (0)
  if (E.bctype == 1) OT_LAUNCH_CM(1);
  else if (E.bctype == 2) OT_LAUNCH_CM(2);
  else return hipErrorInvalidValue;
#undef OT_LAUNCH_CM
  return hipGetLastError();
}

hipError_t launch_raytable_pack(const RayTableP &P, const int64_t *off, const uint16_t *pix, const double *w,
                                uint32_t *rows, uint32_t *ent, uint4 *rows8, double *quad_w64, hipStream_t st) {
  hipLaunchKernelGGL(k_raytable_pack, dim3((unsigned)((P.nentries + 255) / 256)), dim3(256), 0, st, P, off,
                     pix, w, rows, ent, rows8, quad_w64);
  return hipGetLastError();
}

hipError_t launch_eval_cols(bool fp64, const DevTree &T, const EwaldP &E, const ColP &C, const int64_t *off,
                            const double4 *rec, const int32_t *ids, const double *lh, void *phi, void *acc,
                            void *npix, void *tau, double G, int cpw, bool no_gravity, int *wg_per_cu,
                            hipStream_t st, const int32_t *blist, int64_t nblist) {
  if (blist && nblist <= 0) return hipSuccess;
  const bool gmap = cpw == 0;
  if (gmap) cpw = 256;
  // dynamic LDS: the thresholds, and the maps unless they are in npix
  const size_t sm = gmap ? (size_t)C.nthr * sizeof(double)
                         : cols_smem_bytes(C.npix, cpw, fp64, C.nthr) - COLS_STATIC_LDS;
  int lcpw = 0;
  while ((1 << lcpw) < cpw) ++lcpw;
  if ((1 << lcpw) != cpw) return hipErrorInvalidValue;  // cells per workgroup: a power of two
  // map addresses shift the packed pixels by lcpw + 2 (FP32) or + 3 (FP64),
  // at least 9 bits (the bits above 22 hold a long row's count and offset)
  if (lcpw + (fp64 ? 3 : 2) < 9) return hipErrorInvalidValue;
  dim3 grid((unsigned)((blist ? nblist : T.nb) * (512 / cpw))), blk(cpw);
#define OT_LAUNCH2(R, B, N, M)                                                                                \
  do {                                                                                                        \
    if (sm + COLS_STATIC_LDS > 65536) {                                                                       \
      hipError_t ea = hipFuncSetAttribute((const void *)k_eval_cols<R, B, N, M>,                             \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);              \
      if (ea != hipSuccess) return ea;                                                                        \
    }                                                                                                         \
    if (wg_per_cu && hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, k_eval_cols<R, B, N, M>, cpw,   \
                                                                  sm) != hipSuccess)                          \
      *wg_per_cu = 0;                                                                                         \
    hipLaunchKernelGGL((k_eval_cols<R, B, N, M>), grid, blk, sm, st, T, E, C, off, rec, ids, lh, (R *)phi,   \
                       (R *)acc, (R *)npix, (R *)tau, -G, cpw, lcpw, blist);                                 \
  } while (0)
#define OT_LAUNCH(R, B, N)          \
  do {                              \
    if (gmap)                       \
      OT_LAUNCH2(R, B, N, true);    \
    else                            \
      OT_LAUNCH2(R, B, N, false);   \
  } while (0)
  if (fp64) {
    if (no_gravity) return hipErrorInvalidValue;
    if (E.bctype == 0) OT_LAUNCH(double, 0, false);
    else if (E.bctype == 1) OT_LAUNCH(double, 1, false);
    else if (E.bctype == 2) OT_LAUNCH(double, 2, false);
    else OT_LAUNCH(double, 3, false);
  } else if (no_gravity) {
    if (E.bctype == 1) OT_LAUNCH(float, 1, true);
    else if (E.bctype == 2) OT_LAUNCH(float, 2, true);
    else return hipErrorInvalidValue;
  } else {
    if (E.bctype == 0) OT_LAUNCH(float, 0, false);
    else if (E.bctype == 1) OT_LAUNCH(float, 1, false);
    else if (E.bctype == 2) OT_LAUNCH(float, 2, false);
    else OT_LAUNCH(float, 3, false);
  }
#undef OT_LAUNCH
#undef OT_LAUNCH2
  return hipGetLastError();
}

}  // namespace ot
