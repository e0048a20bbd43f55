// Per-cell evaluation of the block interaction lists (Sec. 2.2.1-2.2.5).
//
// Phi(r) = -G sum_a M_a phi(r - r_a), a(r) = -G sum_a M_a A(r - r_a) over the
// accepted nodes (Eqs. 7, 8 and App. A), with phi = 1/r, A = d/r^3 for
// isolated boundaries, and phi = 1/r + phi_c, A = d/r^3 + A_c for periodic
// (3P) or mixed (2P1I, 1P2I) ones, the correction taken from the table by a
// first-order Taylor expansion about the nearest grid point (second approach
// of Sec. 2.2.5) or, for 2P1I beyond |dz| = 2 Lx and for 1P2I beyond 4 Lx
// from the periodic axis, from the analytic limit.
// The target cell itself is skipped (d = 0 exactly).
//
// List records hold absolute centres of mass in FP64.  The FP64 kernel forms
// d = r - r_a (minimum image) from absolute cell centres, the same expression
// for both, so the target cell gives d = 0 exactly.  The FP32 kernel converts
// each record once per workgroup to an FP32 offset from the block centre; the
// block's own cells get the same expression as the thread's own offset, so the
// target cell again gives d = 0.
//
// One workgroup of 256 threads per leaf block; thread t owns cells t and
// t + 256 (NQ = 2).  When only a few blocks are evaluated (the adaptive block
// update), two workgroups share a block, one cell per thread (NQ = 1): the
// same arithmetic per cell in the same order, half the latency.  The list is streamed through LDS in tiles of 256 records, which
// every thread then reads as broadcasts.  The FP32 kernel accumulates Phi with
// Kahan compensation and the acceleration in plain FP32 per tile, the tile
// sums then added (blocked summation).
#include "common.hpp"
#include "ewald_lookup.hpp"
#include "kernels.hpp"

namespace ot {

namespace {

constexpr int WG = 256;
// below this many blocks two workgroups share a block (four resident
// workgroups per CU at one per block)
constexpr int64_t FEW_BLOCKS = 1024;

// ---------------------------------------------------------------- FP64
template <int BC>
__device__ inline void pair64(const EwaldP &E, double cx, double cy, double cz, const double4 r,
                              double &sp, double &ax, double &ay, double &az) {
  double dx = cx - r.x, dy = cy - r.y, dz = cz - r.z;
  if (BC != 0) {
    dx = wrap_axis(dx, E.L[0], E.inv_L[0], 1);
    if (BC != 3) dy = wrap_axis(dy, E.L[1], E.inv_L[1], 1);
    if (BC == 1) dz = wrap_axis(dz, E.L[2], E.inv_L[2], 1);
  }
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (r2 == 0.0) return;
  const double inv = 1.0 / sqrt(r2);
  const double inv3 = inv * inv * inv;
  if (BC == 0) {
    sp += r.w * inv;
    ax += r.w * inv3 * dx;
    ay += r.w * inv3 * dy;
    az += r.w * inv3 * dz;
    return;
  }
  double phi, A0, A1, A2;
  if (BC == 2 && fabs(dz) > E.zfar) {
    phi = E.far_phi_a * fabs(dz) + E.far_phi_b;
    A0 = 0.0;
    A1 = 0.0;
    A2 = dz < 0 ? -E.far_az : E.far_az;
  } else if (BC == 3 && dy * dy + dz * dz > E.zfar * E.zfar) {
    const double rho2 = dy * dy + dz * dz;
    phi = E.far_phi_a * log(rho2) + E.far_phi_b;
    A0 = 0.0;
    A1 = E.far_az * dy / rho2;
    A2 = E.far_az * dz / rho2;
  } else {
    const double u[3] = {fabs(dx), fabs(dy), fabs(dz)};
    double phic, a[3];
    table_taylor64(E, u, phic, a);
    phi = inv + phic;
    A0 = dx * inv3 + (dx < 0 ? -a[0] : a[0]);
    A1 = dy * inv3 + (dy < 0 ? -a[1] : a[1]);
    A2 = dz * inv3 + (dz < 0 ? -a[2] : a[2]);
  }
  sp += r.w * phi;
  ax += r.w * A0;
  ay += r.w * A1;
  az += r.w * A2;
}

template <int BC, int NQ>
__global__ __launch_bounds__(WG) void k_eval64(DevTree T, EwaldP E, const int64_t *__restrict__ off,
                                               const double4 *__restrict__ rec,
                                               double *__restrict__ phi, double *__restrict__ acc,
                                               double negG, const int32_t *__restrict__ blist) {
  __shared__ double4 tile[WG];
  const int64_t g = NQ == 2 ? (int64_t)blockIdx.x : (int64_t)(blockIdx.x >> 1);
  const int part = NQ == 2 ? 0 : (int)(blockIdx.x & 1);
  const int64_t b = blist ? (int64_t)blist[g] : g;
  const int tid = threadIdx.x;
  const int64_t ncell = T.nb * 512;
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const int64_t c0 = 8 * (int64_t)T.bcoord[3 * b], c1 = 8 * (int64_t)T.bcoord[3 * b + 1];
  const int64_t c2 = 8 * (int64_t)T.bcoord[3 * b + 2];
  double cx[NQ], cy[NQ], cz[NQ], sp[NQ], ax[NQ], ay[NQ], az[NQ];
  for (int q = 0; q < NQ; ++q) {
    int ci = tid + (q + part) * WG;
    sp[q] = ax[q] = ay[q] = az[q] = 0.0;
    cx[q] = centre_coord(T.org[0], c0 + (ci & 7), h);
    cy[q] = centre_coord(T.org[1], c1 + ((ci >> 3) & 7), h);
    cz[q] = centre_coord(T.org[2], c2 + (ci >> 6), h);
  }
  const int64_t start = off[b], n = off[b + 1] - start;
  for (int64_t t0 = 0; t0 < n; t0 += WG) {
    if (t0 + tid < n) tile[tid] = rec[start + t0 + tid];
    __syncthreads();
    const int m = (int)(n - t0 < WG ? n - t0 : WG);
    for (int j = 0; j < m; ++j) {
      const double4 r = tile[j];
#pragma unroll
      for (int q = 0; q < NQ; ++q) pair64<BC>(E, cx[q], cy[q], cz[q], r, sp[q], ax[q], ay[q], az[q]);
    }
    __syncthreads();
  }
  for (int q = 0; q < NQ; ++q) {
    int64_t o = b * 512 + tid + (q + part) * WG;
    phi[o] = negG * sp[q];
    acc[o] = negG * ax[q];
    acc[ncell + o] = negG * ay[q];
    acc[2 * ncell + o] = negG * az[q];
  }
}

// Target points (Sec. 2.1, the walk for an arbitrary target point): one wave
// per point, its lanes take every 64th entry of the point's list with the FP64
// pair kernel, then a butterfly adds the 64 partial sums.  A cell whose centre
// is the point gives d = 0 and is skipped, as in the cell walks.
template <int BC>
__global__ __launch_bounds__(WG) void k_eval_points64(EwaldP E, int64_t n, const double *__restrict__ xyz,
                                                      const int64_t *__restrict__ off,
                                                      const double4 *__restrict__ rec, double *__restrict__ phi,
                                                      double *__restrict__ acc, double negG) {
  const int64_t i = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;  // the whole wave
  const double cx = xyz[3 * i], cy = xyz[3 * i + 1], cz = xyz[3 * i + 2];
  double sp = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
  const int64_t e = off[i + 1];
  for (int64_t j = off[i] + lane; j < e; j += 64) pair64<BC>(E, cx, cy, cz, rec[j], sp, ax, ay, az);
  for (int m = 32; m > 0; m >>= 1) {
    sp += __shfl_xor(sp, m);
    ax += __shfl_xor(ax, m);
    ay += __shfl_xor(ay, m);
    az += __shfl_xor(az, m);
  }
  if (lane == 0) {
    phi[i] = negG * sp;
    acc[i] = negG * ax;
    acc[n + i] = negG * ay;
    acc[2 * n + i] = negG * az;
  }
}

// ---------------------------------------------------------------- FP32
struct Acc32 {
  float s, c;  // Kahan sum of M phi and its compensation
  float ax, ay, az;
  float tx, ty, tz;  // acceleration of the current tile (blocked summation)
};

template <int BC>
__device__ inline void pair32(const EwaldP &E, float cx, float cy, float cz, const float4 r,
                              Acc32 &a) {
  float dx = cx - r.x, dy = cy - r.y, dz = cz - r.z;
  if (BC != 0) {
    // minimum image by the FP32 reciprocal: where rounding picks the other
    // image of a pair at |d| = L/2, the Newtonian part and the correction
    // below both refer to it, and their sum is periodic
    const float Lx = (float)E.L[0], Ly = (float)E.L[1];
    dx = dx - Lx * floorf(fmaf(dx, E.rcp_Lf[0], 0.5f));
    if (BC != 3) dy = dy - Ly * floorf(fmaf(dy, E.rcp_Lf[1], 0.5f));
    if (BC == 1) {
      const float Lz = (float)E.L[2];
      dz = dz - Lz * floorf(fmaf(dz, E.rcp_Lf[2], 0.5f));
    }
  }
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float inv = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
  const float mi = r.w * inv;
  float term, fx, fy, fz;
  if (BC == 0) {
    const float mi3 = mi * inv * inv;
    term = mi;
    fx = mi3 * dx;
    fy = mi3 * dy;
    fz = mi3 * dz;
  } else {
    const float inv3 = inv * inv * inv;
    float phi, A0, A1, A2;
    if (BC == 2 && fabsf(dz) > (float)E.zfar) {
      phi = (float)E.far_phi_a * fabsf(dz) + (float)E.far_phi_b;
      A0 = 0.0f;
      A1 = 0.0f;
      A2 = dz < 0 ? -(float)E.far_az : (float)E.far_az;
    } else if (BC == 3 && dy * dy + dz * dz > (float)(E.zfar * E.zfar)) {
      const float rho2 = dy * dy + dz * dz, fa = (float)E.far_az / rho2;
      phi = (float)E.far_phi_a * logf(rho2) + (float)E.far_phi_b;
      A0 = 0.0f;
      A1 = fa * dy;
      A2 = fa * dz;
    } else {
      const float u0 = fabsf(dx), u1 = fabsf(dy), u2 = fabsf(dz);
      int g0 = min((int)(u0 * (float)E.inv_step[0] + 0.5f), E.n - 1);
      int g1 = min((int)(u1 * (float)E.inv_step[1] + 0.5f), E.n - 1);
      int g2 = min((int)(u2 * (float)E.inv_step[2] + 0.5f), E.n - 1);
      const float d0 = u0 - g0 * (float)E.step[0];
      const float d1 = u1 - g1 * (float)E.step[1];
      const float d2 = u2 - g2 * (float)E.step[2];
      const float4 *p = E.tab32 + 3 * (((int64_t)g2 * E.n + g1) * E.n + g0);
      const float4 q0 = p[0], q1 = p[1], q2 = p[2];
      // q0 = {phi_c, A_c}, q1 = {Hxx, Hyy, Hzz, Hxy}, q2 = {Hxz, Hyz, -, -}
      const float phic = q0.x - (q0.y * d0 + q0.z * d1 + q0.w * d2);
      const float a0 = q0.y - (q1.x * d0 + q1.w * d1 + q2.x * d2);
      const float a1 = q0.z - (q1.w * d0 + q1.y * d1 + q2.y * d2);
      const float a2 = q0.w - (q2.x * d0 + q2.y * d1 + q1.z * d2);
      phi = inv + phic;
      A0 = dx * inv3 + (dx < 0 ? -a0 : a0);
      A1 = dy * inv3 + (dy < 0 ? -a1 : a1);
      A2 = dz * inv3 + (dz < 0 ? -a2 : a2);
    }
    const bool self = !(r2 > 0.0f);
    term = self ? 0.0f : r.w * phi;
    fx = self ? 0.0f : r.w * A0;
    fy = self ? 0.0f : r.w * A1;
    fz = self ? 0.0f : r.w * A2;
  }
  // Kahan compensated sum of the potential terms
  const float y = term - a.c;
  const float t = a.s + y;
  a.c = (t - a.s) - y;
  a.s = t;
  a.tx += fx;
  a.ty += fy;
  a.tz += fz;
}

template <int BC, int NQ>
__global__ __launch_bounds__(WG) void k_eval32(DevTree T, EwaldP E, const int64_t *__restrict__ off,
                                               const double4 *__restrict__ rec, const int32_t *__restrict__ ids,
                                               float *__restrict__ phi, float *__restrict__ acc,
                                               float negG, const int32_t *__restrict__ blist) {
  __shared__ float4 tile[WG];
  const int64_t g = NQ == 2 ? (int64_t)blockIdx.x : (int64_t)(blockIdx.x >> 1);
  const int part = NQ == 2 ? 0 : (int)(blockIdx.x & 1);
  const int64_t b = blist ? (int64_t)blist[g] : g;
  const int tid = threadIdx.x;
  const int64_t ncell = T.nb * 512;
  const double sb = size_at(T.root_size, T.blev[b]);
  const double h = sb / 8.0;
  double cT[3];
  for (int k = 0; k < 3; ++k) cT[k] = centre_coord(T.org[k], T.bcoord[3 * b + k], sb);
  const int64_t own0 = T.na + 72 * T.nb + 512 * b;  // id of cell 0 of this block
  float cx[NQ], cy[NQ], cz[NQ];
  Acc32 a[NQ];
  for (int q = 0; q < NQ; ++q) {
    int ci = tid + (q + part) * WG;
    cx[q] = (float)(((double)(ci & 7) - 3.5) * h);
    cy[q] = (float)(((double)((ci >> 3) & 7) - 3.5) * h);
    cz[q] = (float)(((double)(ci >> 6) - 3.5) * h);
    a[q] = Acc32{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  }
  const int64_t start = off[b], n = off[b + 1] - start;
  for (int64_t t0 = 0; t0 < n; t0 += WG) {
    if (t0 + tid < n) {
      const double4 r = rec[start + t0 + tid];
      const int64_t own = (int64_t)ids[start + t0 + tid] - own0;
      float4 v;
      if (own >= 0 && own < 512) {
        // a cell of this block: the same offset expression as the threads' own
        v.x = (float)(((double)(own & 7) - 3.5) * h);
        v.y = (float)(((double)((own >> 3) & 7) - 3.5) * h);
        v.z = (float)(((double)(own >> 6) - 3.5) * h);
      } else {
        v.x = (float)wrap_axis(r.x - cT[0], T.L[0], T.inv_L[0], T.per[0]);
        v.y = (float)wrap_axis(r.y - cT[1], T.L[1], T.inv_L[1], T.per[1]);
        v.z = (float)wrap_axis(r.z - cT[2], T.L[2], T.inv_L[2], T.per[2]);
      }
      v.w = (float)r.w;
      tile[tid] = v;
    }
    __syncthreads();
    const int m = (int)(n - t0 < WG ? n - t0 : WG);
    for (int j = 0; j < m; ++j) {
      const float4 r = tile[j];
#pragma unroll
      for (int q = 0; q < NQ; ++q) pair32<BC>(E, cx[q], cy[q], cz[q], r, a[q]);
    }
    // blocked summation of the acceleration: tile sums into the totals
    for (int q = 0; q < NQ; ++q) {
      a[q].ax += a[q].tx;
      a[q].ay += a[q].ty;
      a[q].az += a[q].tz;
      a[q].tx = a[q].ty = a[q].tz = 0.f;
    }
    __syncthreads();
  }
  for (int q = 0; q < NQ; ++q) {
    int64_t o = b * 512 + tid + (q + part) * WG;
    phi[o] = negG * (a[q].s - a[q].c);
    acc[o] = negG * a[q].ax;
    acc[ncell + o] = negG * a[q].ay;
    acc[2 * ncell + o] = negG * a[q].az;
  }
}

// max |a|^2 over cells (non-negative doubles order like their bit patterns)
__global__ __launch_bounds__(256) void k_amax(const double *__restrict__ acc, int64_t n,
                                              unsigned long long *__restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double x = acc[i], y = acc[n + i], z = acc[2 * n + i];
    double v = x * x + y * y + z * z;
    m = v > m ? v : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

}  // namespace

hipError_t launch_eval64(const DevTree &T, const EwaldP &E, const int64_t *off, const double4 *rec,
                         double *phi, double *acc, double G, hipStream_t st, const int32_t *blist,
                         int64_t nblist) {
  if (blist && nblist <= 0) return hipSuccess;
  const int64_t nwg = blist ? nblist : T.nb;
  const bool split = nwg < FEW_BLOCKS;
  dim3 grid((unsigned)(split ? 2 * nwg : nwg)), blk(WG);
#define OT_E64(B, Q) hipLaunchKernelGGL((k_eval64<B, Q>), grid, blk, 0, st, T, E, off, rec, phi, acc, -G, blist)
  switch (E.bctype) {
    case 0: if (split) OT_E64(0, 1); else OT_E64(0, 2); break;
    case 1: if (split) OT_E64(1, 1); else OT_E64(1, 2); break;
    case 2: if (split) OT_E64(2, 1); else OT_E64(2, 2); break;
    default: if (split) OT_E64(3, 1); else OT_E64(3, 2); break;
  }
#undef OT_E64
  return hipGetLastError();
}

hipError_t launch_eval_points64(const EwaldP &E, int64_t n, const double *xyz, const int64_t *off,
                                const double4 *rec, double *phi, double *acc, double G, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + WG / 64 - 1) / (WG / 64))), blk(WG);
#define OT_EP(B) hipLaunchKernelGGL((k_eval_points64<B>), grid, blk, 0, st, E, n, xyz, off, rec, phi, acc, -G)
  switch (E.bctype) {
    case 0: OT_EP(0); break;
    case 1: OT_EP(1); break;
    case 2: OT_EP(2); break;
    default: OT_EP(3); break;
  }
#undef OT_EP
  return hipGetLastError();
}

// Adaptive block update (Sec. 2.2.6): the eight corner cells (i, j, k in
// {0, 7}) of every leaf block, walked in FP64 over the block's list; one
// workgroup per block, thread t takes corner t % 8 and every 32nd list entry
// from t / 8, and the 32 slices are added in a fixed order (a butterfly in
// each wave, then the four waves in sequence).  flags[b] = 1 when at one
// corner |a_new - a_prev| >= tol.  flags must be zero on entry.
template <int BC, typename Real>
__global__ __launch_bounds__(256) void k_abu_corners(DevTree T, EwaldP E, const int64_t *__restrict__ off,
                                                     const double4 *__restrict__ rec,
                                                     const Real *__restrict__ prev_acc, double negG, double tol,
                                                     int32_t *__restrict__ flags) {
  __shared__ double red[4][3][8];
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, k = tid & 7, sl = tid >> 3;
  const int ci = 7 * (k & 1) + 56 * ((k >> 1) & 1) + 448 * ((k >> 2) & 1);
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const double cx = centre_coord(T.org[0], 8 * (int64_t)T.bcoord[3 * b] + (ci & 7), h);
  const double cy = centre_coord(T.org[1], 8 * (int64_t)T.bcoord[3 * b + 1] + ((ci >> 3) & 7), h);
  const double cz = centre_coord(T.org[2], 8 * (int64_t)T.bcoord[3 * b + 2] + (ci >> 6), h);
  double sp = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
  for (int64_t j = off[b] + sl; j < off[b + 1]; j += 32) pair64<BC>(E, cx, cy, cz, rec[j], sp, ax, ay, az);
  for (int m = 32; m >= 8; m >>= 1) {
    ax += __shfl_xor(ax, m);
    ay += __shfl_xor(ay, m);
    az += __shfl_xor(az, m);
  }
  const int w = tid >> 6;
  if ((tid & 63) < 8) {
    red[w][0][k] = ax;
    red[w][1][k] = ay;
    red[w][2][k] = az;
  }
  __syncthreads();
  if (tid >= 8) return;
  double v[3];
  for (int c = 0; c < 3; ++c) v[c] = ((red[0][c][k] + red[1][c][k]) + red[2][c][k]) + red[3][c][k];
  const int64_t ncell = T.nb * 512, o = b * 512 + ci;
  const double dx = negG * v[0] - (double)prev_acc[o], dy = negG * v[1] - (double)prev_acc[ncell + o];
  const double dz = negG * v[2] - (double)prev_acc[2 * ncell + o];
  if (!(sqrt(dx * dx + dy * dy + dz * dz) < tol)) flags[b] = 1;
}

hipError_t launch_abu_corners(bool fp64, const DevTree &T, const EwaldP &E, const int64_t *off,
                              const double4 *rec, const void *prev_acc, double G, double tol, int32_t *flags,
                              hipStream_t st) {
  dim3 grid((unsigned)T.nb), blk(256);
#define OT_ABU(B, R) \
  hipLaunchKernelGGL((k_abu_corners<B, R>), grid, blk, 0, st, T, E, off, rec, (const R *)prev_acc, -G, tol, flags)
  if (fp64) {
    switch (E.bctype) {
      case 0: OT_ABU(0, double); break;
      case 1: OT_ABU(1, double); break;
      case 2: OT_ABU(2, double); break;
      default: OT_ABU(3, double); break;
    }
  } else {
    switch (E.bctype) {
      case 0: OT_ABU(0, float); break;
      case 1: OT_ABU(1, float); break;
      case 2: OT_ABU(2, float); break;
      default: OT_ABU(3, float); break;
    }
  }
#undef OT_ABU
  return hipGetLastError();
}

hipError_t launch_eval32(const DevTree &T, const EwaldP &E, const int64_t *off, const double4 *rec,
                         const int32_t *ids, float *phi, float *acc, double G, hipStream_t st,
                         const int32_t *blist, int64_t nblist) {
  if (blist && nblist <= 0) return hipSuccess;
  const int64_t nwg = blist ? nblist : T.nb;
  const bool split = nwg < FEW_BLOCKS;
  dim3 grid((unsigned)(split ? 2 * nwg : nwg)), blk(WG);
  float ng = (float)(-G);
#define OT_E32(B, Q) \
  hipLaunchKernelGGL((k_eval32<B, Q>), grid, blk, 0, st, T, E, off, rec, ids, phi, acc, ng, blist)
  switch (E.bctype) {
    case 0: if (split) OT_E32(0, 1); else OT_E32(0, 2); break;
    case 1: if (split) OT_E32(1, 1); else OT_E32(1, 2); break;
    case 2: if (split) OT_E32(2, 1); else OT_E32(2, 2); break;
    default: if (split) OT_E32(3, 1); else OT_E32(3, 2); break;
  }
#undef OT_E32
  return hipGetLastError();
}

hipError_t launch_amax(const double *acc, int64_t n, unsigned long long *out, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_amax, dim3((unsigned)blocks), dim3(256), 0, st, acc, n, out);
  return hipGetLastError();
}

}  // namespace ot
