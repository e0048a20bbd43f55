// Tree build (Sec. 2.1): node masses and centres of mass, bottom-up, FP64.
//
// Compiled with FP contraction off: every node moment is a left-to-right sum
// over the 8 children in octant order, M = sum m, S = sum m x, COM = S / M
// (geometric centre when M = 0); a cell's COM is its centre.  The results are
// therefore reproducible bit for bit.
#include "common.hpp"
#include "kernels.hpp"

namespace ot {

// One workgroup (64 lanes, one wave) per leaf block.  The 512 densities are
// staged through LDS with coalesced loads; lane t then owns the "+2" node t
// (8 cells), lanes 0..7 the "+1" nodes, lane 0 the leaf-block node.
__global__ __launch_bounds__(64) void k_block_moments(DevTree T, const double *__restrict__ rho,
                                                      int *__restrict__ bad) {
  __shared__ double sm[512];
  __shared__ double4 s2[64];
  __shared__ double4 s1[8];
  const int64_t lb = blockIdx.x;
  const int t = threadIdx.x;
  const int lev = T.blev[lb];
  const int c[3] = {T.bcoord[3 * lb], T.bcoord[3 * lb + 1], T.bcoord[3 * lb + 2]};
  const double sblk = size_at(T.root_size, lev);
  const double h = sblk / 8.0;
  const double hcube = h * h * h;
  int badv = 0;
  for (int q = t; q < 512; q += 64) {
    double r = rho[lb * 512 + q];
    if (!(r >= 0.0) || isinf(r)) badv = 1;
    double m = r * hcube;
    sm[q] = m;
    T.cm[lb * 512 + q] = m;
  }
  if (badv) *bad = 1;
  __syncthreads();

  // +2 node t = 8 o1 + o2
  {
    const int o1 = t >> 3, o2 = t & 7;
    double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
    for (int o3 = 0; o3 < 8; ++o3) {
      int ci = cell_index(o1, o2, o3);
      int ii = ci & 7, jj = (ci >> 3) & 7, kk = ci >> 6;
      double x = centre_coord(T.org[0], 8 * (int64_t)c[0] + ii, h);
      double y = centre_coord(T.org[1], 8 * (int64_t)c[1] + jj, h);
      double z = centre_coord(T.org[2], 8 * (int64_t)c[2] + kk, h);
      double m = sm[ci];
      M = M + m;
      Sx = Sx + m * x;
      Sy = Sy + m * y;
      Sz = Sz + m * z;
    }
    s2[t] = make_double4(Sx, Sy, Sz, M);
    double s = sblk / 4.0;
    double g[3];
    for (int k = 0; k < 3; ++k) {
      g[k] = centre_coord(T.org[k], 4 * (int64_t)c[k] + 2 * ((o1 >> k) & 1) + ((o2 >> k) & 1), s);
    }
    double4 mc = M > 0.0 ? make_double4(Sx / M, Sy / M, Sz / M, M) : make_double4(g[0], g[1], g[2], M);
    T.btmc[lb * 72 + 8 + t] = mc;
  }
  __syncthreads();
  if (t < 8) {
    double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
    for (int o2 = 0; o2 < 8; ++o2) {
      double4 v = s2[8 * t + o2];
      M = M + v.w;
      Sx = Sx + v.x;
      Sy = Sy + v.y;
      Sz = Sz + v.z;
    }
    s1[t] = make_double4(Sx, Sy, Sz, M);
    double s = sblk / 2.0;
    double g[3];
    for (int k = 0; k < 3; ++k) {
      g[k] = centre_coord(T.org[k], 2 * (int64_t)c[k] + ((t >> k) & 1), s);
    }
    T.btmc[lb * 72 + t] = M > 0.0 ? make_double4(Sx / M, Sy / M, Sz / M, M)
                                  : make_double4(g[0], g[1], g[2], M);
  }
  __syncthreads();
  if (t == 0) {
    double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
    for (int o1 = 0; o1 < 8; ++o1) {
      double4 v = s1[o1];
      M = M + v.w;
      Sx = Sx + v.x;
      Sy = Sy + v.y;
      Sz = Sz + v.z;
    }
    double g[3];
    for (int k = 0; k < 3; ++k) g[k] = centre_coord(T.org[k], c[k], sblk);
    int64_t a = T.bamr[lb];
    T.amc[a] = M > 0.0 ? make_double4(Sx / M, Sy / M, Sz / M, M) : make_double4(g[0], g[1], g[2], M);
    T.aS[a] = make_double4(Sx, Sy, Sz, 0.0);
  }
}

// amr-tree parents of one level: sum the 8 children (contiguous, octant order).
__global__ __launch_bounds__(256) void k_amr_moments(DevTree T, int64_t begin, int64_t end) {
  int64_t i = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= end || T.aleaf[i] >= 0) return;
  int64_t c0 = T.achild0[i];
  double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
  for (int o = 0; o < 8; ++o) {
    double4 v = T.aS[c0 + o];
    M = M + T.amc[c0 + o].w;
    Sx = Sx + v.x;
    Sy = Sy + v.y;
    Sz = Sz + v.z;
  }
  double s = size_at(T.root_size, T.alev[i]);
  double g[3];
  for (int k = 0; k < 3; ++k) g[k] = centre_coord(T.org[k], T.acoord[3 * i + k], s);
  T.amc[i] = M > 0.0 ? make_double4(Sx / M, Sy / M, Sz / M, M) : make_double4(g[0], g[1], g[2], M);
  T.aS[i] = make_double4(Sx, Sy, Sz, 0.0);
}

// MPE moments (Eqs. (2), (3)): B_2 and B_3 of a node about its own COM, the
// sums of m |r_i - r_a|^2 and m |r_i - r_a|^3 over its cells, |d|^3 =
// d^2 sqrt(d^2).  The cells of a leaf block are visited in octant order (+1,
// +2, cell) into one partial sum per (node, block); an amr node adds its
// blocks' partials in depth-first octant order.

// m |x - ra|^2 and m |x - ra|^3 of cell ci of leaf block lb, added to s
__device__ inline void mpe_cell(const DevTree &T, int64_t lb, int ci, double h, const double ra[3], double2 &s) {
  const int ijk[3] = {ci & 7, (ci >> 3) & 7, ci >> 6};
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double d = centre_coord(T.org[k], 8 * (int64_t)T.bcoord[3 * lb + k] + ijk[k], h) - ra[k];
    d2 = d2 + d * d;
  }
  const double m = T.cm[512 * lb + ci];
  s.x = s.x + m * d2;
  s.y = s.y + m * (d2 * sqrt(d2));
}

// +1 (threads 0..7) and +2 (8..71) nodes of one leaf block per workgroup
__global__ __launch_bounds__(128) void k_mpe_block(DevTree T) {
  const int64_t lb = blockIdx.x;
  const int t = threadIdx.x;
  if (t >= 72) return;
  const double h = size_at(T.root_size, T.blev[lb]) / 8.0;
  const double4 mc = T.btmc[lb * 72 + t];
  const double ra[3] = {mc.x, mc.y, mc.z};
  double2 s = make_double2(0.0, 0.0);
  if (t < 8) {
    for (int o2 = 0; o2 < 8; ++o2)
      for (int o3 = 0; o3 < 8; ++o3) mpe_cell(T, lb, cell_index(t, o2, o3), h, ra, s);
  } else {
    const int o1 = (t - 8) >> 3, o2 = (t - 8) & 7;
    for (int o3 = 0; o3 < 8; ++o3) mpe_cell(T, lb, cell_index(o1, o2, o3), h, ra, s);
  }
  T.bbq[lb * 72 + t] = s;
}

// one (amr node, leaf block under it) pair per thread: the block's partial
__global__ __launch_bounds__(256) void k_mpe_pairs(DevTree T, int64_t npairs, const int32_t *__restrict__ pnode,
                                                   const int32_t *__restrict__ pblock, double2 *__restrict__ part) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int64_t lb = pblock[p];
  const double4 mc = T.amc[pnode[p]];
  const double ra[3] = {mc.x, mc.y, mc.z};
  const double h = size_at(T.root_size, T.blev[lb]) / 8.0;
  double2 s = make_double2(0.0, 0.0);
  for (int o1 = 0; o1 < 8; ++o1)
    for (int o2 = 0; o2 < 8; ++o2)
      for (int o3 = 0; o3 < 8; ++o3) mpe_cell(T, lb, cell_index(o1, o2, o3), h, ra, s);
  part[p] = s;
}

// amr node i: its blocks' partials [poff[i], poff[i + 1]) in depth-first order
__global__ __launch_bounds__(256) void k_mpe_amr(DevTree T, const int64_t *__restrict__ poff,
                                                 const double2 *__restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T.na) return;
  double2 B = make_double2(0.0, 0.0);
  const int64_t p1 = poff[i + 1];
  int64_t p = poff[i];
  // sixteen loads in flight, then the adds in order
  for (; p + 16 <= p1; p += 16) {
    double2 v[16];
    for (int k = 0; k < 16; ++k) v[k] = part[p + k];
    for (int k = 0; k < 16; ++k) {
      B.x = B.x + v[k].x;
      B.y = B.y + v[k].y;
    }
  }
  for (; p < p1; ++p) {
    B.x = B.x + part[p].x;
    B.y = B.y + part[p].y;
  }
  T.abq[i] = B;
}

hipError_t launch_mpe(const DevTree &T, int64_t npairs, const int32_t *pnode, const int32_t *pblock,
                      const int64_t *poff, double2 *part, hipStream_t st) {
  hipLaunchKernelGGL(k_mpe_block, dim3((unsigned)T.nb), dim3(128), 0, st, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (npairs > 0) {
    hipLaunchKernelGGL(k_mpe_pairs, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, T, npairs, pnode,
                       pblock, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mpe_amr, dim3((unsigned)((T.na + 255) / 256)), dim3(256), 0, st, T, poff, part);
  return hipGetLastError();
}

hipError_t launch_build(const DevTree &T, const double *rho, int *bad,
                        const std::vector<int64_t> &level_begin, int lmax, hipStream_t st) {
  hipLaunchKernelGGL(k_block_moments, dim3((unsigned)T.nb), dim3(64), 0, st, T, rho, bad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int l = lmax - 1; l >= 1; --l) {
    int64_t b0 = level_begin[l], b1 = level_begin[l + 1];
    if (b1 <= b0) continue;
    unsigned nblk = (unsigned)((b1 - b0 + 255) / 256);
    hipLaunchKernelGGL(k_amr_moments, dim3(nblk), dim3(256), 0, st, T, b0, b1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ot
