// Device-side tree description and geometry helpers shared by the kernels.
//
// Node numbering (global ids): amr nodes [0, na) in (level, Morton) order;
// then for each leaf block lb its 8 "+1" nodes (na + 8 lb + o1), its 64 "+2"
// nodes (na + 8 nb + 64 lb + 8 o1 + o2) and its 512 cells
// (na + 72 nb + 512 lb + i + 8 j + 64 k).  Octant o has bit 0 = x, bit 1 = y,
// bit 2 = z.  Sec. 2: a leaf block's block-tree has levels l_lb+1 (8 nodes),
// l_lb+2 (64) and l_lb+3 (512 cells).
//
// Geometry is evaluated with the same IEEE operations in the same order
// wherever an integer decision depends on it (MAC accept/open), so that the
// interaction lists are reproducible exactly; files that take such decisions
// are compiled with FP contraction off.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ot {

struct DevTree {
  const int32_t *alev;    // [na]
  const int32_t *acoord;  // [na*3]
  const int32_t *achild0; // [na] first child (children contiguous, octant order) or -1
  const int32_t *aleaf;   // [na] leaf block id or -1
  const int32_t *blev;    // [nb]
  const int32_t *bcoord;  // [nb*3]
  const int32_t *bamr;    // [nb] amr index of each leaf block
  double4 *amc;           // [na] {com.x, com.y, com.z, M}
  double4 *aS;            // [na] {S.x, S.y, S.z, 0}: sum of m x (build only)
  double4 *btmc;          // [nb*72] +1 nodes (8) then +2 nodes (64)
  double *cm;             // [nb*512] cell masses
  double2 *abq;           // [na] MPE moments {B_2, B_3} (MPE MAC only, else null)
  double2 *bbq;           // [nb*72] the same for the +1 and +2 nodes
  int64_t na, nb;
  int32_t nroots;
  int32_t per[3];         // periodic axis flags
  double root_size;
  double org[3];
  double L[3];            // domain edge per axis
  double inv_L[3];        // exact_inverse(L)
};

__host__ __device__ inline double size_at(double root_size, int lev) {
  return root_size / (double)(1LL << (lev - 1));
}

// Centre of the cell / node at integer position pos (in units of size) along
// one axis: org + (pos + 1/2) size.  Every kernel and the host use this one
// expression without FMA contraction, so a cell centre computed in two places
// is the same double (the target cell then gives d = 0 exactly).
__host__ __device__ inline double centre_coord(double org, int64_t pos, double size) {
#pragma clang fp contract(off)
  return org + ((double)pos + 0.5) * size;
}

// minimum image in a periodic axis, wrapped to [-L/2, L/2): d - L floor(d / L
// + 1/2).  inv_L = 1 / L when L is a power of two (then d inv_L is d / L
// exactly), else 0 and the quotient is a division.
__device__ inline double wrap_axis(double d, double L, double inv_L, int per) {
  if (!per) return d;
  const double q = inv_L != 0.0 ? d * inv_L : d / L;
  return d - L * floor(q + 0.5);
}

// 1 / L if that is exact (L a power of two), else 0
__host__ inline double exact_inverse(double L) {
  int e = 0;
  return L > 0.0 && frexp(L, &e) == 0.5 ? 1.0 / L : 0.0;
}

__device__ inline int cell_index(int o1, int o2, int o3) {
  int i = 4 * (o1 & 1) + 2 * (o2 & 1) + (o3 & 1);
  int j = 4 * ((o1 >> 1) & 1) + 2 * ((o2 >> 1) & 1) + ((o3 >> 1) & 1);
  int k = 4 * ((o1 >> 2) & 1) + 2 * ((o2 >> 2) & 1) + ((o3 >> 2) & 1);
  return i + 8 * j + 64 * k;
}

}  // namespace ot
