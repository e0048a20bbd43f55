// Interaction lists: one per leaf block (group walk), Sec. 2.1 + 2.2.1.
//
// The paper walks the tree depth-first per target cell and accepts a node
// when the MAC suite holds.  Here all 512 cells of a leaf block share one
// list: a node is accepted for the block when
//   (i)  the block's cell-centre box lies strictly outside the cuboid of edge
//        eta_SB h centred on the node (safe box), and
//   (ii) the MAC holds at the box point closest to the node's centre of mass
//        (the closest-point distance the paper uses to decide what to export
//        between processors, Sec. 2.1 figure): BH h^2 < theta^2 d^2, APE
//        G M h^2 < a_lim d^4, MPE Eq. (2) with p = 1 (the moments B_2, B_3
//        of Eq. (3)); with columns also h^2 < theta_pix^2 d^2.  The MPE
//        bound falls with d, so the closest point is its largest value.
// Cells are always accepted.  Compiled with FP contraction off so that the
// accept/open decisions reproduce exactly.
//
// Target points (pts != null): the same traversal for each point, the target
// box shrunk to the point (half-extent 0), as the paper's walk for an arbitrary
// target point (a sink particle, say); count, off and the records are then
// per point, and each workgroup is a single wave (a point's frontiers are
// small).
//
// Traversal: a persistent workgroup per target block, level-synchronous over
// the amr-tree (frontier of amr nodes in global scratch), then over the +1
// and +2 levels of opened leaf blocks.  Ballot prefix sums give every thread
// its output slot, so the list order is deterministic.  Pass 1 counts, pass 2
// writes {r_a, M} (absolute centre of mass, FP64), the node ids and sizes.
#include "common.hpp"
#include "kernels.hpp"

namespace ot {

namespace {

// threads per workgroup: 256 for a block's list; one wave for a target
// point's, whose frontiers are small
constexpr int WG = 256;
constexpr int WG_POINT = 64;

struct Target {
  double c[3];
  double ext;
  double h;  // cell size of the target block
};

__device__ inline bool accept(const DevTree &T, const MacP &P, const Target &tg, double h,
                              const double g[3], const double4 mc, const double2 bq) {
  const double half = P.half_eta * h;
  bool outside = false;
  for (int k = 0; k < 3; ++k) {
    double d = wrap_axis(tg.c[k] - g[k], T.L[k], T.inv_L[k], T.per[k]);
    if (fabs(d) - tg.ext > half) outside = true;
  }
  if (!outside) return false;
  const double com[3] = {mc.x, mc.y, mc.z};
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    double d = wrap_axis(tg.c[k] - com[k], T.L[k], T.inv_L[k], T.per[k]);
    double e = fabs(d) - tg.ext;
    if (e > 0.0) d2 = d2 + e * e;
  }
  bool ok;
  if (P.mac == 0) {
    ok = h * h < P.theta2 * d2;
  } else if (P.mac == 1) {
    ok = P.G * mc.w * h * h < P.a_lim * d2 * d2;
  } else {
    // MPE, Eq. (2) with p = 1 multiplied out: d > b_max and
    // G (3 B_2 d - 2 B_3) < a_lim d^3 (d - b_max)^2, b_max the distance from
    // the COM to the node's farthest corner
    double b2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double e = fabs(com[k] - g[k]) + 0.5 * h;
      b2 = b2 + e * e;
    }
    const double d = sqrt(d2), bmax = sqrt(b2), q = d - bmax;
    ok = d > bmax && P.G * (3.0 * bq.x * d - 2.0 * bq.y) < P.a_lim * (d2 * d) * (q * q);
  }
  if (P.use_pix) ok = ok && (h * h < P.tpix2 * d2);
  return ok;
}

// Workgroup-wide exclusive prefix of up to three 0/1 flags.
struct Scan3 {
  int pre[3];
  int tot[3];
};

template <int NW>
__device__ inline Scan3 scan3(bool f0, bool f1, bool f2, int (*swave)[NW]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  unsigned long long m[3] = {__ballot(f0), __ballot(f1), __ballot(f2)};
  Scan3 s;
  if (lane == 0)
    for (int f = 0; f < 3; ++f) swave[f][w] = __popcll(m[f]);
  __syncthreads();
  for (int f = 0; f < 3; ++f) {
    int before = 0, tot = 0;
    for (int q = 0; q < NW; ++q) {
      int v = swave[f][q];
      before += q < w ? v : 0;
      tot += v;
    }
    s.pre[f] = before + __popcll(m[f] & lt);
    s.tot[f] = tot;
  }
  __syncthreads();
  return s;
}

template <bool FILL>
__device__ inline void emit(const DevTree &T, const Target &tg, int64_t pos, int32_t id,
                            const double4 mc, double h, double4 *rec, int32_t *ids, double *lh) {
  if (!FILL) return;
  if (lh) lh[pos] = h;
  rec[pos] = mc;
  ids[pos] = id;
}

// Count pass (FILL false): count[b] = list length of block b and, with
// nodes != null, nodes[2 b] = nodes the MAC suite opened, nodes[2 b + 1] =
// cells in the list (children of opened +2 nodes).
template <bool FILL, int WGS>
__global__ __launch_bounds__(WGS) void k_lists(DevTree T, MacP P, int32_t *__restrict__ count,
                                              int32_t *__restrict__ nodes, const int64_t *__restrict__ off,
                                              double4 *__restrict__ rec, int32_t *__restrict__ ids,
                                              double *__restrict__ lh,
                                              int32_t *__restrict__ scratch, int64_t stride,
                                              int64_t capA, const double *__restrict__ pts, int64_t npts,
                                              int sub) {
  constexpr int NW = WGS / 64;
  __shared__ int swave[3][NW];
  const int tid = threadIdx.x;
  int32_t *fa = scratch + (int64_t)blockIdx.x * stride;
  int32_t *fb = fa + capA;
  int32_t *olb = fb + capA;
  int32_t *op1 = olb + T.nb;
  const int64_t na = T.na, nb = T.nb;

  const int64_t ntg = pts ? npts : (sub ? 8 * nb : nb);
  for (int64_t b = blockIdx.x; b < ntg; b += gridDim.x) {
    Target tg;
    if (pts) {
      for (int k = 0; k < 3; ++k) tg.c[k] = pts[3 * b + k];
      tg.ext = 0.0;
      tg.h = 0.0;
    } else if (sub) {
      // octant b & 7 of block b >> 3: the box of its 4^3 cell centres
      const int64_t bb = b >> 3;
      const int o = (int)(b & 7);
      const double sb = size_at(T.root_size, T.blev[bb]);
      for (int k = 0; k < 3; ++k)
        tg.c[k] = centre_coord(T.org[k], 2 * (int64_t)T.bcoord[3 * bb + k] + ((o >> k) & 1), 0.5 * sb);
      tg.ext = 1.5 * (sb / 8.0);
      tg.h = sb / 8.0;
    } else {
      const int blev = T.blev[b];
      const double sb = size_at(T.root_size, blev);
      for (int k = 0; k < 3; ++k) tg.c[k] = centre_coord(T.org[k], T.bcoord[3 * b + k], sb);
      tg.ext = 3.5 * (sb / 8.0);
      tg.h = sb / 8.0;
    }
    const int64_t base = FILL ? off[b] : 0;
    int64_t nemit = 0, nopened = 0, ncells = 0;

    // ---- amr-tree levels
    int32_t *cur = fa, *nxt = fb;
    for (int i = tid; i < T.nroots; i += WGS) cur[i] = i;
    __syncthreads();
    int64_t ncur = T.nroots, nolb = 0;
    while (ncur > 0) {
      int64_t nnext = 0;
      for (int64_t s0 = 0; s0 < ncur; s0 += WGS) {
        int64_t i = s0 + tid;
        bool acc = false, oi = false, ol = false;
        int32_t node = -1;
        double4 mc = make_double4(0, 0, 0, 0);
        double s = 0.0;
        if (i < ncur) {
          node = cur[i];
          const int lev = T.alev[node];
          s = size_at(T.root_size, lev);
          double g[3];
          for (int k = 0; k < 3; ++k) g[k] = centre_coord(T.org[k], T.acoord[3 * node + k], s);
          mc = T.amc[node];
          acc = accept(T, P, tg, s, g, mc, P.mac == 2 ? T.abq[node] : make_double2(0.0, 0.0));
          if (!acc) {
            if (T.aleaf[node] >= 0) ol = true; else oi = true;
          }
        }
        Scan3 sc = scan3(acc, oi, ol, swave);
        if (acc) emit<FILL>(T, tg, base + nemit + sc.pre[0], node, mc, s, rec, ids, lh);
        if (oi) {
          int32_t c0 = T.achild0[node];
          for (int o = 0; o < 8; ++o) nxt[nnext + 8 * sc.pre[1] + o] = c0 + o;
        }
        if (ol) olb[nolb + sc.pre[2]] = T.aleaf[node];
        nemit += sc.tot[0];
        nnext += 8 * sc.tot[1];
        nolb += sc.tot[2];
        nopened += sc.tot[1] + sc.tot[2];
      }
      __syncthreads();
      int32_t *t = cur;
      cur = nxt;
      nxt = t;
      ncur = nnext;
    }
    __syncthreads();

    // ---- +1 nodes of opened leaf blocks
    int64_t nop1 = 0;
    for (int64_t s0 = 0; s0 < 8 * nolb; s0 += WGS) {
      int64_t i = s0 + tid;
      bool acc = false, op = false;
      int32_t lb = 0, o1 = 0;
      double4 mc = make_double4(0, 0, 0, 0);
      double s = 0.0;
      if (i < 8 * nolb) {
        lb = olb[i >> 3];
        o1 = (int)(i & 7);
        s = size_at(T.root_size, T.blev[lb]) / 2.0;
        double g[3];
        for (int k = 0; k < 3; ++k) {
          g[k] = centre_coord(T.org[k], 2 * (int64_t)T.bcoord[3 * lb + k] + ((o1 >> k) & 1), s);
        }
        mc = T.btmc[(int64_t)lb * 72 + o1];
        acc = accept(T, P, tg, s, g, mc, P.mac == 2 ? T.bbq[(int64_t)lb * 72 + o1] : make_double2(0.0, 0.0));
        op = !acc;
      }
      Scan3 sc = scan3(acc, op, false, swave);
      if (acc)
        emit<FILL>(T, tg, base + nemit + sc.pre[0], (int32_t)(na + 8 * (int64_t)lb + o1), mc, s, rec, ids, lh);
      if (op) op1[nop1 + sc.pre[1]] = lb * 8 + o1;
      nemit += sc.tot[0];
      nop1 += sc.tot[1];
      nopened += sc.tot[1];
    }
    __syncthreads();

    // ---- +2 nodes of opened +1 nodes; an opened +2 node emits its 8 cells
    for (int64_t s0 = 0; s0 < 8 * nop1; s0 += WGS) {
      int64_t i = s0 + tid;
      bool acc = false, op = false;
      int32_t lb = 0, o1 = 0, o2 = 0;
      double4 mc = make_double4(0, 0, 0, 0);
      double s = 0.0;
      if (i < 8 * nop1) {
        int32_t v = op1[i >> 3];
        lb = v >> 3;
        o1 = v & 7;
        o2 = (int)(i & 7);
        s = size_at(T.root_size, T.blev[lb]) / 4.0;
        double g[3];
        for (int k = 0; k < 3; ++k) {
          int64_t pos = 4 * (int64_t)T.bcoord[3 * lb + k] + 2 * ((o1 >> k) & 1) + ((o2 >> k) & 1);
          g[k] = centre_coord(T.org[k], pos, s);
        }
        mc = T.btmc[(int64_t)lb * 72 + 8 + 8 * o1 + o2];
        acc = accept(T, P, tg, s, g, mc,
                     P.mac == 2 ? T.bbq[(int64_t)lb * 72 + 8 + 8 * o1 + o2] : make_double2(0.0, 0.0));
        op = !acc;
      }
      Scan3 sc = scan3(acc, op, false, swave);
      if (acc)
        emit<FILL>(T, tg, base + nemit + sc.pre[0],
                   (int32_t)(na + 8 * nb + 64 * (int64_t)lb + 8 * o1 + o2), mc, s, rec, ids, lh);
      if (op && FILL) {
        const int lev = T.blev[lb];
        const double h = size_at(T.root_size, lev) / 8.0;
        int64_t p0 = base + nemit + sc.tot[0] + 8 * (int64_t)sc.pre[1];
        for (int o3 = 0; o3 < 8; ++o3) {
          int ci = cell_index(o1, o2, o3);
          int ijk[3] = {ci & 7, (ci >> 3) & 7, ci >> 6};
          double4 r;
          r.x = centre_coord(T.org[0], 8 * (int64_t)T.bcoord[3 * lb + 0] + ijk[0], h);
          r.y = centre_coord(T.org[1], 8 * (int64_t)T.bcoord[3 * lb + 1] + ijk[1], h);
          r.z = centre_coord(T.org[2], 8 * (int64_t)T.bcoord[3 * lb + 2] + ijk[2], h);
          r.w = T.cm[(int64_t)lb * 512 + ci];
          rec[p0 + o3] = r;
          ids[p0 + o3] = (int32_t)(na + 72 * nb + 512 * (int64_t)lb + ci);
          if (lh) lh[p0 + o3] = h;
        }
      }
      nemit += sc.tot[0] + 8 * sc.tot[1];
      nopened += sc.tot[1];
      ncells += 8 * sc.tot[1];
    }
    if (!FILL && tid == 0) {
      count[b] = (int32_t)nemit;
      if (nodes) {
        nodes[2 * b] = (int32_t)nopened;
        nodes[2 * b + 1] = (int32_t)ncells;
      }
    }
    __syncthreads();
  }
}

// Exclusive scan of the per-block counts (single workgroup, sequential tiles).
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ count, int64_t nb,
                                               int64_t *__restrict__ off) {
  __shared__ int64_t part[1024];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t s0 = 0; s0 < nb; s0 += 1024) {
    int64_t i = s0 + tid;
    int64_t v = i < nb ? count[i] : 0;
    part[tid] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      int64_t add = tid >= d ? part[tid - d] : 0;
      __syncthreads();
      part[tid] += add;
      __syncthreads();
    }
    if (i < nb) off[i] = carry + part[tid] - v;
    __syncthreads();
    if (tid == 1023) carry += part[1023];
    __syncthreads();
  }
  if (tid == 0) off[nb] = carry;
}

// Index of the first target point outside [lo, hi) on some axis (a NaN
// coordinate fails every comparison), or n when all lie inside: workgroup w
// writes the smallest such index of its grid-strided points to first[w].
__global__ __launch_bounds__(256) void k_points_check(const double *__restrict__ xyz, int64_t n, Box3 box,
                                                      int64_t *__restrict__ first) {
  __shared__ int64_t wmin[4];
  int64_t m = n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    bool in = true;
    for (int k = 0; k < 3; ++k) {
      const double x = xyz[3 * i + k];
      in = in && x >= box.lo[k] && x < box.hi[k];
    }
    if (!in && i < m) m = i;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const int64_t o = __shfl_xor(m, d);
    m = o < m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t r = wmin[0];
    for (int w = 1; w < 4; ++w) r = wmin[w] < r ? wmin[w] : r;
    first[blockIdx.x] = r;
  }
}

}  // namespace

hipError_t launch_points_check(const double *xyz, int64_t n, const Box3 &box, int grid, int64_t *first,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_points_check, dim3(grid), dim3(256), 0, st, xyz, n, box, first);
  return hipGetLastError();
}

hipError_t launch_lists(bool fill, const DevTree &T, const MacP &P, int grid, int32_t *count, int32_t *nodes,
                        const int64_t *off, double4 *rec, int32_t *ids, double *lh, int32_t *scratch,
                        int64_t stride, int64_t capA, hipStream_t st, const double *pts, int64_t npts,
                        int sub) {
#define OT_LISTS(F, W)                                                                                  \
  hipLaunchKernelGGL((k_lists<F, W>), dim3(grid), dim3(W), 0, st, T, P, count, nodes, off, rec, ids, lh, scratch, \
                     stride, capA, pts, npts, sub)
  if (pts) {
    if (fill) OT_LISTS(true, WG_POINT);
    else OT_LISTS(false, WG_POINT);
  } else {
    if (fill) OT_LISTS(true, WG);
    else OT_LISTS(false, WG);
  }
#undef OT_LISTS
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t *count, int64_t nb, int64_t *off, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, count, nb, off);
  return hipGetLastError();
}

}  // namespace ot
