// Kernel launchers (internal to libocttree).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "common.hpp"

namespace ot {

// MAC suite parameters (Sec. 2.1, 2.2.1).  theta2 = theta*theta and
// half_eta = 0.5*eta_SB are formed on the host in FP64.
struct MacP {
  double theta2;
  double half_eta;
  double G;
  double a_lim;
  double tpix2;
  int mac;      // 0 BH, 1 APE, 2 MPE
  int use_pix;  // also require BH at theta_pix
};

// Ewald look-up description passed to the evaluation kernels.
struct EwaldP {
  int bctype;            // 0 iso, 1 3P, 2 2P1I, 3 1P2I
  int n;                 // table points per axis
  double L[3];           // box
  double inv_L[3];       // exact_inverse(L)
  float rcp_Lf[3];       // 1 / L rounded to FP32 (the FP32 walks' wrap)
  double step[3];        // table spacing per axis
  double inv_step[3];
  double zfar;           // 2P1I: |dz|, 1P2I: sqrt(dy^2 + dz^2) beyond which the analytic limit is used
  double far_phi_a;      // 2P1I: phi -> far_phi_a |dz| + far_phi_b; 1P2I: far_phi_a ln(rho^2) + far_phi_b,
                         // A -> far_az (0, dy, dz) / rho^2
  double far_phi_b;
  double far_az;         // A_z -> far_az sign(dz)
  const double *tab64;   // [n^3][10]
  const float4 *tab32;   // [n^3][3] (12 floats: 10 used)
};

// Node-ray intersection table description (Sec. 2.3).
struct RayTableP {
  int nside, npix, ntheta, nphi, npsi, nr, nazi;
  int64_t nentries;
  double dtheta, dphi, dpsi;
};

// Column walk parameters: binning, table rows, map normalisation.
struct ColP {
  int npix, ntheta, nphi, npsi;
  double dtheta, dphi, dpsi;
  double req;       // (3 / (4 pi))^(1/3): equal-volume sphere radius per unit edge
  double omega;     // 4 pi / N_pix
  double kappa;     // opacity of tau_avg
  double max_dist2; // columns only from nodes closer than max_dist (squared)
  int ip_pi;        // phi bin of phi = pi (offsets on the negative x axis)
  int nthr;         // threshold count: ntheta + 1 + npsi + 1 + 2 (nphi/2 + 1)
  int estimate;     // bins from look-up estimates checked at two thresholds,
                    // else binary searches (look-up tables too large)
  float lut_th, lut_ps, lut_ph;  // look-up scales: cell of cos theta, sin psi, pseudo-angle
  const double *thr;       // c|c| (c = cos(k dtheta)), sin^2(k dpsi), cos(k dphi), sin(k dphi)
  const uint8_t *lut;      // [LUT_BYTES] estimated bins (theta, psi, phi tables)
  const uint32_t *rows;    // [nentries + nlat] offset << 6 | count
  const uint4 *rows8;      // [nentries + nlat][2]: four pixels (bit 31 of the first:
                           // more than four, whose count (first) and offset (next
                           // three) are in bits 23 and up), their four FP32 weights
                           // (zero past count)
  const double *quad_w64;  // [nentries + nlat][4]: the four weights in FP64 (FP64 walk)
  int lat0;                // row lat0 + (k W + j) W + i (W = 2 lat_r + 1): copy of the
                           // row of a cell at lattice offset (i, j, k) - lat_r (node
                           // size 1); the origin's has no pixels
  int lat_r;               // half-width of the lattice table; 0: not used (grid not dyadic)
  const uint16_t *pix;     // [npairs] FP64 walk
  const double *w64;       // [npairs]
  const uint32_t *ent;     // [npairs] FP32 walk: pixel << 24 | unorm24 weight
};

// Direction-bin look-up tables of the column walk (one byte per cell, in this
// order): cos theta over [-1, 1], sin psi over [0, 1], the pseudo-angle
// t = x / (|x| + y) of the upper half-plane over [-1, 1]; each holds its
// count of cells plus one.
constexpr int LUT_TH = 512, LUT_PS = 96, LUT_PH = 80, LUT_BYTES = LUT_TH + LUT_PS + LUT_PH;

hipError_t launch_raytable(const RayTableP &P, double *dense, int32_t *cnt, int64_t *off, uint16_t *pix,
                           double *w64, int64_t *total, hipStream_t st);
hipError_t launch_raytable_pack(const RayTableP &P, const int64_t *off, const uint16_t *pix, const double *w,
                                uint32_t *rows, uint32_t *ent, uint4 *rows8, double *quad_w64, hipStream_t st);
size_t cols_smem_bytes(int npix, int cpw, bool fp64, int nthr);
// cells per workgroup with the maps in LDS: 256 or 128 when their LDS fits in
// 64 KB, else 0 (the maps are then accumulated in npix, 256 cells per group)
int cols_lds_cpw(int npix, bool fp64, int nthr);
// no_gravity (FP32, 3P / 2P1I): the columns only, phi and acc untouched (the
// walk with the learned correction computes them)
// table rows of offsets d [n][3] (cell - node) of nodes of size h [n]; -1 for d = 0
hipError_t launch_column_bins(const ColP &C, int64_t n, const double *d, const double *h, int32_t *row,
                              hipStream_t st);
// cpw: cols_lds_cpw (0: maps in npix);
// wg_per_cu (may be null): workgroups of the launched kernel resident per CU;
// blist (optional): evaluate only the nblist leaf blocks listed there
hipError_t launch_eval_cols(bool fp64, const DevTree &T, const EwaldP &E, const ColP &C, const int64_t *off,
                            const double4 *rec, const int32_t *ids, const double *lh, void *phi, void *acc,
                            void *npix, void *tau, double G, int cpw, bool no_gravity, int *wg_per_cu,
                            hipStream_t st, const int32_t *blist = nullptr, int64_t nblist = 0);
// Adaptive block update with columns: flags[b] = 1 where at one of the
// block's eight corner cells (FP64 maps over the block's list) kappa N_p of a
// pixel moved from prev_npix (FP64 or FP32 as fp64) by tol_tau or more
hipError_t launch_abu_corner_cols(bool fp64, const DevTree &T, const EwaldP &E, const ColP &C, const int64_t *off,
                                  const double4 *rec, const double *lh, const void *prev_npix, double tol_tau,
                                  int32_t *flags, hipStream_t st);

// FP32 walk with the surrogate's gravity and columns with the maps in npix
// (one workgroup of 512 cells per block; groups and Taylor step as
// launch_eval_mlp); 3P and 2P1I.  llat [list entries]: scratch for the
// entries' lattice rows.  sub: the lists are per 4^3 block octant (8 nb of
// them, list b of block b / 8 and octant b % 8); needs cell groups of 2^3 or
// more cells at h_max
hipError_t launch_eval_cols_mlp(const DevTree &T, const EwaldP &E, const ColP &C, const void *pk, const int64_t *off,
                                const double4 *rec, const int32_t *ids, const double *lh, int32_t *llat, float *phi,
                                float *acc, float *npix, float *tau, double G, double tmax, double h_max,
                                int *wg_per_cu, hipStream_t st, int sub = 0);
// rows of the offsets (i, j, k) cell sizes between two cells of one size,
// |i|, |j|, |k| <= R (k slowest, i fastest), written at rows C.lat0 + ... of
// rows, rows8 and quad_w64: copies of the table rows that the walk's binning
// gives them (an empty row at the origin)
hipError_t launch_lattice_rows(const ColP &C, int R, uint32_t *rows, uint4 *rows8, double *quad_w64,
                               hipStream_t st);

// MPE moments of every non-cell node (after launch_build): pairs p of (amr
// node pnode[p], leaf block pblock[p]) grouped by node, poff [na + 1]; part
// [npairs] scratch for the per-block partials
hipError_t launch_mpe(const DevTree &T, int64_t npairs, const int32_t *pnode, const int32_t *pblock,
                      const int64_t *poff, double2 *part, hipStream_t st);
hipError_t launch_build(const DevTree &T, const double *rho, int *bad,
                        const std::vector<int64_t> &level_begin, int lmax, hipStream_t st);

// target points: first[w] (w < grid) = the smallest index of a point of
// xyz [n][3] (device, FP64) outside [box.lo, box.hi) on some axis or not a
// number, among those of workgroup w (grid-strided), n if none
struct Box3 {
  double lo[3], hi[3];
};
hipError_t launch_points_check(const double *xyz, int64_t n, const Box3 &box, int grid, int64_t *first,
                               hipStream_t st);

// count pass (fill false): count [nb] list lengths and, when nodes is not
// null, nodes [2 nb] = (opened nodes, cells in the list) per block.  With
// pts [npts][3] (device, FP64) the lists are those of the target points
// instead, counts and offsets per point; with sub set (and no pts) those of
// the 4^3 octants of the blocks, list b of block b / 8 and octant b % 8 (bit a
// set for the upper half of axis a).
hipError_t launch_lists(bool fill, const DevTree &T, const MacP &P, int grid, int32_t *count, int32_t *nodes,
                        const int64_t *off, double4 *rec, int32_t *ids, double *lh, int32_t *scratch,
                        int64_t scratch_stride, int64_t capA, hipStream_t st, const double *pts = nullptr,
                        int64_t npts = 0, int sub = 0);

hipError_t launch_scan(const int32_t *count, int64_t nb, int64_t *off, hipStream_t st);

// blist (optional): evaluate only the nblist leaf blocks listed there
hipError_t launch_eval64(const DevTree &T, const EwaldP &E, const int64_t *off, const double4 *rec,
                         double *phi, double *acc, double G, hipStream_t st, const int32_t *blist = nullptr,
                         int64_t nblist = 0);
// FP64 potential and acceleration at n target points xyz [n][3] from their
// lists (off [n + 1], rec): phi [n], acc [3][n]
hipError_t launch_eval_points64(const EwaldP &E, int64_t n, const double *xyz, const int64_t *off,
                                const double4 *rec, double *phi, double *acc, double G, hipStream_t st);
hipError_t launch_eval32(const DevTree &T, const EwaldP &E, const int64_t *off, const double4 *rec,
                         const int32_t *ids, float *phi, float *acc, double G, hipStream_t st,
                         const int32_t *blist = nullptr, int64_t nblist = 0);
// adaptive block update: flags[b] = 1 for every leaf block with a corner cell
// whose FP64 acceleration differs from prev_acc (FP64 or FP32, [3][nb*512]) by
// at least tol; flags [nb] zero on entry
hipError_t launch_abu_corners(bool fp64, const DevTree &T, const EwaldP &E, const int64_t *off,
                              const double4 *rec, const void *prev_acc, double G, double tol, int32_t *flags,
                              hipStream_t st);

hipError_t launch_amax(const double *acc, int64_t n, unsigned long long *out, hipStream_t st);

hipError_t launch_ewald_table(const EwaldP &E, double alpha, int rcut2, int fcut2, double *tab64,
                              float4 *tab32, hipStream_t st);
// the FP32 copy of an FP64 table [n^3][10]
hipError_t launch_ewald_pack32(const EwaldP &E, const double *tab64, float4 *tab32, hipStream_t st);
// FP64 series at arbitrary offsets d [n][3] (folded to |d| inside): out [n][10]
hipError_t launch_ewald_points(const EwaldP &E, double alpha, int rcut2, int fcut2, int64_t n, const double *u,
                               double *out, hipStream_t st);

// ---------------------------------------------------------------- surrogate
// Network 3 -> 64 -> 64 -> 64 -> 10 over the folded offset: the correction's
// ten channels of the Ewald table, phi_c, A_c (3) and the second derivatives
// of phi_c (xx, yy, zz, xy, xz, yz); parameter layout
// W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[10][64] b4[10].
namespace mlpdef {
constexpr int H = 64, NI = 3, NO = 10;
constexpr int OW1 = 0, OB1 = OW1 + H * NI, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * H,
              OW4 = OB3 + H, OB4 = OW4 + NO * H, NP = OB4 + NO;
// packed matrix-core operands, 8 halves per lane each (see k_mlp.hip)
constexpr int PK_L1 = 0, PK_L2 = 2, PK_L2B = 10, PK_L3 = 12, PK_L3B = 20, PK_L4 = 22, PK_L4B = 26, NPK = 27;
}  // namespace mlpdef

// Input / output scaling: x = 2 u / ext - 1, y = (out - mu) / sig.
struct MlpNorm {
  double ext[3];
  double mu[mlpdef::NO];
  double sig[mlpdef::NO];
};

hipError_t launch_mlp_init(uint64_t seed, float *P, hipStream_t st);
hipError_t launch_mlp_points(uint64_t seed, int64_t n, const double ext[3], double *u, hipStream_t st);
hipError_t launch_mlp_prepare(int64_t n, const double *u, const double *ser, const MlpNorm &N, float *x, float *t,
                              hipStream_t st);
// gradient of the batch MSE at P over samples [s0, s0 + batch) (wrapping at n)
// of x [n][3], t [n][4]: partial [mlp_partials(batch)][NP] and lossp
// [mlp_partials(batch)] scratch, grad [NP], loss (FP32 sum) into *loss
int64_t mlp_partials(int64_t batch);
// largest batch of the allocation-free gradient (its fixed workspace holds
// the partials of that many samples)
constexpr int64_t MLP_NOALLOC_MAX_BATCH = 1024;
// device addresses, for the given device (made current by the first call on
// it), of the fixed workspace: partial [MLP_NOALLOC_MAX_BATCH / 8][NP] and
// lossp [MLP_NOALLOC_MAX_BATCH / 8]
hipError_t mlp_noalloc_workspace(int device, float **partial, float **lossp);
hipError_t launch_mlp_grad(const float *P, int64_t n, int64_t s0, int64_t batch, const float *X, const float *T,
                           float *partial, float *lossp, float *grad, float *loss, hipStream_t st);
// one Adam step (step >= 1, step size lr) on the same batch gradient
hipError_t launch_mlp_step(float *P, int64_t n, int64_t s0, int64_t batch, const float *X, const float *T,
                           float *partial, float *lossp, float *loss, float *m, float *v, float lr, int step,
                           hipStream_t st);
// pack (P, N) into the matrix-core operands used by inference
hipError_t launch_mlp_pack(const float *P, const MlpNorm &N, void *pk, hipStream_t st);
// correction (phi_c, A_c, H_c) at offsets d [n][3] by the surrogate: out [n][10]
hipError_t launch_mlp_points_eval(const void *pk, const EwaldP &E, int64_t n, const double *d, double *out,
                                  hipStream_t st);
// the same offsets by the FP64 series / the FP64 table (Taylor for phi_c and
// A_c, the nearest grid point's H_c): out [n][10]
hipError_t launch_ewald_points10(int method, const EwaldP &E, double alpha, int rcut2, int fcut2, int64_t n,
                                 const double *d, double *out, hipStream_t st);
// FP32 gravity walk with the surrogate's correction (BC 3P or 2P1I): the
// network once per (group of cells, list entry), a first-order Taylor step to
// each cell of the group; groups are the largest block-tree nodes whose cells
// lie within tmax (half the Ewald table's smallest spacing) of their centre
// on every axis; h_max: the largest cell size of the grid (sizes the LDS)
hipError_t launch_eval_mlp(const DevTree &T, const EwaldP &E, const void *pk, const int64_t *off,
                           const double4 *rec, float *phi, float *acc, double G, double tmax, double h_max,
                           hipStream_t st);
size_t eval_mlp_smem(double h_max, double tmax);
// Group level of the surrogate walk for cells of size h: groups of 2^gl cells
// per axis, the largest gl in {2, 1, 0} whose cells lie within tmax of the
// group centre ((2^gl - 1) h / 2 <= tmax).  Groups per leaf block: 512 >> 3 gl.
__host__ __device__ inline int mlp_group_level(double h, double tmax) {
  if ((3.0 * h) * 0.5 <= tmax) return 2;
  if ((1.0 * h) * 0.5 <= tmax) return 1;
  return 0;
}
inline int mlp_groups(double h, double tmax) { return 512 >> (3 * mlp_group_level(h, tmax)); }

}  // namespace ot
