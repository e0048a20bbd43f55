/*
 * octtree.h - C ABI of libocttree, a GPU (MI355X / gfx950) implementation of
 * the tree solver of Wuensch, Walch, Dinnbier & Whitworth (2018), "Tree-based
 * solvers for adaptive mesh refinement code FLASH - I: gravity and optical
 * depths".
 *
 * Problem statement (Sec. 2 and Sec. 2.2-2.3): density is given on the leaf
 * blocks of a block-structured AMR grid (blocks of 8^3 cells, organised as an
 * octree of blocks, the "amr-tree"); the solver returns, for every cell, the
 * gravitational potential and acceleration summed over monopole tree nodes
 * (Eqs. 7-8, with the Ewald forms of Sec. 2.2.2-2.2.3 for periodic or mixed
 * boundaries) and, optionally, the column density in each HEALPix direction
 * (Sec. 2.3).
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers owned by the caller; the
 *     library never frees them.  Pointers named *_host are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their work on it and return after synchronising it, so results are ready
 *     when a call returns OT_OK.
 *   - Cell layout: cell (i, j, k) of leaf block b is element b*512 + i + 8 j
 *     + 64 k (x fastest); vector fields are structure-of-arrays, component c at
 *     c*nb*512 + b*512 + cell.
 *   - Every call returns an ot_status; no exception crosses the ABI.  On an
 *     error the outputs are untouched (validation errors) or undefined (device
 *     errors), and ot_last_error() describes it.
 *   - One host thread at a time per context.
 */
#ifndef OCTTREE_H
#define OCTTREE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ot_ctx ot_ctx;

typedef enum {
  OT_OK = 0,
  OT_ERR_INVALID_ARG = -1, /* bad pointer, size or parameter value           */
  OT_ERR_BAD_GRID = -2,    /* leaf blocks do not tile the domain exactly     */
  OT_ERR_NUMERIC = -3,     /* negative or non-finite density                 */
  OT_ERR_STATE = -4,       /* call out of order (e.g. solve before build)    */
  OT_ERR_OOM = -5,         /* device allocation failed or over the limit     */
  OT_ERR_DEVICE = -6,      /* HIP runtime error                              */
  OT_ERR_UNSUPPORTED = -7  /* valid request this build does not implement   */
} ot_status;

typedef enum { OT_BC_ISOLATED = 0, OT_BC_PERIODIC = 1 } ot_bc;
typedef enum { OT_MAC_BH = 0, OT_MAC_APE = 1 } ot_mac;
typedef enum { OT_EWALD_TABLE = 0, OT_EWALD_EXACT = 1 } ot_ewald;

/* Solver parameters; defaults (ot_params_default) follow App. B where the
 * paper gives one. */
typedef struct {
  int32_t nroot[3];      /* root blocks per axis (a forest, Sec. 2)            [1,1,1] */
  int32_t bc[3];         /* per-axis boundary, App. B grav_boundary_type_*     [iso]   */
                         /* supported: all isolated, all periodic (3P), and
                            x, y periodic with z isolated (2P1I, Sec. 2.2.3)           */
  double root_size;      /* edge of a cubic root block                          [1.0]  */
  double origin[3];      /* domain corner                                       [0,0,0]*/
  double G;              /* gravitational constant, App. B grv_bhNewton         [1.0]  */
  double theta_lim;      /* BH opening angle, Eq. (1), gr_bhTreeLimAngle        [0.5]  */
  double eta_sb;         /* safe-box factor, Sec. 2.1, gr_bhTreeSafeBox         [1.2]  */
  int32_t mac;           /* ot_mac; APE uses Eq. (6) with p = 1, Eq. (4)        [BH]   */
  int32_t ewald;         /* ot_ewald: correction from the table (Sec. 2.2.4,
                            second approach) or the exact series per pair      [TABLE] */
  double a_lim;          /* APE absolute limit, Eq. (4); <= 0: a_lim = eps_lim *
                            a_max from a BH (theta_lim) FP64 pass, Sec. 3      [0]    */
  double eps_lim;        /* relative device of Sec. 3 for a_lim                 [1e-3] */
  int32_t ewald_n;       /* table points per axis (grv_bhEwaldNPer)             [64]   */
  int32_t ewald_rcut2;   /* real-space cut-off |i|^2, Eq. (10); <=0: 15 (3P), 10 (2P1I) */
  int32_t ewald_fcut2;   /* Fourier cut-off |l|^2, Eq. (10); <= 0: 10                  */
  int32_t device;        /* HIP device ordinal                                  [0]    */
  double ewald_alpha;    /* Ewald splitting constant; <= 0: 2 / Lx (Sec. 2.2.2) [0]    */
  uint64_t max_device_bytes; /* cap on library allocations; 0 = none           [0]    */
  /* column densities (OpticalDepth module, Sec. 2.3; App. B tr_* parameters) */
  int32_t nside;         /* HEALPix Nside of the per-cell maps: 1, 2 or 4
                            (N_pix = 12 Nside^2: 12, 48, 192); 0 = no columns  [0]    */
  int32_t il_ntheta;     /* node-ray table: theta bins (tr_ilNTheta)            [25]   */
  int32_t il_nphi;       /*                 phi bins (tr_ilNPhi)                [50]   */
  int32_t il_npsi;       /*                 angular-size bins (tr_ilNNS)        [25]   */
  int32_t il_nr;         /*                 disc sample radii (tr_ilNR)         [50]   */
  int32_t il_nazi;       /*                 disc sample azimuths                [100]  */
  double theta_pix;      /* with columns a node must also pass BH at this angle
                            (Sec. 2.3: theta_lim ~ sqrt(Omega_pix)); <= 0: 1/Nside [0] */
  double kappa;          /* opacity in tau_avg = -ln <exp(-kappa N_p)>_p       [1]    */
  double max_dist;       /* columns only from nodes closer (tr_bhMaxDist)       [1e99] */
  double psi_max;        /* upper edge of the angular-size bins (rad)          [0.98] */
} ot_params;

/* Run statistics of the last solve. */
typedef struct {
  int64_t n_interactions;  /* sum over cells of accepted list entries (N_int) */
  int64_t max_list;        /* longest block interaction list                 */
  int64_t total_list;      /* sum of block list lengths                      */
  double a_lim_used;       /* APE limit actually used (0 for BH)             */
  double ms_build;         /* tree build (moments), device time              */
  double ms_list;          /* interaction-list construction, device time      */
  double ms_eval;          /* per-cell evaluation, device time               */
} ot_stats;

void ot_params_default(ot_params *p);

/* Create a context bound to p->device.  No device work until ot_build. */
ot_status ot_create(const ot_params *p, ot_ctx **out);

/* Leaf-block layout (Sec. 2): level[b] >= 1 (root = 1) and the integer block
 * position coord[3*b + k] at that level, 0 <= coord < nroot[k] * 2^(level-1).
 * Host arrays, copied.  Validates that the blocks tile the domain exactly
 * (no overlap, no hole; OT_ERR_BAD_GRID) and builds the amr-tree topology on
 * the host: amr nodes ordered by (level, Morton key of the finest-level
 * integer corner, x in bit 0), children in octant order (bit 0 = x). */
ot_status ot_set_blocks(ot_ctx *c, int64_t nb, const int32_t *level_host,
                        const int32_t *coord_host);

/* Tree build, Sec. 2.1: cell masses m = rho h^3 and, bottom-up, each node's
 * mass and centre of mass in FP64 (children summed in octant order; leaf
 * COM = cell centre).  rho_dev: [nb*512] FP64 device array, finite, >= 0
 * (OT_ERR_NUMERIC otherwise, checked on the device). */
ot_status ot_build(ot_ctx *c, const double *rho_dev, void *stream);

/* Tree walk, Sec. 2.1 + 2.2 + 2.3: one interaction list per leaf block (all
 * its cells share it; a node is accepted when the safe box and the MAC hold
 * at the block's closest cell centre, and with columns also BH at
 * theta_pix), then per cell
 *   Phi = -G sum M phi(d),  a = -G sum M A(d),  d = r - r_a,
 * phi = 1/|d| (isolated) or the Ewald kernel (periodic / mixed), and with
 * nside > 0 the column map N_p = sum w_p M / (Omega_pix |d|^2) over the
 * node-ray table's pixels w_p of each node and tau_avg = -ln <exp(-kappa N_p)>.
 * ot_solve: FP32 arithmetic with compensated (Kahan) summation of Phi;
 * ot_solve64: FP64 throughout.  Direction bins are decided in FP64 in both.
 * phi_dev [nb*512], acc_dev [3*nb*512]; npix_dev [nb][N_pix][512] and
 * tau_dev [nb*512] are required when nside > 0 and ignored otherwise.
 * stats_host may be NULL. */
ot_status ot_solve(ot_ctx *c, float *phi_dev, float *acc_dev, float *npix_dev, float *tau_dev,
                   ot_stats *stats_host, void *stream);
ot_status ot_solve64(ot_ctx *c, double *phi_dev, double *acc_dev, double *npix_dev,
                     double *tau_dev, ot_stats *stats_host, void *stream);

/* Ewald correction table, Sec. 2.2.4 (second approach): phi_c = phi - 1/r,
 * A_c = A - d/r^3 and the six second derivatives of phi_c, FP64, on a
 * uniform n^3 grid over the folded domain [0, Lx/2] x [0, Ly/2] x
 * [0, Lz/2] (3P) or [0, min(Lz, 2 Lx)] in z (2P1I).  Built on the device by
 * the first solve that needs it; this call builds it eagerly.  Only for
 * periodic or mixed boundaries (OT_ERR_STATE otherwise). */
ot_status ot_ewald_prepare(ot_ctx *c, void *stream);

/* ---- inspection (tests, tools) ---- */
/* Number of amr nodes (all blocks, leaf or not) after ot_set_blocks. */
int64_t ot_num_amr_nodes(const ot_ctx *c);
/* amr-tree topology as built on the host: level [na], coord [na*3], leaf
 * block index or -1 [na], children [na*8] (-1 for leaf blocks), Morton
 * keys [na].  Any pointer may be NULL. */
ot_status ot_export_topology(const ot_ctx *c, int32_t *level_host, int32_t *coord_host,
                             int64_t *leaf_host, int64_t *child_host, uint64_t *key_host);
/* Node moments after ot_build, by global node id: amr nodes [0, na), then the
 * 8 +1 nodes of each leaf block, the 64 +2 nodes, the 512 cells.
 * M_host [nn], com_host [nn*3] with nn = na + 584 nb. */
ot_status ot_export_moments(ot_ctx *c, double *M_host, double *com_host);
/* Interaction list of leaf block b from the last solve (global node ids). */
ot_status ot_export_list(ot_ctx *c, int64_t b, int32_t *ids_host, int64_t cap, int64_t *len);
/* Ewald table (n^3 x 10 doubles, x fastest; channels phi_c, A_c[3],
 * H_xx, H_yy, H_zz, H_xy, H_xz, H_yz) after ot_ewald_prepare. */
ot_status ot_export_ewald_table(ot_ctx *c, double *tab_host);
/* Node-ray intersection table (Sec. 2.3), built on the device on first use:
 * entry e = (itheta * nphi + iphi) * npsi + ipsi owns pixels
 * pix[off[e] .. off[e+1]) (ascending) with weights w summing to 1.  Call with
 * NULL arrays to get the sizes: *nentries and *npairs. */
ot_status ot_export_raytable(ot_ctx *c, int64_t *nentries, int64_t *npairs, int64_t *off_host,
                             int32_t *pix_host, double *w_host, void *stream);

const char *ot_last_error(const ot_ctx *c); /* owned by ctx; valid until the next call */
void ot_destroy(ot_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
