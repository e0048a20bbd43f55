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
 * (Eqs. 7-8, with the Ewald forms of Sec. 2.2.3-2.2.4 for periodic or mixed
 * boundaries) and, optionally, the column density in each HEALPix direction
 * (Sec. 2.3).  The same tree can be walked for arbitrary target points
 * (Sec. 2.1; ot_solve_points).
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers owned by the caller; the
 *     library never frees them.  Pointers named *_host are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their work on it and return after synchronising it, so results are ready
 *     when a call returns OT_OK (ot_mlp_grad_noalloc alone only enqueues).
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
  OT_ERR_UNSUPPORTED = -7, /* valid request this build does not implement   */
  OT_ERR_IO = -8           /* a cache file cannot be read or written         */
} ot_status;

typedef enum { OT_BC_ISOLATED = 0, OT_BC_PERIODIC = 1 } ot_bc;
typedef enum { OT_MAC_BH = 0, OT_MAC_APE = 1, OT_MAC_MPE = 2 } ot_mac;
/* TABLE: FP64-generated table with the Taylor term (Sec. 2.2.5, second
 * approach); EXACT: the FP64 series itself (point evaluation only); MLP: the
 * learned surrogate once ot_mlp_train (or ot_mlp_set) has accepted it, else
 * the table. */
typedef enum { OT_EWALD_TABLE = 0, OT_EWALD_EXACT = 1, OT_EWALD_MLP = 2 } ot_ewald;

/* Solver parameters; defaults (ot_params_default) follow App. B where the
 * paper gives one. */
typedef struct {
  int32_t nroot[3];      /* root blocks per axis (a forest, Sec. 2)            [1,1,1] */
  int32_t bc[3];         /* per-axis boundary, App. B grav_boundary_type_*     [iso]   */
                         /* supported: all isolated, all periodic (3P), x, y
                            periodic with z isolated (2P1I, Sec. 2.2.4; needs
                            Ly <= Lx, else OT_ERR_UNSUPPORTED), and x periodic
                            with y, z isolated (1P2I, Sec. 2.2.4)                      */
  double root_size;      /* edge of a cubic root block                          [1.0]  */
  double origin[3];      /* domain corner                                       [0,0,0]*/
  double G;              /* gravitational constant, App. B grv_bhNewton         [1.0]  */
  double theta_lim;      /* BH opening angle, Eq. (1), gr_bhTreeLimAngle        [0.5]  */
  double eta_sb;         /* safe-box factor, Sec. 2.1, gr_bhTreeSafeBox         [1.2]  */
  int32_t mac;           /* ot_mac; APE uses Eq. (6) with p = 1, Eq. (4); MPE uses    */
                         /* Eq. (2) with p = 1 (B_2, B_3 of Eq. (3)), Eq. (4)  [BH]   */
  int32_t ewald;         /* ot_ewald: correction in the walk: TABLE or MLP (the
                            FP32 walks, with or without columns; the FP64 walks
                            use the table); EXACT is rejected by the walk     [TABLE] */
  double a_lim;          /* APE/MPE absolute limit, Eq. (4); <= 0: a_lim = eps_lim *
                            a_max from a BH (theta_lim) FP64 pass, Sec. 3      [0]    */
  double eps_lim;        /* relative device of Sec. 3 for a_lim                 [1e-3] */
  int32_t ewald_n;       /* table points per axis (grv_bhEwaldNPer)             [64]   */
  int32_t ewald_rcut2;   /* real-space cut-off |i|^2, Eq. (10); <=0: 15 (3P), 10 (2P1I, 1P2I) */
  int32_t ewald_fcut2;   /* Fourier cut-off |l|^2, Eq. (10); <= 0: 10                  */
  int32_t device;        /* HIP device ordinal                                  [0]    */
  double ewald_alpha;    /* Ewald splitting constant; <= 0: 2 / Lx (Sec. 2.2.3) [0]    */
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
  /* learned Ewald surrogate in the walk */
  double mlp_reach;      /* the walk evaluates the network once per group of cells
                            and list entry and takes a first-order Taylor step to
                            each cell; the group is the block's 4^3, 2^3 or single
                            cells, the largest whose cells lie, per axis, within
                            mlp_reach times half the Ewald table's smallest grid
                            spacing of its centre (1: the table's own Taylor
                            offset, Sec. 2.2.5; larger: fewer evaluations and a
                            Taylor remainder growing as its square); <= 0: 1 [1] */
  int32_t list_group;    /* cells per axis of a walk target (Sec. 2.1's group walk
                            with a smaller group): 8 (or 0) one interaction list
                            per leaf block; 4 one list per 4^3 octant of a block,
                            the same MAC suite against the box of the octant's
                            cell centres (shorter lists, each still passing the
                            suite at every cell it serves).  4 is walked by the
                            FP32 solve with an accepted surrogate, Nside 4 maps
                            and cell groups of 2^3 or 4^3 cells; other solves of
                            such a context, and the adaptive update, return
                            OT_ERR_UNSUPPORTED                              [8] */
} ot_params;

/* Run statistics of the last solve. */
typedef struct {
  int64_t n_interactions;  /* sum over cells of accepted list entries (N_int) */
  int64_t max_list;        /* longest interaction list (one per block, or per
                              block octant with list_group 4)               */
  int64_t total_list;      /* sum of the list lengths                         */
  double a_lim_used;       /* APE/MPE limit actually used (0 for BH)         */
  double ms_build;         /* tree build (moments), device time              */
  double ms_list;          /* interaction-list construction, device time      */
  double ms_eval;          /* per-cell evaluation, device time               */
  int32_t ewald_used;      /* ot_ewald the evaluation used (TABLE or MLP; TABLE
                              also for isolated boundaries)                   */
  int32_t eval_wg_per_cu;  /* workgroups of the column walk resident per compute
                              unit (its occupancy); 0 without columns         */
  int64_t n_opened;        /* nodes the MAC suite opened, summed over lists   */
  int64_t n_accepted;      /* list entries that are not cells: nodes the MAC
                              suite accepted, summed over lists (ot_solve,
                              ot_solve64; 0 for the adaptive update)          */
  int64_t list_hist[32];   /* lists whose length L has 2^k <= L < 2^(k+1)     */
  int64_t n_mlp_evals;     /* network evaluations of the surrogate walk
                              (cell groups x list entries); 0 without it      */
  double ms_gravity;       /* device time of the surrogate gravity walk; 0 when
                              the column walk carries it (maps in memory)     */
  double ms_columns;       /* device time of the column walk (with the table,
                              or with the surrogate and maps in memory, it
                              computes the gravity too)                       */
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
 * COM = cell centre); with the MPE MAC also each node's B_2 and B_3 of
 * Eq. (3) about its COM (per leaf block a partial over its cells in octant
 * order, an amr node adding its blocks' partials depth first).  rho_dev:
 * [nb*512] FP64 device array, finite, >= 0 (OT_ERR_NUMERIC otherwise,
 * checked on the device). */
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

/* Adaptive block update, Sec. 2.2.6 (periodic boundaries use the Ewald
 * table; the surrogate is not used).  On entry phi_dev, acc_dev and, when
 * nside > 0, npix_dev and tau_dev hold the previous step's solution on the
 * same grid (layouts as ot_solve; npix_dev and tau_dev are ignored when
 * nside = 0).  After building the lists, the walk first evaluates the eight
 * corner cells (i, j, k in {0, 7}) of every leaf block in FP64: their
 * acceleration and, when nside > 0, their maps (the section counts the
 * optical depth among the quantities compared at the corners).  A block
 * whose corners all moved by less than tol (Euclidean norm of the
 * acceleration change, an absolute accuracy) and, with columns, whose
 * corners' optical depth kappa N_p moved by less than tol_tau in every pixel
 * (absolute; this also bounds the change of tau_avg by tol_tau) keeps all
 * its previous values; the others are evaluated in full, with their columns (FP32-Kahan,
 * or FP64 for ot_solve_abu64).  updated_host [nb] (may be NULL) receives 1
 * per evaluated block.  tol = 0 (or tol_tau = 0 with columns) evaluates
 * every block; tol_tau is ignored when nside = 0.
 * stats->n_interactions counts the pairs of the evaluated blocks.  Errors:
 * OT_ERR_INVALID_ARG (tol < 0 or not finite, npix_dev or tau_dev NULL or
 * tol_tau < 0 or not finite with nside > 0), OT_ERR_STATE (no build). */
ot_status ot_solve_abu(ot_ctx *c, float *phi_dev, float *acc_dev, float *npix_dev, float *tau_dev, double tol,
                       double tol_tau, int32_t *updated_host, ot_stats *stats_host, void *stream);
ot_status ot_solve_abu64(ot_ctx *c, double *phi_dev, double *acc_dev, double *npix_dev, double *tau_dev,
                         double tol, double tol_tau, int32_t *updated_host, ot_stats *stats_host, void *stream);

/* Gravity at arbitrary target points, Sec. 2.1 (the walk for any target
 * point, e.g. the position of a sink particle): each point gets its own list,
 * the MAC suite of ot_solve evaluated at the point itself (the safe box about
 * the node's geometric centre, BH / APE / MPE at the point's distance to the
 * node's centre of mass; cells always accepted), and the FP64 pair kernels of
 * ot_solve64 over it (Newtonian, plus the Ewald table or the far-field limit
 * for periodic and mixed boundaries; the surrogate is not used here).  A cell
 * whose centre coincides with a point is skipped, so at cell centres this is
 * the paper's per-cell walk.  APE / MPE take the limit ot_solve uses (a_lim,
 * or eps_lim times the BH pre-pass maximum).  Needs a successful ot_build.
 * xyz_dev  [n][3] FP64 device positions, each inside the domain: origin <= x <
 *          origin + nroot root_size on every axis (periodic ones too), else
 *          OT_ERR_INVALID_ARG naming the first such point (also for NaN);
 *          checked on the device before any list is built.
 * phi_dev  [n] FP64 device output; acc_dev [3][n] FP64 device output
 *          (component-major), both owned by the caller.
 * n        0 <= n <= 2^31; n = 0 returns OT_OK and touches nothing.
 * The traversal uses up to 4 GB of device scratch (kept by the context, as
 * its other buffers).
 * The lists of a successful call with n > 0 stay in the context until the
 * next ot_solve_points (which drops them first, even when it fails), ot_build
 * or ot_set_blocks (ot_export_point_list); stats: list lengths per point
 * (n_interactions = total_list = entries summed over the points). */
ot_status ot_solve_points(ot_ctx *c, int64_t n, const double *xyz_dev, double *phi_dev, double *acc_dev,
                          ot_stats *stats_host, void *stream);

/* Ewald correction table, Sec. 2.2.5 (second approach): phi_c = phi - 1/r,
 * A_c = A - d/r^3 and the six second derivatives of phi_c, FP64, on a
 * uniform n^3 grid over the folded domain [0, Lx/2] x [0, Ly/2] x
 * [0, Lz/2] (3P), [0, min(Lz, 2 Lx)] in z (2P1I), or [0, Lx/2] x
 * [0, min(Ly, 4 Lx)] x [0, min(Lz, 4 Lx)] (1P2I).  Built on the device by
 * the first solve that needs it; this call builds it eagerly.  Only for
 * periodic or mixed boundaries (OT_ERR_STATE otherwise).
 * cache_path (may be NULL; App. B grv_bhEwaldFName): a file that keeps the
 * FP64 table.  It is read when its header matches this context's table
 * (boundary type, box, alpha, cut-offs, n, domain, channel layout) and its
 * checksum holds; otherwise (missing, other inputs, truncated, corrupted)
 * the table is generated and the file rewritten (through a temporary file
 * next to it, renamed into place).  OT_ERR_IO when the file exists but
 * cannot be read, or cannot be written, before any device work. */
ot_status ot_ewald_prepare(ot_ctx *c, const char *cache_path, void *stream);

/* ---- learned Ewald surrogate --------------------------------------------
 * Not part of the paper: a network 3 -> 64 -> 64 -> 64 -> 10 (activation
 * z S(z), S the cubic smoothstep over [-3, 3]) maps the folded offset to the
 * ten channels of the Ewald table of Sec. 2.2.5 (phi_c, A_c and the six
 * second derivatives of phi_c), which stays the fallback and the judge of
 * its error.  Trained on the device in FP32 (Adam, batch MSE on standardised
 * outputs) on FP64 series values at offsets drawn uniformly from the folded
 * domain; evaluated with FP16-input / FP32-accumulate matrix instructions.
 * The FP32 walk evaluates it once per (group of cells, list entry), a group
 * being the largest block-tree node (4^3 or 2^3 cells, else a single cell)
 * whose cells lie within half the table's smallest spacing of its centre on
 * every axis, and takes the first-order Taylor step from the group's centre
 * to each cell as the table look-up does (second approach of Sec. 2.2.5). */
typedef struct {
  int64_t nsamples;  /* training offsets; multiple of 32                    [2097152] */
  int64_t nval;      /* held-out offsets for validation                     [100000]  */
  int32_t epochs;    /* passes over the training offsets                    [300]     */
  int32_t batch;     /* offsets per Adam step; multiple of 32, <= nsamples  [2048]    */
  double lr_max;     /* Adam step size, cosine decay from lr_max ...        [3e-3]    */
  double lr_min;     /* ... to lr_min over all steps                        [1e-5]    */
  uint64_t seed;     /* counter-based streams: init, training and held-out  [4]       */
  double tol;        /* accepted when the held-out error of phi_c and A_c is
                        at most tol and that of the second derivatives at
                        most 10 tol (max |error| / max |exact value|)     [5e-3]    */
} ot_mlp_config;

typedef struct {
  double loss_first;    /* mean batch loss of the first epoch (standardised)  */
  double loss_last;     /* mean batch loss of the last epoch                  */
  double err_mlp[10];   /* held-out error per channel (phi_c, A_c x, y, z, the
                           second derivatives xx, yy, zz, xy, xz, yz): max
                           |error| / max |exact value|                        */
  double err_table[10]; /* the same for this context's FP64 table (Taylor term
                           for phi_c and A_c, nearest point for the others)   */
  double ms_samples;    /* series evaluation of the training offsets          */
  double ms_train;      /* all Adam steps                                     */
  double ms_validate;   /* held-out evaluation                                */
  int32_t ok;           /* 1: accepted, the walk uses it for OT_EWALD_MLP     */
  int32_t from_cache;   /* 1: read from the cache file (times are then 0)     */
} ot_mlp_report;

#define OT_MLP_NPARAM 9226 /* W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[10][64] b4[10] */
#define OT_MLP_NOUT 10     /* outputs: phi_c, A_c[3], second derivatives xx yy zz xy xz yz */
#define OT_MLP_NNORM 23    /* ext[3] (x = 2 u / ext - 1), mu[10], sig[10] (y = (out - mu) / sig) */

void ot_mlp_config_default(ot_mlp_config *cfg);

/* Generate the training and held-out offsets, their FP64 series values, train,
 * validate against the series and the table, and accept or reject the
 * surrogate.  3P and 2P1I only (OT_ERR_STATE when isolated, OT_ERR_UNSUPPORTED
 * for 1P2I, whose walks use the table).  Synchronous; the training buffers
 * are freed before returning.  report may be NULL.
 * cache_path (may be NULL): a file that keeps the trained parameters, their
 * scaling and the report; read when its header matches (boundary type, box,
 * the table's domain and the series' alpha and cut-offs, every field of cfg,
 * the network's shape and the training recipe's version) and its checksum
 * holds, else the surrogate is trained and the file rewritten.  OT_ERR_IO as
 * for ot_ewald_prepare. */
ot_status ot_mlp_train(ot_ctx *c, const ot_mlp_config *cfg, const char *cache_path, ot_mlp_report *report,
                       void *stream);

/* Current surrogate: params_host [OT_MLP_NPARAM], norm_host [OT_MLP_NNORM]
 * (either may be NULL).  OT_ERR_STATE before training or ot_mlp_set. */
ot_status ot_mlp_get(ot_ctx *c, float *params_host, double *norm_host);

/* Install a surrogate (host arrays as in ot_mlp_get); accept != 0 lets the
 * walk use it.  sig must be > 0 and ext > 0. */
ot_status ot_mlp_set(ot_ctx *c, const float *params_host, const double *norm_host, int32_t accept,
                     void *stream);

/* Batch loss and gradient of the training objective at params_dev [NPARAM]
 * over x_dev [batch][3] (network inputs) and t_dev [batch][10] (standardised
 * targets): L = 1/(10 batch) sum (y - t)^2.  grad_dev [NPARAM]; *loss_host
 * gets L.  batch a multiple of 32.  Device pointers are the caller's. */
ot_status ot_mlp_grad(ot_ctx *c, const float *params_dev, int64_t batch, const float *x_dev,
                      const float *t_dev, float *grad_dev, float *loss_host, void *stream);

/* One training step of the surrogate, in place: the batch loss and gradient
 * at params_dev as ot_mlp_grad, then the Adam update the trainer applies
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias corrections 1 - beta^step) with
 * step size lr to params_dev [NPARAM] and its moment estimates m_dev, v_dev
 * [NPARAM].  step >= 1 is the update's index; *loss_host gets the loss at
 * the parameters before the update.  An inspection entry for tests (the
 * trainer runs the same kernels).  Errors: OT_ERR_INVALID_ARG (null pointer,
 * batch as ot_mlp_grad, step < 1, lr <= 0 or not finite). */
ot_status ot_mlp_adam_step(ot_ctx *c, float *params_dev, float *m_dev, float *v_dev, int64_t batch,
                           const float *x_dev, const float *t_dev, double lr, int64_t step, float *loss_host,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): ot_mlp_grad without any allocation.  The per-workgroup partial
 * gradients live in a fixed workspace of the library, a static device array
 * of 4.7 MB (the partials of 1024 samples) that each GPU the library runs on
 * holds until the process ends.  Arguments as ot_mlp_grad, except that the
 * loss goes to a device scalar, loss_dev [1], and that the call only enqueues
 * its kernels on stream and returns without synchronising.  batch: a
 * positive multiple of 32, at most 1024 (OT_ERR_INVALID_ARG beyond; use
 * ot_mlp_grad for larger batches).  Every call on one GPU shares that GPU's
 * workspace: calls that overlap in time on one GPU (other streams, other
 * host threads, other contexts) race and must be serialised by the caller. */
ot_status ot_mlp_grad_noalloc(ot_ctx *c, const float *params_dev, int64_t batch, const float *x_dev,
                              const float *t_dev, float *grad_dev, float *loss_dev, void *stream);

/* The correction at offsets d_dev [n][3] (any sign; folded and unfolded
 * inside) into out_dev [n][10], FP64: phi_c, A_c (3) and the second
 * derivatives of phi_c (xx, yy, zz, xy, xz, yz), by method: OT_EWALD_EXACT
 * (series), OT_EWALD_TABLE (FP64 table with the Taylor term for phi_c and
 * A_c, the nearest grid point's second derivatives) or OT_EWALD_MLP (the
 * installed surrogate, accepted or not; 3P and 2P1I only).  2P1I beyond
 * |dz| = 2 Lx and 1P2I beyond sqrt(dy^2 + dz^2) = 4 Lx (a line of mass 1/Lx:
 * phi = -(ln(alpha^2 rho^2) + gamma_E)/Lx): the analytic limit for every
 * method, minus the Newtonian 1/r and its derivatives. */
ot_status ot_ewald_points(ot_ctx *c, int32_t method, int64_t n, const double *d_dev, double *out_dev,
                          void *stream);

/* ---- inspection (tests, tools) ---- */
/* Node-ray table entry (Sec. 2.3: the (theta, phi, psi) bin of a node seen
 * from a cell) that the column walk uses for nodes of size h_dev [n] at
 * offsets d_dev [n][3] = cell centre minus node centre of mass (FP64, any
 * sign; the periodic wrap is the caller's), into row_dev [n]: entry
 * (itheta * il_nphi + iphi) * il_npsi + ipsi, or -1 for d = 0.  Runs the walk's
 * own device function (look-up estimate, FP64 threshold tests, exact
 * fallback).  Needs nside > 0; builds the node-ray table on first use.
 * Device pointers are the caller's; n <= 2^30. */
ot_status ot_column_bins(ot_ctx *c, int64_t n, const double *d_dev, const double *h_dev, int32_t *row_dev,
                         void *stream);

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
/* Interaction list b from the last solve (global node ids): that of leaf
 * block b, or with list_group 4 that of octant b % 8 of block b / 8 (bit a
 * of the octant set for the upper half of axis a), b < 8 nb. */
ot_status ot_export_list(ot_ctx *c, int64_t b, int32_t *ids_host, int64_t cap, int64_t *len);
/* node ids of target point i's list from the last ot_solve_points (as above) */
ot_status ot_export_point_list(ot_ctx *c, int64_t i, int32_t *ids_host, int64_t cap, int64_t *len);
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
