/*
 * FP64 CPU oracle for the OctTree solver of Wuensch, Walch, Dinnbier &
 * Whitworth (2018), "Tree-based solvers for adaptive mesh refinement code
 * FLASH - I".
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct C: recursion,
 * per-cell loops, no blocking or fusion.  It shares no code with the GPU
 * library and must only be called from tests, the smoke check and the
 * benchmark's CPU-baseline leg.
 */
#ifndef OCTORACLE_H
#define OCTORACLE_H
#include <stdint.h>

typedef struct {
  int32_t nroot[3];   /* root blocks per axis (forest, Sec. 2 footnote)      */
  int32_t bc[3];      /* per axis: 0 isolated, 1 periodic (Sec. 2.2.3-2.2.4) */
  double root_size;   /* edge of a cubic root block                         */
  double origin[3];
  double G;           /* gravitational constant                             */
  double theta;       /* BH opening angle theta_lim, Eq. (1)                */
  double eta_sb;      /* safe-box factor eta_SB (Sec. 2.1)                  */
  double a_lim;       /* APE absolute acceleration limit, Eqs. (4), (6)     */
  double theta_pix;   /* extra BH angle when columns are on; <= 0: off      */
  int32_t mac;        /* 0 = BH, 1 = APE, 2 = MPE                           */
  int32_t ewald;      /* 0 = exact series, 1 = table (periodic/mixed only)  */
  int32_t ew_n;       /* table points per axis                              */
  int32_t ew_rcut2;   /* real-space cut-off |i|^2 (<= 0: 15 for 3P, 10 2P1I) */
  int32_t ew_fcut2;   /* Fourier cut-off |l|^2 (<= 0: 10)                    */
  int32_t pad_;
  double ew_alpha;    /* Ewald splitting alpha (<= 0: 2 / Lx)               */
  int32_t nside;      /* HEALPix Nside of the column maps; 0 = no columns   */
  int32_t il_ntheta;  /* intersection table: theta bins                      */
  int32_t il_nphi;    /*                     phi bins                        */
  int32_t il_npsi;    /*                     angular-size bins               */
  int32_t il_nr;      /*                     disc sample radii               */
  int32_t il_nazi;    /*                     disc sample azimuths            */
  double kappa;       /* opacity in tau_avg = -ln <exp(-kappa N)>            */
  double max_dist;    /* columns only from nodes closer than this            */
  double psi_max;     /* upper edge of the psi bins                          */
  double mlp_reach;   /* surrogate walk: group cells within mlp_reach x half the
                         table's smallest spacing of the group centre (<= 0: 1) */
  int32_t list_group; /* cells per axis of a walk target: 8 (or 0) one list per
                         leaf block, 4 one list per 4^3 octant of a block  */
} or_params;

typedef struct or_tree or_tree;

/* Returns NULL on an invalid grid; *err receives a short reason code:
 * 1 bad level/coord, 2 duplicate block, 3 overlap, 4 hole, 5 bad density,
 * 6 unsupported boundary combination, 7 list_group not 0, 4 or 8. */
or_tree *or_tree_new(const or_params *p, int64_t nb, const int32_t *level,
                     const int32_t *coord, const double *rho, int *err);
void or_tree_free(or_tree *t);
/* MPE moments B_2, B_3 [na + 72 nb] (node ids below the cells); mac = 2 only */
void or_tree_mpe_export(const or_tree *t, double *B2, double *B3);
/* adaptive block update of the group walk (gravity only), Sec. 2.2.6 */
void or_walk_group_abu(const or_tree *t, const double *prev_phi, const double *prev_acc, double tol,
                       const double *prev_npix, double tol_tau, double *phi, double *acc, int32_t *updated);
/* the walk at arbitrary target points (Sec. 2.1): the list of one point, and
 * phi [n], acc [3][n] at the points xyz [n][3] */
int64_t or_point_list(const or_tree *t, const double x[3], int64_t *out, int64_t cap);
void or_walk_points(const or_tree *t, int64_t n, const double *xyz, double *phi, double *acc,
                    int64_t *nint);
int64_t or_tree_na(const or_tree *t);
int64_t or_tree_nn(const or_tree *t);
#endif
