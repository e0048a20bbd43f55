/* Internal declarations of the FP64 oracle (test infrastructure only). */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H
#include "octoracle.h"

enum { OR_KIND_AMR = 0, OR_KIND_P1 = 1, OR_KIND_P2 = 2, OR_KIND_CELL = 3 };
enum { OR_BC_ISO = 0, OR_BC_3P = 1, OR_BC_2P1I = 2, OR_BC_1P2I = 3 };

/* 1P2I: beyond this distance from the periodic axis (in units of Lx) the
 * analytic line-mass limit replaces the series and the table */
#define OR_1P2I_RFAR 4.0

/* Ewald set-up for periodic (3P) and mixed (2P1I, 1P2I) boundaries, Sec. 2.2.3-2.2.5 */
typedef struct {
  int bctype;
  double Lx, b, c;      /* box: Lx, Ly = b Lx, Lz = c Lx                    */
  double alpha, zeta;   /* alpha (2/Lx by default), zeta = pi^2/(alpha Lx)^2 */
  int rcut2, fcut2;     /* real-space and Fourier cut-offs (squared radii)   */
  int n;                /* table points per axis                            */
  double ext[3];        /* folded table extent per axis                     */
  double step[3];       /* ext / (n - 1)                                    */
  double *tab;          /* [n][n][n][10]: phi_c, A_c (3), H_c (xx,yy,zz,xy,xz,yz) */
} or_ewald;

/* radius of the sphere with the volume of a unit cube, (3 / (4 pi))^(1/3) */
#define OR_REQ 0.6203504908994001

/* node-ray intersection table, compressed rows: entry e = (itheta * nphi +
 * iphi) * npsi + ipsi owns pixels pix[off[e] .. off[e+1]) with weights w */
typedef struct {
  int nside, npix, ntheta, nphi, npsi, nr, nazi;
  double psimax, dtheta, dphi, dpsi;
  int64_t nentries;
  int64_t *off;
  int32_t *pix;
  double *w;
} or_raytable;

struct or_tree {
  or_params p;
  int bctype;
  double box[3];
  int64_t nb;
  int32_t lmax;
  int32_t *blev, *bcoord;
  int64_t na;
  int32_t *alev, *acoord;
  uint64_t *akey;
  int64_t *aleaf, *achild;
  int64_t nroots;
  int64_t *roots;
  int64_t nn;
  const double *rho; /* only during construction */
  double *M, *S, *com;
  double *B2, *B3; /* MPE moments of the na + 72 nb non-cell nodes (MPE MAC only) */
  or_ewald ew;
  or_raytable rt;
};

uint64_t or_morton(uint64_t x, uint64_t y, uint64_t z);
double or_size_at(const or_tree *t, int lev);
double or_wrap(const or_tree *t, int k, double d);
int or_node_geom(const or_tree *t, int64_t id, double *size, double gc[3]);
int or_children(const or_tree *t, int64_t id, int64_t ch[8]);
int64_t or_id_p1(const or_tree *t, int64_t lb, int o1);
int64_t or_id_p2(const or_tree *t, int64_t lb, int o1, int o2);
int64_t or_id_cell(const or_tree *t, int64_t lb, int ci);
int or_accept(const or_tree *t, int64_t id, const double cT[3], double ext);
void or_block_target(const or_tree *t, int64_t lb, double cT[3], double *ext);
/* walk target so of leaf block lb: the block (so < 0) or its octant so */
void or_group_target(const or_tree *t, int64_t lb, int so, double cT[3], double *ext);
/* interaction list of walk target so of leaf block lb (ids, walk order) */
int64_t or_group_list(const or_tree *t, int64_t lb, int so, int64_t *out, int64_t cap);
/* octant of a block's cell ci = i + 8 j + 64 k: bit a set on the upper half
 * of axis a */
static inline int or_cell_octant(int ci) {
  return ((ci & 7) >> 2) | ((((ci >> 3) & 7) >> 2) << 1) | ((ci >> 8) << 2);
}
void or_cell_centre(const or_tree *t, int64_t lb, int ci, double x[3]);

/* Ewald */
int or_ewald_setup(or_ewald *e, int bctype, const double box[3], double alpha, int rcut2,
                   int fcut2, int n, int with_table);
void or_ewald_release(or_ewald *e);
/* full kernel phi, A (and Hessian if H != NULL); with correction != 0 the
 * Newtonian 1/r part is removed: phi_c = phi - 1/r, A_c = A - d/r^3 */
void or_ewald_series(const or_ewald *e, const double d[3], int correction, double *phi,
                     double A[3], double H[6]);
void or_ewald_total(const or_tree *t, const double d[3], double *phi, double A[3]);

/* columns */
int64_t or_vec2pix_nest(int64_t nside, double x, double y, double z);
void or_pix2ang_nest(int64_t nside, int64_t p, double *z, double *phi);
int or_raytable_build(or_raytable *T, int nside, int ntheta, int nphi, int npsi, int nr,
                      int nazi, double psimax);
void or_raytable_free(or_raytable *T);
int64_t or_raytable_entry(const or_raytable *T, const double v[3], double d, double h);
#endif
