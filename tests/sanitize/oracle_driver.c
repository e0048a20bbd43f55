/*
 * Drives every exported function of the CPU oracle on small inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (see
 * tests/test_sanitize.py).  Each result is checked for finiteness and a few
 * plain invariants; the sanitizers catch out-of-bounds accesses, leaks and
 * undefined behaviour on the way.  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/octoracle.h"

/* exported by the oracle library, declared here as the Python binding sees them */
void or_tree_export(const or_tree *t, int32_t *alev, int32_t *acoord, int64_t *aleaf, int64_t *achild,
                    uint64_t *akey, double *M, double *com);
int64_t or_block_list(const or_tree *t, int64_t lb, int64_t *out, int64_t cap);
int64_t or_group_list(const or_tree *t, int64_t lb, int so, int64_t *out, int64_t cap);
void or_walk_group(const or_tree *t, double *phi, double *acc, int64_t *nint);
void or_walk_group_blocks(const or_tree *t, int64_t nsel, const int64_t *sel, double *phi, double *acc,
                          double *npix, double *tau, int64_t *nint);
void or_walk_percell(const or_tree *t, int64_t ntg, const int64_t *tg, double *phi, double *acc, int64_t *nint);
void or_direct(const or_tree *t, int64_t ntg, const int64_t *tg, double *phi, double *acc);
void or_raymarch(const or_tree *t, const double *rho, int64_t tg, int64_t nside, int64_t nside_f, double *out);
int64_t or_healpix_vec2pix(int64_t nside, double x, double y, double z);
void or_healpix_pix2ang(int64_t nside, int64_t p, double *out);
void or_raytable_entries(int ntheta, int nphi, int npsi, double psimax, int64_t n, const double *d, const double *h,
                         int64_t *out);
int64_t or_raytable_export(int nside, int ntheta, int nphi, int npsi, int nr, int nazi, double psimax, int64_t *off,
                           int32_t *pix, double *w);
uint64_t or_morton(uint64_t x, uint64_t y, uint64_t z);
void or_ewald_eval(int bctype, const double box[3], double alpha, int rcut2, int fcut2, int correction, int64_t npts,
                   const double *d, double *out);
void or_ewald_table(int bctype, const double box[3], double alpha, int rcut2, int fcut2, int n, double *out);
void or_ewald_table_lookup(int bctype, const double box[3], int n, const double *tab, int64_t npts, const double *d,
                           double *out);
void or_itilde(double s, double zeta, double gam, double *out);
void or_kfuncs(int l, double eta, double zeta, double *out);
int or_mlp_nparam(void);
void or_mlp_forward(const double *p, int64_t B, const double *x, double *y);
double or_mlp_grad(const double *p, int64_t B, const double *x, const double *t, double *g);
void or_adam_update(double *p, const double *g, double *m, double *v, int64_t n, double lr, int64_t step);
double or_mlp_adam(double *p, double *m, double *v, int64_t B, const double *x, const double *t, double lr,
                   int64_t step);
int or_mlp_group_level(const or_tree *t, int64_t lb);
void or_walk_group_mlp(const or_tree *t, const double *params, const double *norm, int64_t nsel, const int64_t *sel,
                       double *phi, double *acc, int64_t *nint);

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static uint64_t rng_state = 12345;
static double urand(void) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int all_finite(const double *v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* nroot[0] x nroot[1] x nroot[2] roots of 2^3 level-2 blocks each; the first
 * block refined into 2^3 level-3 blocks.  Returns nb. */
static int64_t make_grid(const int32_t nroot[3], int32_t **level, int32_t **coord, double **rho) {
  const int64_t nb = 8 * (int64_t)nroot[0] * nroot[1] * nroot[2] - 1 + 8;
  *level = (int32_t *)malloc(sizeof(int32_t) * nb);
  *coord = (int32_t *)malloc(sizeof(int32_t) * 3 * nb);
  *rho = (double *)malloc(sizeof(double) * 512 * nb);
  int64_t b = 0;
  for (int z = 0; z < 2 * nroot[2]; ++z)
    for (int y = 0; y < 2 * nroot[1]; ++y)
      for (int x = 0; x < 2 * nroot[0]; ++x) {
        if (x == 0 && y == 0 && z == 0) {
          for (int o = 0; o < 8; ++o) {
            (*level)[b] = 3;
            (*coord)[3 * b] = o & 1;
            (*coord)[3 * b + 1] = (o >> 1) & 1;
            (*coord)[3 * b + 2] = o >> 2;
            ++b;
          }
          continue;
        }
        (*level)[b] = 2;
        (*coord)[3 * b] = x;
        (*coord)[3 * b + 1] = y;
        (*coord)[3 * b + 2] = z;
        ++b;
      }
  for (int64_t i = 0; i < 512 * nb; ++i) (*rho)[i] = 0.2 + urand();
  return nb;
}

static or_params base_params(const int32_t nroot[3], const int32_t bc[3]) {
  or_params p;
  memset(&p, 0, sizeof(p));
  for (int k = 0; k < 3; ++k) {
    p.nroot[k] = nroot[k];
    p.bc[k] = bc[k];
  }
  p.root_size = 1.0;
  p.G = 1.0;
  p.theta = 0.5;
  p.eta_sb = 1.2;
  p.ewald = 1;
  p.ew_n = 8;
  p.il_ntheta = 25;
  p.il_nphi = 50;
  p.il_npsi = 25;
  p.il_nr = 50;
  p.il_nazi = 100;
  p.kappa = 1.0;
  p.max_dist = 1e99;
  p.psi_max = 0.98;
  return p;
}

/* walks of one tree: group walk (all blocks), selected blocks with columns
 * when nside > 0, per-cell walk and direct sum of a few cells, lists,
 * export and the adaptive block update */
static void exercise_tree(const or_params *p, const char *name) {
  int32_t *level, *coord;
  double *rho;
  const int64_t nb = make_grid(p->nroot, &level, &coord, &rho);
  int err = 0;
  or_tree *t = or_tree_new(p, nb, level, coord, rho, &err);
  if (!t) {
    fprintf(stderr, "%s: or_tree_new failed (%d)\n", name, err);
    ++failures;
    free(level);
    free(coord);
    free(rho);
    return;
  }
  const int64_t n = 512 * nb, na = or_tree_na(t), nn = or_tree_nn(t);
  CHECK(na > 0 && nn > na);
  {
    int32_t *alev = malloc(sizeof(int32_t) * na), *acoord = malloc(sizeof(int32_t) * 3 * na);
    int64_t *aleaf = malloc(sizeof(int64_t) * na), *achild = malloc(sizeof(int64_t) * 8 * na);
    uint64_t *akey = malloc(sizeof(uint64_t) * na);
    double *M = malloc(sizeof(double) * nn), *com = malloc(sizeof(double) * 3 * nn);
    or_tree_export(t, alev, acoord, aleaf, achild, akey, M, com);
    CHECK(all_finite(M, nn) && all_finite(com, 3 * nn));
    free(alev), free(acoord), free(aleaf), free(achild), free(akey), free(M), free(com);
  }
  if (p->mac == 2) {
    const int64_t nm = na + 72 * nb;
    double *B2 = malloc(sizeof(double) * nm), *B3 = malloc(sizeof(double) * nm);
    or_tree_mpe_export(t, B2, B3);
    CHECK(all_finite(B2, nm) && all_finite(B3, nm));
    free(B2), free(B3);
  }
  for (int64_t lb = 0; lb < nb; lb += 5) {
    const int64_t len = or_block_list(t, lb, NULL, 0);
    int64_t *ids = malloc(sizeof(int64_t) * (len > 0 ? len : 1));
    CHECK(or_block_list(t, lb, ids, len) == len);
    for (int64_t q = 0; q < len; ++q) CHECK(ids[q] >= 0 && ids[q] < nn);
    free(ids);
    for (int so = 0; so < 8; so += 7) {
      const int64_t lo = or_group_list(t, lb, so, NULL, 0);
      int64_t *oi = malloc(sizeof(int64_t) * (lo > 0 ? lo : 1));
      CHECK(lo > 0 && lo <= len && or_group_list(t, lb, so, oi, lo) == lo);
      for (int64_t q = 0; q < lo; ++q) CHECK(oi[q] >= 0 && oi[q] < nn);
      free(oi);
    }
  }
  double *phi = malloc(sizeof(double) * n), *acc = malloc(sizeof(double) * 3 * n);
  int64_t *nint = malloc(sizeof(int64_t) * nb);
  or_walk_group(t, phi, acc, nint);
  CHECK(all_finite(phi, n) && all_finite(acc, 3 * n));
  const int64_t tg[4] = {0, 511, 512 * 3 + 77, n - 1};
  double ph4[4], ac4[12];
  int64_t ni4[4];
  or_walk_percell(t, 4, tg, ph4, ac4, ni4);
  CHECK(all_finite(ph4, 4) && all_finite(ac4, 12));
  or_direct(t, 4, tg, ph4, ac4);
  CHECK(all_finite(ph4, 4) && all_finite(ac4, 12));
  {
    /* arbitrary target points: the domain's lower corner, an interior point
     * and a point a little inside the upper corner */
    double xyz[9];
    for (int k = 0; k < 3; ++k) {
      const double L = p->nroot[k] * p->root_size;
      xyz[k] = p->origin[k];
      xyz[3 + k] = p->origin[k] + 0.37 * L;
      xyz[6 + k] = p->origin[k] + 0.999 * L;
    }
    const int64_t len = or_point_list(t, xyz + 3, NULL, 0);
    int64_t *ids = malloc(sizeof(int64_t) * (len > 0 ? len : 1));
    CHECK(len > 0 && or_point_list(t, xyz + 3, ids, len) == len);
    for (int64_t q = 0; q < len; ++q) CHECK(ids[q] >= 0 && ids[q] < nn);
    free(ids);
    double ph3[3], ac3[9];
    int64_t ni3[3];
    or_walk_points(t, 3, xyz, ph3, ac3, ni3);
    CHECK(all_finite(ph3, 3) && all_finite(ac3, 9) && ni3[1] == len);
  }
  const int64_t sel[2] = {1, nb - 1};
  double *sp = malloc(sizeof(double) * 1024), *sa = malloc(sizeof(double) * 3 * 1024);
  double *npix = NULL, *tau = NULL, *prev_npix = NULL;
  const int npx = 12 * p->nside * p->nside;
  if (p->nside > 0) {
    npix = malloc(sizeof(double) * 2 * npx * 512);
    tau = malloc(sizeof(double) * 1024);
  }
  or_walk_group_blocks(t, 2, sel, sp, sa, npix, tau, NULL);
  CHECK(all_finite(sp, 1024) && all_finite(sa, 3 * 1024));
  if (p->nside > 0) {
    CHECK(all_finite(npix, 2 * npx * 512) && all_finite(tau, 1024));
    double *cols = malloc(sizeof(double) * npx);
    or_raymarch(t, rho, 512 + 300, p->nside, 4 * p->nside, cols);
    CHECK(all_finite(cols, npx));
    free(cols);
    prev_npix = calloc((size_t)n * npx, sizeof(double));
  }
  /* adaptive block update: from zeros every block moves; from the walk itself none */
  double *zp = calloc(n, sizeof(double)), *za = calloc(3 * n, sizeof(double));
  double *up = malloc(sizeof(double) * n), *ua = malloc(sizeof(double) * 3 * n);
  int32_t *upd = malloc(sizeof(int32_t) * nb);
  or_walk_group_abu(t, zp, za, 1e-12, prev_npix, 1e-12, up, ua, upd);
  for (int64_t b = 0; b < nb; ++b) CHECK(upd[b] == 1);
  or_walk_group_abu(t, phi, acc, 1e-9, NULL, 0.0, up, ua, upd);
  for (int64_t b = 0; b < nb; ++b) CHECK(upd[b] == 0);
  free(zp), free(za), free(up), free(ua), free(upd), free(prev_npix);
  /* the surrogate walk with a zero network on periodic trees */
  if (p->bc[0] && p->ewald == 1) {
    const int np = or_mlp_nparam();
    double *prm = calloc(np, sizeof(double)), norm[23];
    for (int k = 0; k < 3; ++k) norm[k] = 0.5;
    for (int k = 0; k < 10; ++k) {
      norm[3 + k] = 0.01 * (k + 1);
      norm[13 + k] = 1.0;
    }
    or_walk_group_mlp(t, prm, norm, 2, sel, sp, sa, NULL);
    CHECK(all_finite(sp, 1024) && all_finite(sa, 3 * 1024));
    CHECK(or_mlp_group_level(t, 0) >= 0 && or_mlp_group_level(t, 0) <= 2);
    free(prm);
  }
  free(sp), free(sa), free(npix), free(tau), free(phi), free(acc), free(nint);
  or_tree_free(t);
  free(level), free(coord), free(rho);
}

static void exercise_invalid(void) {
  const int32_t nroot[3] = {1, 1, 1}, bc[3] = {0, 0, 0};
  or_params p = base_params(nroot, bc);
  int32_t level[2] = {2, 2}, coord[6] = {0, 0, 0, 0, 0, 0};
  double rho[1024];
  for (int i = 0; i < 1024; ++i) rho[i] = 1.0;
  int err = 0;
  CHECK(or_tree_new(&p, 2, level, coord, rho, &err) == NULL && err != 0); /* duplicate */
  level[1] = 0;
  CHECK(or_tree_new(&p, 2, level, coord, rho, &err) == NULL && err != 0); /* bad level */
  level[1] = 2;
  coord[3] = 1;
  CHECK(or_tree_new(&p, 2, level, coord, rho, &err) == NULL && err != 0); /* holes */
  coord[3] = 0;
  level[0] = level[1] = 1;
  p.list_group = 2;
  CHECK(or_tree_new(&p, 1, level, coord, rho, &err) == NULL && err == 7); /* list group */
}

static void exercise_columns_and_healpix(void) {
  for (int nside = 1; nside <= 4; nside *= 2) {
    const int64_t npx = 12 * nside * nside;
    for (int64_t q = 0; q < npx; ++q) {
      double zp[2];
      or_healpix_pix2ang(nside, q, zp);
      const double s = sqrt(1.0 - zp[0] * zp[0]);
      CHECK(or_healpix_vec2pix(nside, s * cos(zp[1]), s * sin(zp[1]), zp[0]) == q);
    }
    const int64_t ne = 6 * 8 * 5;  /* theta x phi x psi bins */
    const int64_t np = or_raytable_export(nside, 6, 8, 5, 8, 12, 0.98, NULL, NULL, NULL);
    CHECK(np > 0);
    int64_t *off = malloc(sizeof(int64_t) * (ne + 1));
    int32_t *pix = malloc(sizeof(int32_t) * (np > 0 ? np : 1));
    double *w = malloc(sizeof(double) * (np > 0 ? np : 1));
    CHECK(or_raytable_export(nside, 6, 8, 5, 8, 12, 0.98, off, pix, w) == np);
    CHECK(off[0] == 0 && off[ne] == np);
    for (int64_t q = 0; q < np; ++q) CHECK(pix[q] >= 0 && pix[q] < npx && isfinite(w[q]));
    free(off), free(pix), free(w);
  }
  double d[12], h[4];
  int64_t e[4];
  for (int i = 0; i < 12; ++i) d[i] = urand() - 0.5;
  for (int i = 0; i < 4; ++i) h[i] = 0.05 * urand();
  or_raytable_entries(25, 50, 25, 0.98, 4, d, h, e);
  for (int i = 0; i < 4; ++i) CHECK(e[i] >= 0);
  CHECK(or_morton(1, 0, 0) == 1 && or_morton(0, 1, 0) == 2 && or_morton(0, 0, 1) == 4);
}

static void exercise_ewald(void) {
  const double box3[3] = {1.0, 1.0, 1.0}, box2[3] = {1.0, 1.0, 4.0}, box1[3] = {1.0, 1.0, 1.0};
  double d[9], out[3 * 10];
  for (int i = 0; i < 9; ++i) d[i] = 0.4 * urand();
  or_ewald_eval(1, box3, 0.0, 0, 0, 1, 3, d, out);
  CHECK(all_finite(out, 3 * 10));
  or_ewald_eval(2, box2, 0.0, 0, 0, 1, 3, d, out);
  CHECK(all_finite(out, 3 * 10));
  or_ewald_eval(3, box1, 0.0, 0, 0, 1, 3, d, out);
  CHECK(all_finite(out, 3 * 10));
  const int n = 6;
  double *tab = malloc(sizeof(double) * n * n * n * 10);
  or_ewald_table(1, box3, 0.0, 0, 0, n, tab);
  CHECK(all_finite(tab, n * n * n * 10));
  or_ewald_table_lookup(1, box3, n, tab, 3, d, out);
  CHECK(all_finite(out, 3 * 4));
  free(tab);
  double it[8], kf[8];
  or_itilde(0.3, 0.7, 0.5, it);
  or_kfuncs(1, 0.4, 0.9, kf);
  CHECK(isfinite(it[0]) && isfinite(kf[0]));
}

static void exercise_mlp(void) {
  const int np = or_mlp_nparam();
  CHECK(np > 0);
  double *p = malloc(sizeof(double) * np), *g = malloc(sizeof(double) * np);
  double *m = calloc((size_t)(np > 0 ? np : 1), sizeof(double)), *v = calloc((size_t)(np > 0 ? np : 1), sizeof(double));
  for (int i = 0; i < np; ++i) p[i] = 0.1 * (urand() - 0.5);
  enum { B = 7 };
  double x[3 * B], y[10 * B], t[10 * B];
  for (int i = 0; i < 3 * B; ++i) x[i] = 2.0 * urand() - 1.0;
  for (int i = 0; i < 10 * B; ++i) t[i] = urand();
  or_mlp_forward(p, B, x, y);
  CHECK(all_finite(y, 10 * B));
  const double l0 = or_mlp_grad(p, B, x, t, g);
  CHECK(isfinite(l0) && all_finite(g, np));
  or_adam_update(p, g, m, v, np, 1e-3, 1);
  double l1 = 0.0;
  for (int s = 2; s < 6; ++s) l1 = or_mlp_adam(p, m, v, B, x, t, 1e-3, s);
  CHECK(isfinite(l1));
  free(p), free(g), free(m), free(v);
}

int main(void) {
  const int32_t one[3] = {1, 1, 1}, iso[3] = {0, 0, 0}, p3[3] = {1, 1, 1};
  const int32_t tall[3] = {1, 1, 2}, p2[3] = {1, 1, 0}, line[3] = {1, 1, 1}, p1[3] = {1, 0, 0};
  or_params p = base_params(one, iso);
  p.nside = 1;
  p.theta_pix = 1.0;
  exercise_tree(&p, "isolated BH, Nside 1");
  p = base_params(one, iso);
  p.mac = 2;
  p.a_lim = 1e-2;
  exercise_tree(&p, "isolated MPE");
  p = base_params(one, iso);
  p.mac = 1;
  p.a_lim = 1e-2;
  p.nside = 2;
  p.theta_pix = 0.5;
  exercise_tree(&p, "isolated APE, Nside 2");
  p = base_params(one, p3);
  exercise_tree(&p, "3P table");
  p = base_params(tall, p2);
  exercise_tree(&p, "2P1I table");
  p = base_params(line, p1);
  exercise_tree(&p, "1P2I table");
  p = base_params(tall, p2);
  p.list_group = 4;
  p.nside = 1;
  p.theta_pix = 1.0;
  exercise_tree(&p, "2P1I table, octant lists, Nside 1");
  exercise_invalid();
  exercise_columns_and_healpix();
  exercise_ewald();
  exercise_mlp();
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("oracle driver: all checks passed\n");
  return 0;
}
