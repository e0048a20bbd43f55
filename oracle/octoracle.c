/*
 * FP64 CPU oracle: grid, tree build, MACs, tree walks and direct sums.
 *
 * TEST INFRASTRUCTURE ONLY (see octoracle.h).  Everything here follows the
 * paper's definitions step by step:
 *   - amr-tree of blocks and block-trees down to cells (Sec. 2, first part);
 *   - node moments: total mass and centre of mass, built bottom-up (Sec. 2.1);
 *   - depth-first walk from the roots; a node is accepted by the MAC suite or
 *     opened (Sec. 2.1); geometric BH MAC, Eq. (1), with the safe box;
 *   - APE MAC, Eq. (6) with p = 1, against an absolute limit, Eq. (4);
 *   - MPE MAC, Eq. (2) with p = 1 (B_2, B_3 of Eq. (3), summed over the
 *     node's cells), against an absolute limit, Eq. (4);
 *   - monopole potential and acceleration, Eqs. (7) and (8);
 *   - adaptive block update (Sec. 2.2.6) from the eight corner cells;
 *   - reference solution by direct summation over all other cells (Sec. 3).
 *
 * Readings of the paper taken here (they bind the GPU library as well):
 *   - sums over the 8 children run in octant order o = 0..7 (bit 0 = x,
 *     bit 1 = y, bit 2 = z), left to right, in FP64 without FMA;
 *     S = sum of m x over the node, COM = S / M (geometric centre if M = 0);
 *     a cell's COM is its geometric centre (Sec. 2.1);
 *   - the safe box is a cuboid of edge eta_SB h centred on the node's
 *     geometric centre; the target (point or box) must lie strictly outside;
 *   - the MAC distance is from the node's COM to the closest target point;
 *     BH accepts if h^2 < theta^2 d^2, APE if G M h^2 < a_lim d^4, MPE if
 *     d > b_max and G (3 B_2 d - 2 B_3) < a_lim d^3 (d - b_max)^2 (Eq. (2)
 *     multiplied out), b_max the distance from the COM to the farthest corner;
 *   - B_p = sum of m |r_i - r_a|^p over the node's cells: per leaf block a
 *     partial sum over its cells in octant order (the walk's +1, +2, cell
 *     nesting), the partials added in the amr-tree's depth-first octant order;
 *     |d|^3 = d^2 sqrt(d^2);
 *   - leaf nodes (cells) are always accepted; the target cell itself is
 *     skipped by r^2 = 0 (the direct sum runs over "all the other cells");
 *   - periodic axes use the minimum image, wrapped to [-L/2, L/2).
 */
#include "octoracle.h"
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ utils */
static uint64_t spread3(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ULL) << (3 * b);
  return r;
}

uint64_t or_morton(uint64_t x, uint64_t y, uint64_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

typedef struct {
  int32_t level;
  int32_t c[3];
  uint64_t key;
  int64_t leaf; /* leaf block index or -1 */
} anode;

static int cmp_anode(const void *a, const void *b) {
  const anode *x = (const anode *)a, *y = (const anode *)b;
  if (x->level != y->level) return x->level < y->level ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  /* equal keys: leaves first so duplicates are easy to spot */
  if (x->leaf != y->leaf) return x->leaf > y->leaf ? -1 : 1;
  return 0;
}

double or_size_at(const or_tree *t, int lev) {
  return t->p.root_size / (double)(1LL << (lev - 1));
}

double or_wrap(const or_tree *t, int k, double d) {
  if (!t->p.bc[k]) return d;
  double L = t->box[k];
  return d - L * floor(d / L + 0.5);
}

static int64_t find_anode(const or_tree *t, int lev, const int32_t c[3]) {
  int sh = t->lmax - lev;
  uint64_t key = or_morton((uint64_t)c[0] << sh, (uint64_t)c[1] << sh, (uint64_t)c[2] << sh);
  int64_t lo = 0, hi = t->na - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    int32_t ml = t->alev[mid];
    uint64_t mk = t->akey[mid];
    if (ml == lev && mk == key) return mid;
    if (ml < lev || (ml == lev && mk < key)) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* --------------------------------------------------------------- geometry */
/* Node kind, size and geometric centre from its global id. */
int or_node_geom(const or_tree *t, int64_t id, double *size, double gc[3]) {
  const double *o = t->p.origin;
  if (id < t->na) {
    int l = t->alev[id];
    double s = or_size_at(t, l);
    *size = s;
    for (int k = 0; k < 3; ++k) gc[k] = o[k] + ((double)t->acoord[3 * id + k] + 0.5) * s;
    return OR_KIND_AMR;
  }
  int64_t r = id - t->na;
  if (r < 8 * t->nb) {
    int64_t lb = r / 8;
    int o1 = (int)(r % 8);
    double s = or_size_at(t, t->blev[lb]) / 2.0;
    *size = s;
    for (int k = 0; k < 3; ++k) {
      int64_t pos = 2 * (int64_t)t->bcoord[3 * lb + k] + ((o1 >> k) & 1);
      gc[k] = o[k] + ((double)pos + 0.5) * s;
    }
    return OR_KIND_P1;
  }
  r -= 8 * t->nb;
  if (r < 64 * t->nb) {
    int64_t lb = r / 64;
    int q = (int)(r % 64), o1 = q / 8, o2 = q % 8;
    double s = or_size_at(t, t->blev[lb]) / 4.0;
    *size = s;
    for (int k = 0; k < 3; ++k) {
      int64_t pos = 4 * (int64_t)t->bcoord[3 * lb + k] + 2 * ((o1 >> k) & 1) + ((o2 >> k) & 1);
      gc[k] = o[k] + ((double)pos + 0.5) * s;
    }
    return OR_KIND_P2;
  }
  r -= 64 * t->nb;
  int64_t lb = r / 512;
  int ci = (int)(r % 512);
  int ijk[3] = {ci % 8, (ci / 8) % 8, ci / 64};
  double s = or_size_at(t, t->blev[lb]) / 8.0;
  *size = s;
  for (int k = 0; k < 3; ++k) {
    int64_t pos = 8 * (int64_t)t->bcoord[3 * lb + k] + ijk[k];
    gc[k] = o[k] + ((double)pos + 0.5) * s;
  }
  return OR_KIND_CELL;
}

int64_t or_id_p1(const or_tree *t, int64_t lb, int o1) { return t->na + 8 * lb + o1; }
int64_t or_id_p2(const or_tree *t, int64_t lb, int o1, int o2) {
  return t->na + 8 * t->nb + 64 * lb + 8 * o1 + o2;
}
int64_t or_id_cell(const or_tree *t, int64_t lb, int ci) {
  return t->na + 72 * t->nb + 512 * lb + ci;
}
/* cell index i + 8 j + 64 k of the cell in octant o3 of +2 node (o1, o2) */
static int cell_of(int o1, int o2, int o3) {
  int ijk[3];
  for (int k = 0; k < 3; ++k)
    ijk[k] = 4 * ((o1 >> k) & 1) + 2 * ((o2 >> k) & 1) + ((o3 >> k) & 1);
  return ijk[0] + 8 * ijk[1] + 64 * ijk[2];
}

/* children of a node in octant order; returns the count (0 for a cell) */
int or_children(const or_tree *t, int64_t id, int64_t ch[8]) {
  if (id < t->na) {
    if (t->aleaf[id] >= 0) {
      for (int o = 0; o < 8; ++o) ch[o] = or_id_p1(t, t->aleaf[id], o);
    } else {
      for (int o = 0; o < 8; ++o) ch[o] = t->achild[8 * id + o];
    }
    return 8;
  }
  int64_t r = id - t->na;
  if (r < 8 * t->nb) {
    int64_t lb = r / 8;
    int o1 = (int)(r % 8);
    for (int o = 0; o < 8; ++o) ch[o] = or_id_p2(t, lb, o1, o);
    return 8;
  }
  r -= 8 * t->nb;
  if (r < 64 * t->nb) {
    int64_t lb = r / 64;
    int q = (int)(r % 64);
    for (int o = 0; o < 8; ++o) ch[o] = or_id_cell(t, lb, cell_of(q / 8, q % 8, o));
    return 8;
  }
  return 0;
}

/* ------------------------------------------------------------- tree build */
/* Bottom-up moments, Sec. 2.1: M = sum of child masses, S = sum of child
 * mass-weighted positions, both in octant order; COM = S / M. */
static void moments(or_tree *t, int64_t id) {
  double size, gc[3];
  int kind = or_node_geom(t, id, &size, gc);
  if (kind == OR_KIND_CELL) {
    int64_t r = id - t->na - 72 * t->nb;
    int64_t lb = r / 512;
    int ci = (int)(r % 512);
    double hcube = size * size * size;
    double m = t->rho[512 * lb + ci] * hcube;
    t->M[id] = m;
    for (int k = 0; k < 3; ++k) {
      t->S[3 * id + k] = m * gc[k];
      t->com[3 * id + k] = gc[k];
    }
    return;
  }
  int64_t ch[8];
  or_children(t, id, ch);
  double M = 0.0, S[3] = {0.0, 0.0, 0.0};
  for (int o = 0; o < 8; ++o) {
    moments(t, ch[o]);
    M = M + t->M[ch[o]];
    for (int k = 0; k < 3; ++k) S[k] = S[k] + t->S[3 * ch[o] + k];
  }
  t->M[id] = M;
  for (int k = 0; k < 3; ++k) {
    t->S[3 * id + k] = S[k];
    t->com[3 * id + k] = M > 0.0 ? S[k] / M : gc[k];
  }
}

/* MPE moments, Eq. (3): B_2 and B_3 of node `id` about its own COM, as the
 * sum of m |r_i - r_a|^2 and m |r_i - r_a|^3 over its cells.  The cells of a
 * leaf-block subtree are visited in octant order (+1, +2, cell) and summed
 * from zero into one partial per leaf block; an amr node adds its blocks'
 * partials in depth-first octant order. */
static void cells_partial(const or_tree *t, int64_t id, const double ra[3], double *s2, double *s3) {
  int64_t ch[8];
  if (id >= t->na + 72 * t->nb) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double d = t->com[3 * id + k] - ra[k];
      d2 = d2 + d * d;
    }
    *s2 = *s2 + t->M[id] * d2;
    *s3 = *s3 + t->M[id] * (d2 * sqrt(d2));
    return;
  }
  or_children(t, id, ch);
  for (int o = 0; o < 8; ++o) cells_partial(t, ch[o], ra, s2, s3);
}

static void amr_partials(const or_tree *t, int64_t id, const double ra[3], double *B2, double *B3) {
  if (t->aleaf[id] >= 0) {
    double s2 = 0.0, s3 = 0.0;
    cells_partial(t, id, ra, &s2, &s3);
    *B2 = *B2 + s2;
    *B3 = *B3 + s3;
    return;
  }
  for (int o = 0; o < 8; ++o) amr_partials(t, t->achild[8 * id + o], ra, B2, B3);
}

static void mpe_moments(or_tree *t) {
  const int64_t nnode = t->na + 72 * t->nb;
  t->B2 = (double *)calloc(nnode, sizeof(double));
  t->B3 = (double *)calloc(nnode, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t id = 0; id < nnode; ++id) {
    const double *ra = t->com + 3 * id;
    double B2 = 0.0, B3 = 0.0;
    if (id < t->na) amr_partials(t, id, ra, &B2, &B3);
    else cells_partial(t, id, ra, &B2, &B3);
    t->B2[id] = B2;
    t->B3[id] = B3;
  }
}

void or_tree_mpe_export(const or_tree *t, double *B2, double *B3) {
  const int64_t nnode = t->na + 72 * t->nb;
  if (t->B2 && B2) memcpy(B2, t->B2, sizeof(double) * nnode);
  if (t->B3 && B3) memcpy(B3, t->B3, sizeof(double) * nnode);
}

or_tree *or_tree_new(const or_params *p, int64_t nb, const int32_t *level,
                     const int32_t *coord, const double *rho, int *err) {
  *err = 0;
  if (nb <= 0) { *err = 1; return NULL; }
  int lmax = 1;
  for (int64_t b = 0; b < nb; ++b) {
    if (level[b] < 1 || level[b] > 20) { *err = 1; return NULL; }
    for (int k = 0; k < 3; ++k) {
      int64_t nmax = (int64_t)p->nroot[k] << (level[b] - 1);
      if (coord[3 * b + k] < 0 || coord[3 * b + k] >= nmax) { *err = 1; return NULL; }
    }
    if (level[b] > lmax) lmax = level[b];
  }
  if (rho) {
    for (int64_t i = 0; i < 512 * nb; ++i)
      if (!(rho[i] >= 0.0) || !isfinite(rho[i])) { *err = 5; return NULL; }
  }
  int bct;
  if (!p->bc[0] && !p->bc[1] && !p->bc[2]) bct = OR_BC_ISO;
  else if (p->bc[0] && p->bc[1] && p->bc[2]) bct = OR_BC_3P;
  else if (p->bc[0] && p->bc[1] && !p->bc[2]) bct = OR_BC_2P1I;
  else if (p->bc[0] && !p->bc[1] && !p->bc[2]) bct = OR_BC_1P2I;
  else { *err = 6; return NULL; }
  if (p->list_group != 0 && p->list_group != 4 && p->list_group != 8) { *err = 7; return NULL; }
  or_tree *t = (or_tree *)calloc(1, sizeof(or_tree));
  t->p = *p;
  t->bctype = bct;
  t->nb = nb;
  t->lmax = lmax;
  for (int k = 0; k < 3; ++k) t->box[k] = p->nroot[k] * p->root_size;
  t->blev = (int32_t *)malloc(sizeof(int32_t) * nb);
  t->bcoord = (int32_t *)malloc(sizeof(int32_t) * 3 * nb);
  memcpy(t->blev, level, sizeof(int32_t) * nb);
  memcpy(t->bcoord, coord, sizeof(int32_t) * 3 * nb);

  /* every leaf block and every ancestor of it */
  int64_t cap = 0;
  for (int64_t b = 0; b < nb; ++b) cap += level[b];
  anode *all = (anode *)malloc(sizeof(anode) * cap);
  int64_t n = 0;
  for (int64_t b = 0; b < nb; ++b) {
    for (int l = level[b]; l >= 1; --l) {
      anode a;
      a.level = l;
      int sh = level[b] - l;
      for (int k = 0; k < 3; ++k) a.c[k] = coord[3 * b + k] >> sh;
      int sf = lmax - l;
      a.key = or_morton((uint64_t)a.c[0] << sf, (uint64_t)a.c[1] << sf, (uint64_t)a.c[2] << sf);
      a.leaf = (l == level[b]) ? b : -1;
      all[n++] = a;
    }
  }
  qsort(all, n, sizeof(anode), cmp_anode);
  /* unique; a key that is a leaf must appear exactly once */
  int64_t na = 0;
  for (int64_t i = 0; i < n;) {
    int64_t j = i + 1;
    while (j < n && all[j].level == all[i].level && all[j].key == all[i].key) ++j;
    int nleaf = 0;
    for (int64_t q = i; q < j; ++q) nleaf += all[q].leaf >= 0;
    if (nleaf > 1) { *err = 2; free(all); or_tree_free(t); return NULL; }
    if (nleaf == 1 && j - i > 1) { *err = 3; free(all); or_tree_free(t); return NULL; }
    all[na++] = all[i];
    i = j;
  }
  t->na = na;
  t->alev = (int32_t *)malloc(sizeof(int32_t) * na);
  t->acoord = (int32_t *)malloc(sizeof(int32_t) * 3 * na);
  t->akey = (uint64_t *)malloc(sizeof(uint64_t) * na);
  t->aleaf = (int64_t *)malloc(sizeof(int64_t) * na);
  t->achild = (int64_t *)malloc(sizeof(int64_t) * 8 * na);
  for (int64_t i = 0; i < na; ++i) {
    t->alev[i] = all[i].level;
    for (int k = 0; k < 3; ++k) t->acoord[3 * i + k] = all[i].c[k];
    t->akey[i] = all[i].key;
    t->aleaf[i] = all[i].leaf;
  }
  free(all);
  /* children of internal amr nodes must all exist (no holes) */
  for (int64_t i = 0; i < na; ++i) {
    for (int o = 0; o < 8; ++o) t->achild[8 * i + o] = -1;
    if (t->aleaf[i] >= 0) continue;
    for (int o = 0; o < 8; ++o) {
      int32_t c[3];
      for (int k = 0; k < 3; ++k) c[k] = 2 * t->acoord[3 * i + k] + ((o >> k) & 1);
      int64_t ch = find_anode(t, t->alev[i] + 1, c);
      if (ch < 0) { *err = 4; or_tree_free(t); return NULL; }
      t->achild[8 * i + o] = ch;
    }
  }
  /* all root positions must be present */
  int64_t nr = 0;
  for (int64_t i = 0; i < na; ++i) nr += t->alev[i] == 1;
  if (nr != (int64_t)p->nroot[0] * p->nroot[1] * p->nroot[2]) { *err = 4; or_tree_free(t); return NULL; }
  t->nroots = nr;
  t->roots = (int64_t *)malloc(sizeof(int64_t) * nr);
  nr = 0;
  for (int64_t i = 0; i < na; ++i)
    if (t->alev[i] == 1) t->roots[nr++] = i;

  t->nn = na + 72 * nb + 512 * nb;
  if (bct != OR_BC_ISO) {
    int rc = p->ew_rcut2 > 0 ? p->ew_rcut2 : (bct == OR_BC_3P ? 15 : 10);
    int fc = p->ew_fcut2 > 0 ? p->ew_fcut2 : 10;
    or_ewald_setup(&t->ew, bct, t->box, p->ew_alpha, rc, fc, p->ew_n > 1 ? p->ew_n : 64,
                   p->ewald == 1);
  }
  if (p->nside > 0)
    or_raytable_build(&t->rt, p->nside, p->il_ntheta, p->il_nphi, p->il_npsi, p->il_nr,
                      p->il_nazi, p->psi_max);
  if (rho) {
    t->rho = rho;
    t->M = (double *)malloc(sizeof(double) * t->nn);
    t->S = (double *)malloc(sizeof(double) * 3 * t->nn);
    t->com = (double *)malloc(sizeof(double) * 3 * t->nn);
    for (int64_t r = 0; r < t->nroots; ++r) moments(t, t->roots[r]);
    t->rho = NULL;
    if (p->mac == 2) mpe_moments(t);
  }
  return t;
}

void or_tree_free(or_tree *t) {
  if (!t) return;
  free(t->blev); free(t->bcoord); free(t->alev); free(t->acoord); free(t->akey);
  free(t->aleaf); free(t->achild); free(t->roots); free(t->M); free(t->S); free(t->com);
  free(t->B2); free(t->B3);
  or_ewald_release(&t->ew);
  if (t->rt.off) or_raytable_free(&t->rt);
  free(t);
}
int64_t or_tree_na(const or_tree *t) { return t->na; }
int64_t or_tree_nn(const or_tree *t) { return t->nn; }

/* Export of the amr-tree topology and all node moments. */
void or_tree_export(const or_tree *t, int32_t *alev, int32_t *acoord, int64_t *aleaf,
                    int64_t *achild, uint64_t *akey, double *M, double *com) {
  if (alev) memcpy(alev, t->alev, sizeof(int32_t) * t->na);
  if (acoord) memcpy(acoord, t->acoord, sizeof(int32_t) * 3 * t->na);
  if (aleaf) memcpy(aleaf, t->aleaf, sizeof(int64_t) * t->na);
  if (achild) memcpy(achild, t->achild, sizeof(int64_t) * 8 * t->na);
  if (akey) memcpy(akey, t->akey, sizeof(uint64_t) * t->na);
  if (M) memcpy(M, t->M, sizeof(double) * t->nn);
  if (com) memcpy(com, t->com, sizeof(double) * 3 * t->nn);
}

/* -------------------------------------------------------------------- MAC */
/* MAC suite for a target box (centre cT, half-extent ext per axis; ext = 0
 * for a single target point).  Returns 1 to accept, 0 to open. */
int or_accept(const or_tree *t, int64_t id, const double cT[3], double ext) {
  const or_params *p = &t->p;
  double h, gc[3];
  or_node_geom(t, id, &h, gc);
  /* safe box: strictly outside the eta_SB-enlarged node cuboid */
  double half = 0.5 * p->eta_sb * h;
  int outside = 0;
  for (int k = 0; k < 3; ++k) {
    double d = or_wrap(t, k, cT[k] - gc[k]);
    if (fabs(d) - ext > half) outside = 1;
  }
  if (!outside) return 0;
  /* squared distance from the COM to the closest target point */
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    double d = or_wrap(t, k, cT[k] - t->com[3 * id + k]);
    double e = fabs(d) - ext;
    if (e > 0.0) d2 = d2 + e * e;
  }
  int ok;
  if (p->mac == 0) {
    ok = h * h < p->theta * p->theta * d2;
  } else if (p->mac == 1) {
    ok = p->G * t->M[id] * h * h < p->a_lim * d2 * d2;
  } else {
    /* Eq. (2), p = 1: G / d^2 (1 - b/d)^-2 (3 B_2 / d^2 - 2 B_3 / d^3) < a_lim */
    double b2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double e = fabs(t->com[3 * id + k] - gc[k]) + 0.5 * h;
      b2 = b2 + e * e;
    }
    double d = sqrt(d2), bmax = sqrt(b2), q = d - bmax;
    ok = d > bmax && p->G * (3.0 * t->B2[id] * d - 2.0 * t->B3[id]) < p->a_lim * (d2 * d) * (q * q);
  }
  if (p->theta_pix > 0.0) ok = ok && (h * h < p->theta_pix * p->theta_pix * d2);
  return ok;
}

/* ------------------------------------------------------------------- walk */
typedef struct {
  int64_t *v;
  int64_t n, cap;
} idlist;

static void push(idlist *l, int64_t x) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 1024;
    l->v = (int64_t *)realloc(l->v, sizeof(int64_t) * l->cap);
  }
  l->v[l->n++] = x;
}

/* depth-first traversal, Sec. 2.1: accept or open; cells always accepted */
static void visit(const or_tree *t, int64_t id, const double cT[3], double ext, idlist *out) {
  int64_t ch[8];
  if (id >= t->na + 72 * t->nb) { push(out, id); return; }
  if (or_accept(t, id, cT, ext)) { push(out, id); return; }
  int nc = or_children(t, id, ch);
  for (int o = 0; o < nc; ++o) visit(t, ch[o], cT, ext, out);
}

void or_block_target(const or_tree *t, int64_t lb, double cT[3], double *ext) {
  double s = or_size_at(t, t->blev[lb]);
  for (int k = 0; k < 3; ++k) cT[k] = t->p.origin[k] + ((double)t->bcoord[3 * lb + k] + 0.5) * s;
  *ext = 3.5 * (s / 8.0);
}

/* The group walk's target may also be one octant of the block, the 4^3
 * cells with the upper (bit a of so set) or lower half on each axis a: the
 * same closest-point MAC suite, with the box of those cells' centres
 * (half-extent 1.5 h about the octant's centre).  Every cell's list then
 * still passes the suite at the cell itself. */
void or_group_target(const or_tree *t, int64_t lb, int so, double cT[3], double *ext) {
  or_block_target(t, lb, cT, ext);
  if (so < 0) return;
  const double h = or_size_at(t, t->blev[lb]) / 8.0;
  for (int k = 0; k < 3; ++k) cT[k] += (((so >> k) & 1) ? 2.0 : -2.0) * h;
  *ext = 1.5 * h;
}

static idlist group_list(const or_tree *t, int64_t lb, int so) {
  double cT[3], ext;
  or_group_target(t, lb, so, cT, &ext);
  idlist l = {0, 0, 0};
  for (int64_t r = 0; r < t->nroots; ++r) visit(t, t->roots[r], cT, ext, &l);
  return l;
}

int64_t or_group_list(const or_tree *t, int64_t lb, int so, int64_t *out, int64_t cap) {
  idlist l = group_list(t, lb, so);
  int64_t n = l.n;
  if (out) for (int64_t i = 0; i < n && i < cap; ++i) out[i] = l.v[i];
  free(l.v);
  return n;
}

/* Interaction list of leaf block lb under the group MAC (ids, walk order). */
int64_t or_block_list(const or_tree *t, int64_t lb, int64_t *out, int64_t cap) {
  return or_group_list(t, lb, -1, out, cap);
}

/* The lists the cells of one leaf block use: the block's own, or with
 * list_group = 4 one per octant. */
typedef struct {
  idlist l[8];
  int n;
} blists;

static blists block_lists(const or_tree *t, int64_t lb) {
  blists b;
  memset(&b, 0, sizeof(b));
  b.n = t->p.list_group == 4 ? 8 : 1;
  for (int so = 0; so < b.n; ++so) b.l[so] = group_list(t, lb, b.n == 8 ? so : -1);
  return b;
}

static const idlist *cell_list(const blists *b, int ci) { return &b->l[b->n == 8 ? or_cell_octant(ci) : 0]; }

static int64_t blists_len(const blists *b) {
  int64_t n = 0;
  for (int so = 0; so < b->n; ++so) n += b->l[so].n;
  return n;
}

static void blists_free(blists *b) {
  for (int so = 0; so < b->n; ++so) free(b->l[so].v);
}

/* Neumaier-compensated sum */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
  a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* contribution of a source of unit mass at offset d = r - r_a:
 * phi (potential kernel, Phi = -G M phi) and A (a = -G M A), Eqs. (7), (8)
 * and, for periodic/mixed BCs, the Ewald forms of Sec. 2.2.3-2.2.4. */
static void pair_kernel(const or_tree *t, const double d[3], double *phi, double A[3]) {
  if (t->bctype == OR_BC_ISO) {
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    *phi = 1.0 / r;
    double r3 = r2 * r;
    for (int k = 0; k < 3; ++k) A[k] = d[k] / r3;
    return;
  }
  or_ewald_total(t, d, phi, A);
}

/* potential and acceleration at a target point x from a list of nodes and,
 * if cols != NULL, the column density map of the point (Sec. 2.3): every
 * node adds w M / (Omega_pix d^2) to the pixels its table entry lists. */
static void sum_list(const or_tree *t, const double x[3], const int64_t *ids, int64_t n,
                     double *phi_out, double acc_out[3], double *cols) {
  nsum ph = {0, 0}, ac[3] = {{0, 0}, {0, 0}, {0, 0}};
  const or_raytable *T = &t->rt;
  double omega = 0.0;
  if (cols) {
    omega = 4.0 * M_PI / (double)T->npix;
    for (int p = 0; p < T->npix; ++p) cols[p] = 0.0;
  }
  for (int64_t q = 0; q < n; ++q) {
    int64_t id = ids[q];
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = or_wrap(t, k, x[k] - t->com[3 * id + k]);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) continue; /* the target cell itself */
    double phi, A[3];
    pair_kernel(t, d, &phi, A);
    double GM = t->p.G * t->M[id];
    nadd(&ph, -GM * phi);
    for (int k = 0; k < 3; ++k) nadd(&ac[k], -GM * A[k]);
    if (cols) {
      double dist = sqrt(r2);
      if (dist > t->p.max_dist) continue;
      double h, gc[3];
      or_node_geom(t, id, &h, gc);
      double v[3] = {-d[0], -d[1], -d[2]};
      int64_t e = or_raytable_entry(T, v, dist, h);
      double base = t->M[id] / (omega * r2);
      for (int64_t j = T->off[e]; j < T->off[e + 1]; ++j) cols[T->pix[j]] += T->w[j] * base;
    }
  }
  *phi_out = nval(&ph);
  for (int k = 0; k < 3; ++k) acc_out[k] = nval(&ac[k]);
}

/* tau_avg = -ln( mean_p exp(-kappa N_p) ), Eq. (A_V) in generic form */
static double tau_avg(const or_tree *t, const double *cols) {
  double s = 0.0;
  for (int p = 0; p < t->rt.npix; ++p) s += exp(-t->p.kappa * cols[p]);
  return -log(s / (double)t->rt.npix);
}

void or_cell_centre(const or_tree *t, int64_t lb, int ci, double x[3]) {
  double s, gc[3];
  or_node_geom(t, or_id_cell(t, lb, ci), &s, gc);
  for (int k = 0; k < 3; ++k) x[k] = gc[k];
}

/* Group walk (one interaction list per leaf block, closest-point MAC) over a
 * subset of leaf blocks.  Outputs: phi [nsel*512], acc [3][nsel*512], and
 * with columns on npix [nsel][Npix][512], tau [nsel*512]; nint [nsel]. */
void or_walk_group_blocks(const or_tree *t, int64_t nsel, const int64_t *sel, double *phi,
                          double *acc, double *npix, double *tau, int64_t *nint) {
  int64_t ncell = 512 * nsel;
  int cols = npix && t->rt.off;
  int np = cols ? t->rt.npix : 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nsel; ++q) {
    int64_t lb = sel[q];
    blists bl = block_lists(t, lb);
    if (nint) nint[q] = blists_len(&bl);
    double *map = cols ? (double *)malloc(sizeof(double) * np) : NULL;
    for (int ci = 0; ci < 512; ++ci) {
      double x[3], ph, a[3];
      const idlist *l = cell_list(&bl, ci);
      or_cell_centre(t, lb, ci, x);
      sum_list(t, x, l->v, l->n, &ph, a, map);
      phi[512 * q + ci] = ph;
      for (int k = 0; k < 3; ++k) acc[k * ncell + 512 * q + ci] = a[k];
      if (cols) {
        for (int p = 0; p < np; ++p) npix[(q * np + p) * 512 + ci] = map[p];
        if (tau) tau[512 * q + ci] = tau_avg(t, map);
      }
    }
    free(map);
    blists_free(&bl);
  }
}

/* Adaptive block update (Sec. 2.2.6): per leaf block the group walk first
 * evaluates the eight corner cells (i, j, k in {0, 7}); when at each of them
 * the acceleration differs from the previous step's by less than tol (the
 * Euclidean norm of the difference, an absolute accuracy as in Eq. (4)) and,
 * with columns (prev_npix not NULL, the tree's ray table built), the optical
 * depth kappa N_p of every direction differs from the previous one by less
 * than tol_tau (the section names the optical depth among the quantities
 * compared at the corners; this also bounds the change of tau_avg), the
 * block keeps the previous values of all its cells, else all 512 cells are
 * evaluated.  prev_* and the outputs are full-size ([nb*512], acc
 * [3][nb*512], prev_npix [nb][Npix][512]); updated[lb] = 1 where the block
 * was evaluated. */
void or_walk_group_abu(const or_tree *t, const double *prev_phi, const double *prev_acc, double tol,
                       const double *prev_npix, double tol_tau, double *phi, double *acc, int32_t *updated) {
  const int64_t ncell = 512 * t->nb;
  const int cols = prev_npix && t->rt.off;
  const int np = t->rt.npix;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t lb = 0; lb < t->nb; ++lb) {
    blists bl = block_lists(t, lb);
    double *map = cols ? (double *)malloc(sizeof(double) * np) : NULL;
    int changed = 0;
    for (int k = 0; k < 8; ++k) {
      const int ci = 7 * (k & 1) + 56 * ((k >> 1) & 1) + 448 * ((k >> 2) & 1);
      double x[3], ph, a[3];
      const idlist *l = cell_list(&bl, ci);
      or_cell_centre(t, lb, ci, x);
      sum_list(t, x, l->v, l->n, &ph, a, map);
      double d2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double d = a[q] - prev_acc[q * ncell + 512 * lb + ci];
        d2 = d2 + d * d;
      }
      if (!(sqrt(d2) < tol)) changed = 1;
      for (int p = 0; cols && p < np; ++p)
        if (!(t->p.kappa * fabs(map[p] - prev_npix[(lb * np + p) * 512 + ci]) < tol_tau)) changed = 1;
    }
    free(map);
    updated[lb] = changed;
    for (int ci = 0; ci < 512; ++ci) {
      const int64_t o = 512 * lb + ci;
      if (changed) {
        double x[3], ph, a[3];
        const idlist *l = cell_list(&bl, ci);
        or_cell_centre(t, lb, ci, x);
        sum_list(t, x, l->v, l->n, &ph, a, NULL);
        phi[o] = ph;
        for (int q = 0; q < 3; ++q) acc[q * ncell + o] = a[q];
      } else {
        phi[o] = prev_phi[o];
        for (int q = 0; q < 3; ++q) acc[q * ncell + o] = prev_acc[q * ncell + o];
      }
    }
    blists_free(&bl);
  }
}

void or_walk_group(const or_tree *t, double *phi, double *acc, int64_t *nint) {
  int64_t *sel = (int64_t *)malloc(sizeof(int64_t) * t->nb);
  for (int64_t b = 0; b < t->nb; ++b) sel[b] = b;
  or_walk_group_blocks(t, t->nb, sel, phi, acc, NULL, NULL, nint);
  free(sel);
}

/* Sec. 2.1: the tree walked for one target point, the MAC suite evaluated at
 * the point itself (a target box of half-extent 0). */
static idlist point_list(const or_tree *t, const double x[3]) {
  idlist l = {0, 0, 0};
  for (int64_t r = 0; r < t->nroots; ++r) visit(t, t->roots[r], x, 0.0, &l);
  return l;
}

/* Interaction list of one target point (ids, walk order). */
int64_t or_point_list(const or_tree *t, const double x[3], int64_t *out, int64_t cap) {
  idlist l = point_list(t, x);
  int64_t n = l.n;
  if (out) for (int64_t i = 0; i < n && i < cap; ++i) out[i] = l.v[i];
  free(l.v);
  return n;
}

/* Potential and acceleration at one target point from its own list; a cell
 * whose centre is the point itself is skipped. */
static void walk_point(const or_tree *t, const double x[3], double *phi, double a[3], int64_t *nint) {
  idlist l = point_list(t, x);
  sum_list(t, x, l.v, l.n, phi, a, NULL);
  *nint = l.n;
  free(l.v);
}

/* Paper-literal walk: one depth-first traversal per target cell (point MAC).
 * Targets are global cell indices 512*lb + ci. */
void or_walk_percell(const or_tree *t, int64_t ntg, const int64_t *tg, double *phi,
                     double *acc, int64_t *nint) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < ntg; ++q) {
    int64_t lb = tg[q] / 512;
    int ci = (int)(tg[q] % 512);
    double x[3], ph, a[3];
    int64_t n;
    or_cell_centre(t, lb, ci, x);
    walk_point(t, x, &ph, a, &n);
    phi[q] = ph;
    for (int k = 0; k < 3; ++k) acc[k * ntg + q] = a[k];
    if (nint) nint[q] = n;
  }
}

/* The same walk at arbitrary target points xyz [n][3] (the position of a sink
 * particle, say); outputs phi [n], acc [3][n]. */
void or_walk_points(const or_tree *t, int64_t n, const double *xyz, double *phi, double *acc,
                    int64_t *nint) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n; ++q) {
    double ph, a[3];
    int64_t m;
    walk_point(t, xyz + 3 * q, &ph, a, &m);
    phi[q] = ph;
    for (int k = 0; k < 3; ++k) acc[k * n + q] = a[k];
    if (nint) nint[q] = m;
  }
}

/* Reference solution: direct summation over all other cells (Sec. 3).
 * Targets are global cell indices; outputs [ntg], [3][ntg]. */
void or_direct(const or_tree *t, int64_t ntg, const int64_t *tg, double *phi, double *acc) {
  int64_t ncell = 512 * t->nb;
  int64_t base = t->na + 72 * t->nb;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < ntg; ++q) {
    int64_t lb = tg[q] / 512;
    int ci = (int)(tg[q] % 512);
    double x[3];
    or_cell_centre(t, lb, ci, x);
    nsum ph = {0, 0}, ac[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t j = 0; j < ncell; ++j) {
      int64_t id = base + j;
      double d[3];
      for (int k = 0; k < 3; ++k) d[k] = or_wrap(t, k, x[k] - t->com[3 * id + k]);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 == 0.0) continue;
      double phk, A[3];
      pair_kernel(t, d, &phk, A);
      double GM = t->p.G * t->M[id];
      nadd(&ph, -GM * phk);
      for (int k = 0; k < 3; ++k) nadd(&ac[k], -GM * A[k]);
    }
    phi[q] = nval(&ph);
    for (int k = 0; k < 3; ++k) acc[k * ntg + q] = nval(&ac[k]);
  }
}
