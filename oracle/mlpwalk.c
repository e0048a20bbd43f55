/*
 * FP64 group walk with the learned surrogate in place of the Ewald table.
 * TEST INFRASTRUCTURE ONLY (see octoracle.h).
 *
 * The surrogate network (mlp.c) maps a folded offset u = |d| to the Ewald
 * table's ten channels at u: phi_c, A_c (3) and the second derivatives of
 * phi_c (xx, yy, zz, xy, xz, yz).  The walk uses it the way the table is used
 * in the second look-up approach of Sec. 2.2.5, a value plus a first-order
 * Taylor step, with the expansion point at the centre of a group of cells:
 *
 *   1. For leaf block lb (cell size h) the group is the block-tree node of
 *      side 2^gl cells, gl the largest of 2, 1, 0 with (2^gl - 1) h / 2 <=
 *      tmax, tmax = mlp_reach x half the table's smallest grid spacing: with
 *      mlp_reach = 1 its cells lie within the table's own Taylor offset of
 *      the group centre c_g.
 *   2. The group's interaction list is that of the group walk: the block's
 *      (or_block_list), or with list_group = 4 that of the block octant
 *      holding the group (or_group_list; groups of 4^3 cells or fewer never
 *      straddle two octants).
 *   3. Per (group, listed node): d0 = c_g - r_node, minimum image in periodic
 *      axes; network input x_k = 2 |d0_k| / ext_k - 1; output y_o sig_o +
 *      mu_o; signs restored (A_c,k odd in d_k; the xy, xz, yz derivatives
 *      odd in both of their components).
 *   4. Per cell x of the group, delta = x - c_g, d = d0 + delta (the image of
 *      its group):
 *        phi = 1/|d| + phi_c(d0) - A_c(d0) . delta
 *        A   = d/|d|^3 + A_c(d0) - H_c(d0) delta
 *      and Phi -= G M phi, a -= G M A (Neumaier sums), skipping d = 0.  In
 *      2P1I a group with |d0_z| > 2 Lx uses, at every cell, the far-field
 *      limit phi = -2 pi |d_z| / (b Lx^2) + sqrt(pi) / (b Lx),
 *      A = (0, 0, 2 pi sgn(d_z) / (b Lx^2)).
 * With columns on, the maps and tau_avg are those of the plain group walk
 * (they do not depend on the Ewald correction).
 */
#include "octoracle.h"
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

void or_mlp_forward(const double *p, int64_t B, const double *x, double *y);

enum { NOUT = 10 };

typedef struct { double s, c; } msum;
static void madd(msum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
  a->s = t;
}

/* group level of leaf block lb (step 1) */
int or_mlp_group_level(const or_tree *t, int64_t lb) {
  const or_ewald *e = &t->ew;
  double tmax = e->step[0];
  for (int k = 1; k < 3; ++k)
    if (e->step[k] < tmax) tmax = e->step[k];
  tmax = (t->p.mlp_reach > 0.0 ? t->p.mlp_reach : 1.0) * (0.5 * tmax);
  const double h = or_size_at(t, t->blev[lb]) / 8.0;
  if ((3.0 * h) * 0.5 <= tmax) return 2;
  if ((1.0 * h) * 0.5 <= tmax) return 1;
  return 0;
}

/* the ten channels of the surrogate at offset d0, signs restored (step 3);
 * norm = ext[3], mu[10], sig[10] */
static void surrogate10(const double *params, const double *norm, const double d0[3], double v[NOUT]) {
  double x[3], y[NOUT];
  for (int k = 0; k < 3; ++k) x[k] = 2.0 * fabs(d0[k]) / norm[k] - 1.0;
  or_mlp_forward(params, 1, x, y);
  for (int o = 0; o < NOUT; ++o) v[o] = y[o] * norm[3 + NOUT + o] + norm[3 + o];
  const double s[3] = {d0[0] < 0 ? -1.0 : 1.0, d0[1] < 0 ? -1.0 : 1.0, d0[2] < 0 ? -1.0 : 1.0};
  for (int k = 0; k < 3; ++k) v[1 + k] *= s[k];
  v[7] *= s[0] * s[1];
  v[8] *= s[0] * s[2];
  v[9] *= s[1] * s[2];
}

/* Group walk over the blocks sel[0..nsel) with the surrogate.  Outputs phi
 * [nsel*512], acc [3][nsel*512]; nint [nsel] (list lengths). */
void or_walk_group_mlp(const or_tree *t, const double *params, const double *norm, int64_t nsel,
                       const int64_t *sel, double *phi, double *acc, int64_t *nint) {
  const int64_t ncell = 512 * nsel;
  const or_ewald *e = &t->ew;
  const double bL2 = e->b * e->Lx * e->Lx;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nsel; ++q) {
    const int64_t lb = sel[q];
    const int nl = t->p.list_group == 4 ? 8 : 1;
    int64_t nl_len[8], *nl_ids[8], tot = 0;
    for (int so = 0; so < nl; ++so) {
      const int oct = nl == 8 ? so : -1;
      nl_len[so] = or_group_list(t, lb, oct, NULL, 0);
      nl_ids[so] = (int64_t *)malloc(sizeof(int64_t) * (nl_len[so] > 0 ? nl_len[so] : 1));
      or_group_list(t, lb, oct, nl_ids[so], nl_len[so]);
      tot += nl_len[so];
    }
    if (nint) nint[q] = tot;
    const int gl = or_mlp_group_level(t, lb), gs = 1 << gl, ga = 8 / gs;
    const double h = or_size_at(t, t->blev[lb]) / 8.0, gsz = h * (double)gs;
    msum *ph = (msum *)calloc(512, sizeof(msum)), *ac = (msum *)calloc(3 * 512, sizeof(msum));
    for (int gz = 0; gz < ga; ++gz)
      for (int gy = 0; gy < ga; ++gy)
        for (int gx = 0; gx < ga; ++gx) {
          const int gi[3] = {gx, gy, gz};
          double gc[3];
          for (int k = 0; k < 3; ++k)
            gc[k] = t->p.origin[k] + ((double)((int64_t)ga * t->bcoord[3 * lb + k] + gi[k]) + 0.5) * gsz;
          const int so = nl == 8 ? or_cell_octant(gx * gs + 8 * (gy * gs) + 64 * (gz * gs)) : 0;
          const int64_t n = nl_len[so], *ids = nl_ids[so];
          for (int64_t j = 0; j < n; ++j) {
            const int64_t id = ids[j];
            double d0[3], v[NOUT];
            for (int k = 0; k < 3; ++k) d0[k] = or_wrap(t, k, gc[k] - t->com[3 * id + k]);
            const int far = t->bctype == OR_BC_2P1I && fabs(d0[2]) > 2.0 * e->Lx;
            if (!far) surrogate10(params, norm, d0, v);
            const double GM = t->p.G * t->M[id];
            for (int cz = 0; cz < gs; ++cz)
              for (int cy = 0; cy < gs; ++cy)
                for (int cx = 0; cx < gs; ++cx) {
                  const int ijk[3] = {gx * gs + cx, gy * gs + cy, gz * gs + cz};
                  const int ci = ijk[0] + 8 * ijk[1] + 64 * ijk[2];
                  double x[3], dl[3], d[3];
                  or_cell_centre(t, lb, ci, x);
                  for (int k = 0; k < 3; ++k) {
                    dl[k] = x[k] - gc[k];
                    d[k] = d0[k] + dl[k];
                  }
                  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                  if (r2 == 0.0) continue; /* the target cell itself */
                  double p, A[3];
                  if (far) {
                    p = -2.0 * M_PI * fabs(d[2]) / bL2 + sqrt(M_PI) / (e->b * e->Lx);
                    A[0] = 0.0;
                    A[1] = 0.0;
                    A[2] = (d[2] < 0 ? -2.0 : 2.0) * M_PI / bL2;
                  } else {
                    static const int hidx[3][3] = {{4, 7, 8}, {7, 5, 9}, {8, 9, 6}};
                    const double r = sqrt(r2), r3 = r2 * r;
                    p = 1.0 / r + (v[0] - (v[1] * dl[0] + v[2] * dl[1] + v[3] * dl[2]));
                    for (int k = 0; k < 3; ++k) {
                      double a = v[1 + k];
                      for (int i = 0; i < 3; ++i) a -= v[hidx[k][i]] * dl[i];
                      A[k] = d[k] / r3 + a;
                    }
                  }
                  madd(&ph[ci], -GM * p);
                  for (int k = 0; k < 3; ++k) madd(&ac[3 * ci + k], -GM * A[k]);
                }
          }
        }
    for (int ci = 0; ci < 512; ++ci) {
      phi[512 * q + ci] = ph[ci].s + ph[ci].c;
      for (int k = 0; k < 3; ++k) acc[k * ncell + 512 * q + ci] = ac[3 * ci + k].s + ac[3 * ci + k].c;
    }
    free(ph);
    free(ac);
    for (int so = 0; so < nl; ++so) free(nl_ids[so]);
  }
}
