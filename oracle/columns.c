/*
 * Column densities (OpticalDepth module, Sec. 2.3) for the FP64 oracle.
 * TEST INFRASTRUCTURE ONLY (see octoracle.h).
 *
 * - HEALPix NESTED pixelisation (Gorski et al. 2005): ang2pix from a direction
 *   vector and pix2ang of pixel centres, written from the published
 *   construction (12 base pixels; polar caps |z| > 2/3 and the equatorial belt).
 * - Node-ray intersection table (Sec. 2.3, "Node-Ray intersection"): for a
 *   grid of node directions (theta, phi) and angular sizes psi, the fraction
 *   of the node's mass that falls in each pixel.  Reading: the node is a
 *   uniform sphere of the node's volume, R_eq = h (3 / 4 pi)^(1/3), seen at
 *   angular radius psi; its disc is sampled on nr radii x nazi azimuths with
 *   weight sqrt(1 - (b/psi)^2) sin b (projected column x solid-angle element);
 *   samples are assigned at twice the resolution (Nside_f = 2 Nside, the
 *   paper's oversampling) and coarsened (NESTED parent = fine >> 2); weights are
 *   normalised to sum 1.  Bins: theta in [0, pi] and psi in [0, psi_max] are
 *   split into equal bins (entry at the bin centre), phi in [0, 2 pi) likewise;
 *   a direction falls in bin floor(x / dx), clamped to the last bin.
 * - In the walk, every accepted node adds w M / (Omega_pix d^2) to each of its
 *   pixels (the pixel-averaged column of mass M at distance d).
 * - tau_avg = -ln( (1/N_pix) sum_p exp(-kappa N_p) ), the generic form of the
 *   mean visual extinction, Eq. (A_V).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

static const double TWO_THIRDS = 2.0 / 3.0;

static int64_t interleave2(int64_t ix, int64_t iy) {
  int64_t r = 0;
  for (int b = 0; b < 30; ++b) {
    r |= ((ix >> b) & 1) << (2 * b);
    r |= ((iy >> b) & 1) << (2 * b + 1);
  }
  return r;
}

static void deinterleave2(int64_t v, int64_t *ix, int64_t *iy) {
  *ix = 0;
  *iy = 0;
  for (int b = 0; b < 30; ++b) {
    *ix |= ((v >> (2 * b)) & 1) << b;
    *iy |= ((v >> (2 * b + 1)) & 1) << b;
  }
}

/* NESTED pixel of direction (x, y, z) (any positive length). */
int64_t or_vec2pix_nest(int64_t nside, double x, double y, double z) {
  double s2 = x * x + y * y;
  double r = sqrt(s2 + z * z);
  double zn = z / r;
  double za = fabs(zn);
  double phi = atan2(y, x);
  if (phi < 0.0) phi += 2.0 * M_PI;
  double tt = phi / (0.5 * M_PI); /* [0, 4) */
  if (tt >= 4.0) tt = 0.0;
  int64_t face, ix, iy;
  if (za <= TWO_THIRDS) {
    /* equatorial belt: the pixel edges are lines of slope +-3/8 in (tt, z) */
    double t1 = (double)nside * (0.5 + tt);
    double t2 = (double)nside * (zn * 0.75);
    int64_t jp = (int64_t)(t1 - t2);
    int64_t jm = (int64_t)(t1 + t2);
    int64_t ifp = jp / nside, ifm = jm / nside;
    if (ifp == ifm) face = (ifp & 3) + 4;
    else if (ifp < ifm) face = ifp & 3;
    else face = (ifm & 3) + 8;
    ix = jm & (nside - 1);
    iy = nside - (jp & (nside - 1)) - 1;
  } else {
    /* polar caps: 1 - |z| computed without cancellation */
    int64_t ntt = (int64_t)tt;
    if (ntt > 3) ntt = 3;
    double tp = tt - (double)ntt;
    double one_minus = s2 / (r * (r + fabs(z)));
    double tmp = (double)nside * sqrt(3.0 * one_minus);
    int64_t jp = (int64_t)(tp * tmp);
    int64_t jm = (int64_t)((1.0 - tp) * tmp);
    if (jp > nside - 1) jp = nside - 1;
    if (jm > nside - 1) jm = nside - 1;
    if (zn >= 0) {
      face = ntt;
      ix = nside - jm - 1;
      iy = nside - jp - 1;
    } else {
      face = ntt + 8;
      ix = jp;
      iy = jm;
    }
  }
  return face * nside * nside + interleave2(ix, iy);
}

/* centre (z, phi) of NESTED pixel p */
void or_pix2ang_nest(int64_t nside, int64_t p, double *z, double *phi) {
  static const int jrll[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
  static const int jpll[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
  int64_t npface = nside * nside;
  int64_t face = p / npface, ix, iy;
  deinterleave2(p % npface, &ix, &iy);
  int64_t jr = jrll[face] * nside - ix - iy - 1;
  int64_t nr, kshift;
  if (jr < nside) {
    nr = jr;
    *z = 1.0 - (double)(nr * nr) / (3.0 * (double)npface);
    kshift = 0;
  } else if (jr > 3 * nside) {
    nr = 4 * nside - jr;
    *z = (double)(nr * nr) / (3.0 * (double)npface) - 1.0;
    kshift = 0;
  } else {
    nr = nside;
    *z = (double)(2 * nside - jr) * 2.0 / (3.0 * (double)nside);
    kshift = (jr - nside) & 1;
  }
  int64_t jp = (jpll[face] * nr + ix - iy + 1 + kshift) / 2;
  if (jp > 4 * nr) jp -= 4 * nr;
  if (jp < 1) jp += 4 * nr;
  *phi = ((double)jp - (double)(kshift + 1) * 0.5) * (0.5 * M_PI / (double)nr);
}

/* ---------------------------------------------------------- ray table */
int or_raytable_build(or_raytable *T, int nside, int ntheta, int nphi, int npsi, int nr,
                      int nazi, double psimax) {
  memset(T, 0, sizeof(*T));
  T->nside = nside;
  T->npix = 12 * nside * nside;
  T->ntheta = ntheta;
  T->nphi = nphi;
  T->npsi = npsi;
  T->nr = nr;
  T->nazi = nazi;
  T->psimax = psimax;
  T->dtheta = M_PI / (double)ntheta;
  T->dphi = (2.0 * M_PI) / (double)nphi;
  T->dpsi = psimax / (double)npsi;
  int64_t ne = (int64_t)ntheta * nphi * npsi;
  T->nentries = ne;
  int npix = T->npix;
  double *dense = (double *)calloc((size_t)ne * npix, sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t e = 0; e < ne; ++e) {
    int it = (int)(e / ((int64_t)nphi * npsi));
    int ip = (int)((e / npsi) % nphi);
    int is = (int)(e % npsi);
    double th = ((double)it + 0.5) * T->dtheta;
    double ph = ((double)ip + 0.5) * T->dphi;
    double ps = ((double)is + 0.5) * T->dpsi;
    double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    double c[3] = {st * cp, st * sp, ct};
    double et[3] = {ct * cp, ct * sp, -st};
    double ep[3] = {-sp, cp, 0.0};
    double *w = dense + e * npix;
    for (int r = 0; r < nr; ++r) {
      double u = ((double)r + 0.5) / (double)nr;
      double b = u * ps;
      double wr = sqrt(1.0 - u * u) * sin(b);
      double cb = cos(b), sb = sin(b);
      for (int a = 0; a < nazi; ++a) {
        double al = ((double)a + 0.5) * ((2.0 * M_PI) / (double)nazi);
        double ca = cos(al), sa = sin(al);
        double n[3];
        for (int k = 0; k < 3; ++k) n[k] = cb * c[k] + sb * (ca * et[k] + sa * ep[k]);
        int64_t fine = or_vec2pix_nest(2 * (int64_t)nside, n[0], n[1], n[2]);
        w[fine >> 2] += wr;
      }
    }
    double tot = 0.0;
    for (int p = 0; p < npix; ++p) tot += w[p];
    for (int p = 0; p < npix; ++p) w[p] = w[p] / tot;
  }
  T->off = (int64_t *)malloc(sizeof(int64_t) * (ne + 1));
  int64_t n = 0;
  for (int64_t e = 0; e < ne; ++e) {
    T->off[e] = n;
    for (int p = 0; p < npix; ++p) n += dense[e * npix + p] > 0.0;
  }
  T->off[ne] = n;
  T->pix = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
  T->w = (double *)malloc(sizeof(double) * (n ? n : 1));
  n = 0;
  for (int64_t e = 0; e < ne; ++e)
    for (int p = 0; p < npix; ++p)
      if (dense[e * npix + p] > 0.0) {
        T->pix[n] = p;
        T->w[n] = dense[e * npix + p];
        ++n;
      }
  free(dense);
  return 0;
}

void or_raytable_free(or_raytable *T) {
  free(T->off);
  free(T->pix);
  free(T->w);
  memset(T, 0, sizeof(*T));
}

/* table entry of a node seen from the target at offset v = r_a - r (|v| = d) */
int64_t or_raytable_entry(const or_raytable *T, const double v[3], double d, double h) {
  double q = v[2] / d; /* |q| <= 1 up to rounding */
  if (q > 1.0) q = 1.0;
  if (q < -1.0) q = -1.0;
  double th = acos(q);
  double ph = atan2(v[1], v[0]);
  if (ph < 0.0) ph += 2.0 * M_PI;
  int it = (int)floor(th / T->dtheta);
  if (it > T->ntheta - 1) it = T->ntheta - 1;
  int ip = (int)floor(ph / T->dphi);
  if (ip > T->nphi - 1) ip = T->nphi - 1;
  double s = OR_REQ * h / d;
  double ps = s >= 1.0 ? 0.5 * M_PI : asin(s);
  int is = (int)floor(ps / T->dpsi);
  if (is > T->npsi - 1) is = T->npsi - 1;
  return ((int64_t)it * T->nphi + ip) * T->npsi + is;
}

/* ---------------------------------------------------------- test exports */
/* table entries of nodes of size h[i] at offsets d[i] = r - r_a (target cell
 * minus node), as the walk bins them (v = -d, |v| = sqrt of the plain sum of
 * squares); -1 for d = 0 */
void or_raytable_entries(int ntheta, int nphi, int npsi, double psimax, int64_t n, const double *d,
                         const double *h, int64_t *out) {
  or_raytable T;
  memset(&T, 0, sizeof(T));
  T.ntheta = ntheta;
  T.nphi = nphi;
  T.npsi = npsi;
  T.psimax = psimax;
  T.dtheta = M_PI / (double)ntheta;
  T.dphi = (2.0 * M_PI) / (double)nphi;
  T.dpsi = psimax / (double)npsi;
  for (int64_t i = 0; i < n; ++i) {
    const double *di = d + 3 * i;
    double r2 = di[0] * di[0] + di[1] * di[1] + di[2] * di[2];
    if (r2 == 0.0) {
      out[i] = -1;
      continue;
    }
    double v[3] = {-di[0], -di[1], -di[2]};
    out[i] = or_raytable_entry(&T, v, sqrt(r2), h[i]);
  }
}

int64_t or_healpix_vec2pix(int64_t nside, double x, double y, double z) {
  return or_vec2pix_nest(nside, x, y, z);
}

void or_healpix_pix2ang(int64_t nside, int64_t p, double *out) {
  or_pix2ang_nest(nside, p, &out[0], &out[1]);
}

/* table sizes, then contents: off [ne+1], pix [n], w [n] */
int64_t or_raytable_export(int nside, int ntheta, int nphi, int npsi, int nr, int nazi,
                           double psimax, int64_t *off, int32_t *pix, double *w) {
  or_raytable T;
  or_raytable_build(&T, nside, ntheta, nphi, npsi, nr, nazi, psimax);
  int64_t n = T.off[T.nentries];
  if (off) memcpy(off, T.off, sizeof(int64_t) * (T.nentries + 1));
  if (pix) memcpy(pix, T.pix, sizeof(int32_t) * n);
  if (w) memcpy(w, T.w, sizeof(double) * n);
  or_raytable_free(&T);
  return n;
}

/* ---------------------------------------------------------- ray march */
/* Leaf cell containing point x (inside the domain): returns the global
 * cell index 512 lb + ci and the cell's box; -1 if x is outside. */
static int64_t locate(const or_tree *t, const double x[3], double lo[3], double *hsz) {
  int32_t rc[3];
  for (int k = 0; k < 3; ++k) {
    double u = (x[k] - t->p.origin[k]) / t->p.root_size;
    if (u < 0.0 || u >= (double)t->p.nroot[k]) return -1;
    rc[k] = (int32_t)floor(u);
  }
  /* root with this position */
  int64_t node = -1;
  for (int64_t r = 0; r < t->nroots; ++r) {
    int64_t id = t->roots[r];
    if (t->acoord[3 * id] == rc[0] && t->acoord[3 * id + 1] == rc[1] && t->acoord[3 * id + 2] == rc[2]) {
      node = id;
      break;
    }
  }
  while (t->aleaf[node] < 0) {
    double s = or_size_at(t, t->alev[node]);
    int o = 0;
    for (int k = 0; k < 3; ++k) {
      double mid = t->p.origin[k] + ((double)t->acoord[3 * node + k] + 0.5) * s;
      if (x[k] >= mid) o |= 1 << k;
    }
    node = t->achild[8 * node + o];
  }
  int64_t lb = t->aleaf[node];
  double h = or_size_at(t, t->blev[lb]) / 8.0;
  int ijk[3];
  for (int k = 0; k < 3; ++k) {
    double base = t->p.origin[k] + (double)(8 * (int64_t)t->bcoord[3 * lb + k]) * h;
    int i = (int)floor((x[k] - base) / h);
    if (i < 0) i = 0;
    if (i > 7) i = 7;
    ijk[k] = i;
    lo[k] = base + i * h;
  }
  *hsz = h;
  return 512 * lb + ijk[0] + 8 * ijk[1] + 64 * ijk[2];
}

/* integral of rho along the ray x0 + s n (s > s0) through the AMR cells,
 * until the isolated boundary, the edge of the minimum-image box around the
 * target in periodic axes, or max_dist. */
static double ray_column(const or_tree *t, const double x0[3], const double n[3], double s0,
                         const double *rho) {
  double sum = 0.0, s = s0;
  double lim = t->p.max_dist;
  for (int k = 0; k < 3; ++k)
    if (t->p.bc[k] && n[k] != 0.0) {
      double sk = 0.5 * t->box[k] / fabs(n[k]);
      if (sk < lim) lim = sk;
    }
  for (int guard = 0; guard < 1000000 && s < lim; ++guard) {
    double p[3], lo[3], h;
    for (int k = 0; k < 3; ++k) {
      p[k] = x0[k] + (s + 1e-12 * t->p.root_size) * n[k];
      if (t->p.bc[k]) {
        double L = t->box[k];
        p[k] = t->p.origin[k] + (p[k] - t->p.origin[k]) - L * floor((p[k] - t->p.origin[k]) / L);
      }
    }
    int64_t c = locate(t, p, lo, &h);
    if (c < 0) break;
    /* distance to the exit face of this cell along n */
    double ds = 1e300;
    for (int k = 0; k < 3; ++k) {
      if (n[k] > 0) ds = fmin(ds, (lo[k] + h - p[k]) / n[k]);
      else if (n[k] < 0) ds = fmin(ds, (lo[k] - p[k]) / n[k]);
    }
    if (ds < 0) ds = 0;
    double step = ds + 1e-12 * t->p.root_size;
    if (s + step > lim) step = lim - s;
    sum += rho[c] * step;
    s += step;
  }
  return sum;
}

/* Reference column map of target cell tg (global cell index) at coarse Nside
 * nside: mean over the NESTED Nside_f pixel-centre rays inside each coarse
 * pixel.  out [12 nside^2]. */
void or_raymarch(const or_tree *t, const double *rho, int64_t tg, int64_t nside, int64_t nside_f,
                 double *out) {
  int64_t lb = tg / 512;
  int ci = (int)(tg % 512);
  double x[3];
  or_cell_centre(t, lb, ci, x);
  double h = or_size_at(t, t->blev[lb]) / 8.0;
  int64_t nfine = 12 * nside_f * nside_f, ncoarse = 12 * nside * nside;
  int shift = 0;
  while ((nside << (shift / 2)) < nside_f) shift += 2;
  for (int64_t p = 0; p < ncoarse; ++p) out[p] = 0.0;
  for (int64_t f = 0; f < nfine; ++f) {
    double z, ph;
    or_pix2ang_nest(nside_f, f, &z, &ph);
    double st = sqrt((1.0 - z) * (1.0 + z));
    double n[3] = {st * cos(ph), st * sin(ph), z};
    /* leave the target cell first (the self cell is excluded) */
    double s0 = 1e300;
    for (int k = 0; k < 3; ++k)
      if (n[k] != 0.0) s0 = fmin(s0, 0.5 * h / fabs(n[k]));
    out[f >> shift] += ray_column(t, x, n, s0, rho);
  }
  double per = (double)(nfine / ncoarse);
  for (int64_t p = 0; p < ncoarse; ++p) out[p] /= per;
}
