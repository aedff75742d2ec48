/*
 * mdref.c -- plain FP64 CPU oracle (test infrastructure only; see mdref.h).
 *
 * Built with gcc -O2 -ffp-contract=off (no fast-math, no FMA contraction) so
 * that every expression is evaluated exactly as written.  Global sums use
 * long double accumulators.  OpenMP only splits independent per-particle
 * rows; every reduction is done serially in particle-id order.
 */
#include "mdref.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define AB(a, b) ((a) * MDREF_MAXT + (b))

static int valid_params(const mdref_params* p) {
  if (!p || p->ntypes < 1 || p->ntypes > MDREF_MAXT) return 0;
  if (p->potential < 0 || p->potential > 1 || p->trunc < 0 || p->trunc > 1) return 0;
  for (int a = 0; a < p->ntypes; ++a)
    for (int b = 0; b < p->ntypes; ++b)
      if (!(p->rc[AB(a, b)] > 0.0) || !(p->sig[AB(a, b)] > 0.0)) return 0;
  return 1;
}

static double max_rc(const mdref_params* p) {
  double m = 0.0;
  for (int a = 0; a < p->ntypes; ++a)
    for (int b = 0; b < p->ntypes; ++b)
      if (p->rc[AB(a, b)] > m) m = p->rc[AB(a, b)];
  return m;
}

/* ---- Eq. (1) / Eq. (2): untruncated pair potential and dV/dr ---------- */
double mdref_v(const mdref_params* p, int32_t a, int32_t b, double r) {
  double s = p->sig[AB(a, b)] / r;
  double s6 = s * s * s * s * s * s;
  double s12 = s6 * s6;
  if (p->potential == 1) return 4.0 * p->eps[AB(a, b)] * s12;
  return 4.0 * p->eps[AB(a, b)] * (s12 - s6);
}

double mdref_dv(const mdref_params* p, int32_t a, int32_t b, double r) {
  /* d/dr (s/r)^k = -k (s/r)^k / r */
  double s = p->sig[AB(a, b)] / r;
  double s6 = s * s * s * s * s * s;
  double s12 = s6 * s6;
  if (p->potential == 1) return -48.0 * p->eps[AB(a, b)] * s12 / r;
  return -4.0 * p->eps[AB(a, b)] * (12.0 * s12 - 6.0 * s6) / r;
}

/* ---- Eq. (3): V*(r) = [V(r) - V(rc) - (r - rc) V'(rc)] (1 - Theta(r - rc))
 * and f(r) = -d(V*)/dr = -V'(r) + V'(rc).  trunc = 1 drops the linear term. */
int mdref_pair(const mdref_params* p, int32_t a, int32_t b, double r,
               double* vstar, double* f) {
  double rc = p->rc[AB(a, b)];
  if (!(r < rc)) {
    *vstar = 0.0;
    *f = 0.0;
    return 0;
  }
  double vr = mdref_v(p, a, b, r), dvr = mdref_dv(p, a, b, r);
  double vc = mdref_v(p, a, b, rc), dvc = mdref_dv(p, a, b, rc);
  if (p->trunc == 0) {
    *vstar = vr - vc - (r - rc) * dvc;
    *f = -dvr + dvc;
  } else {
    *vstar = vr - vc;
    *f = -dvr;
  }
  return 0;
}

/* Minimum-image displacement component. */
static double min_image(double d, double L) {
  double k = nearbyint(d / L);
  double t = L * k;
  return d - t;
}

/* ---- brute force: every pair once (Newton's third law) ----------------- */
int mdref_forces_brute(const mdref_params* p, int64_t n, double L,
                       const double* x, const int32_t* type,
                       double* F, double* pe, double* w) {
  if (!valid_params(p) || n < 0 || !(L >= 2.0 * max_rc(p))) return -1;
  memset(F, 0, sizeof(double) * 3 * (size_t)n);
  long double upe = 0.0L, uw = 0.0L;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i + 1; j < n; ++j) {
      double d[3];
      for (int k = 0; k < 3; ++k) d[k] = min_image(x[3 * i + k] - x[3 * j + k], L);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double r = sqrt(r2);
      double vs, f;
      mdref_pair(p, type[i], type[j], r, &vs, &f);
      if (f == 0.0 && vs == 0.0) continue;
      for (int k = 0; k < 3; ++k) {
        double fk = f * d[k] / r;
        F[3 * i + k] += fk;
        F[3 * j + k] -= fk;
      }
      upe += vs;
      uw += f * r;
    }
  }
  *pe = (double)upe;
  *w = (double)uw;
  return 0;
}

/* ---- cell grid (cubic cells of side >= max cutoff + skin) -------------- */
int mdref_cell_grid(const mdref_params* p, double L, int32_t* nc, double* inv_cell) {
  if (!valid_params(p) || !(L > 0.0)) return -1;
  double side = max_rc(p) + p->skin;
  int32_t m = (int32_t)floor(L / side);
  if (m < 3) m = 1;
  *nc = m;
  *inv_cell = (double)m / L;
  return 0;
}

/* One periodic wrap of a coordinate, keeping the image counter. */
static int wrap_coord(double* c, int32_t* im, double L) {
  double v = *c;
  if (v < 0.0) {
    v += L;
    if (im) *im -= 1;
  } else if (v >= L) {
    v -= L;
    if (im) *im += 1;
  }
  if (v == L) { /* v was a tiny negative number and v + L rounded up to L */
    v = 0.0;
    if (im) *im += 1;
  }
  *c = v;
  return (v >= 0.0 && v < L) ? 0 : -1;
}

int mdref_build_cells(int64_t n, double L, int32_t nc, double inv_cell,
                      double* x, int32_t* img, int32_t* cell,
                      int32_t* cell_start, int32_t* order) {
  if (n < 0 || nc < 1 || !(L > 0.0)) return -1;
  int64_t ncell = (int64_t)nc * nc * nc;
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t q[3];
    for (int k = 0; k < 3; ++k) {
      if (wrap_coord(&x[3 * i + k], img ? &img[3 * i + k] : NULL, L) != 0) {
        bad = 1;
        q[k] = 0;
        continue;
      }
      int32_t t = (int32_t)(x[3 * i + k] * inv_cell);
      if (t > nc - 1) t = nc - 1;
      q[k] = t;
    }
    cell[i] = (q[2] * nc + q[1]) * nc + q[0];
  }
  if (bad) return -2;
  /* counting sort by (cell, id): ids are visited in ascending order */
  int64_t* cursor = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  if (!cursor) return -3;
  for (int64_t i = 0; i < n; ++i) cursor[cell[i] + 1] += 1;
  for (int64_t c = 0; c < ncell; ++c) cursor[c + 1] += cursor[c];
  for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = (int32_t)cursor[c];
  for (int64_t i = 0; i < n; ++i) order[cursor[cell[i]]++] = (int32_t)i;
  free(cursor);
  return 0;
}

/* Shift of a stencil neighbour: cell index q + o wrapped into [0, nc), with
 * the periodic image s in {-1, 0, 1}. */
static void stencil_axis(int32_t q, int32_t o, int32_t nc, int32_t* qn, double* s) {
  int32_t t = q + o;
  *s = 0.0;
  if (t < 0) {
    t += nc;
    *s = -1.0;
  } else if (t >= nc) {
    t -= nc;
    *s = 1.0;
  }
  *qn = t;
}

int mdref_build_nlist(const mdref_params* p, int64_t n, double L, int32_t nc,
                      const double* x, const int32_t* type,
                      const int32_t* cell, const int32_t* cell_start,
                      const int32_t* order, int32_t cap,
                      int32_t* count, int32_t* ids) {
  if (!valid_params(p) || n < 0 || cap < 0 || nc < 1) return -1;
  double thr[16];
  for (int a = 0; a < MDREF_MAXT; ++a)
    for (int b = 0; b < MDREF_MAXT; ++b) {
      double t = p->rc[AB(a, b)] + p->skin;
      thr[AB(a, b)] = t * t;
    }
  int overflow = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : overflow)
  for (int64_t i = 0; i < n; ++i) {
    int32_t cnt = 0;
    const double* xi = &x[3 * i];
    int32_t ti = type[i];
    if (nc == 1) {
      for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double e[3];
        for (int k = 0; k < 3; ++k) e[k] = min_image(x[3 * j + k] - xi[k], L);
        double r2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
        if (r2 < thr[AB(ti, type[j])]) {
          if (cnt < cap) ids[i * (int64_t)cap + cnt] = (int32_t)j;
          ++cnt;
        }
      }
    } else {
      int32_t c = cell[i];
      int32_t qx = c % nc, qy = (c / nc) % nc, qz = c / (nc * nc);
      for (int32_t oz = -1; oz <= 1; ++oz)
        for (int32_t oy = -1; oy <= 1; ++oy)
          for (int32_t ox = -1; ox <= 1; ++ox) {
            int32_t nx, ny, nz;
            double sx, sy, sz;
            stencil_axis(qx, ox, nc, &nx, &sx);
            stencil_axis(qy, oy, nc, &ny, &sy);
            stencil_axis(qz, oz, nc, &nz, &sz);
            double shx = sx * L, shy = sy * L, shz = sz * L;
            int32_t cn = (nz * nc + ny) * nc + nx;
            for (int32_t k = cell_start[cn]; k < cell_start[cn + 1]; ++k) {
              int32_t j = order[k];
              if (j == i) continue;
              /* the difference first, then the box shift: exchanging i and
               * j (and s for -s) negates every step exactly, so the test
               * is symmetric and the list pairs are those of the third-law
               * halving (section "Grid-search method") */
              double ex = (x[3 * (int64_t)j + 0] - xi[0]) + shx;
              double ey = (x[3 * (int64_t)j + 1] - xi[1]) + shy;
              double ez = (x[3 * (int64_t)j + 2] - xi[2]) + shz;
              double r2 = (ex * ex + ey * ey) + ez * ez;
              if (r2 < thr[AB(ti, type[j])]) {
                if (cnt < cap) ids[i * (int64_t)cap + cnt] = j;
                ++cnt;
              }
            }
          }
    }
    count[i] = cnt;
    if (cnt > cap) overflow = 1;
  }
  return overflow ? 1 : 0;
}

int mdref_forces_list(const mdref_params* p, int64_t n, double L,
                      const double* x, const int32_t* type, int32_t cap,
                      const int32_t* count, const int32_t* ids,
                      double* F, double* pe, double* w) {
  if (!valid_params(p) || n < 0) return -1;
  double* pei = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* wi = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!pei || !wi) {
    free(pei);
    free(wi);
    return -3;
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    double fi[3] = {0.0, 0.0, 0.0};
    double ui = 0.0, vi = 0.0;
    if (count[i] > cap) bad = 1;
    int32_t m = count[i] < cap ? count[i] : cap;
    for (int32_t k = 0; k < m; ++k) {
      int64_t j = ids[i * (int64_t)cap + k];
      double d[3];
      for (int q = 0; q < 3; ++q) d[q] = min_image(x[3 * i + q] - x[3 * j + q], L);
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double vs, f;
      mdref_pair(p, type[i], type[j], r, &vs, &f);
      if (f == 0.0 && vs == 0.0) continue;
      for (int q = 0; q < 3; ++q) fi[q] += f * d[q] / r;
      ui += 0.5 * vs;
      vi += 0.5 * f * r;
    }
    for (int q = 0; q < 3; ++q) F[3 * i + q] = fi[q];
    pei[i] = ui;
    wi[i] = vi;
  }
  long double upe = 0.0L, uw = 0.0L;
  for (int64_t i = 0; i < n; ++i) {
    upe += pei[i];
    uw += wi[i];
  }
  *pe = (double)upe;
  *w = (double)uw;
  free(pei);
  free(wi);
  return bad ? -4 : 0;
}

int mdref_forces_cells(const mdref_params* p, int64_t n, double L, int32_t nc,
                       const double* x, const int32_t* type,
                       const int32_t* cell, const int32_t* cell_start,
                       const int32_t* order, int64_t nsel, const int64_t* sel,
                       double* F, double* pe_i, double* w_i) {
  if (!valid_params(p) || n < 0 || nc < 1) return -1;
  if (!sel) nsel = n;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t s = 0; s < nsel; ++s) {
    int64_t i = sel ? sel[s] : s;
    double fi[3] = {0.0, 0.0, 0.0};
    double ui = 0.0, vi = 0.0;
    const double* xi = &x[3 * i];
    if (nc == 1) {
      for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3];
        for (int q = 0; q < 3; ++q) d[q] = min_image(xi[q] - x[3 * j + q], L);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double vs, f;
        mdref_pair(p, type[i], type[j], r, &vs, &f);
        if (f == 0.0 && vs == 0.0) continue;
        for (int q = 0; q < 3; ++q) fi[q] += f * d[q] / r;
        ui += 0.5 * vs;
        vi += 0.5 * f * r;
      }
    } else {
      int32_t c = cell[i];
      int32_t qx = c % nc, qy = (c / nc) % nc, qz = c / (nc * nc);
      for (int32_t oz = -1; oz <= 1; ++oz)
        for (int32_t oy = -1; oy <= 1; ++oy)
          for (int32_t ox = -1; ox <= 1; ++ox) {
            int32_t nx, ny, nz;
            double sx, sy, sz;
            stencil_axis(qx, ox, nc, &nx, &sx);
            stencil_axis(qy, oy, nc, &ny, &sy);
            stencil_axis(qz, oz, nc, &nz, &sz);
            double sh[3] = {sx * L, sy * L, sz * L};
            int32_t cn = (nz * nc + ny) * nc + nx;
            for (int32_t k = cell_start[cn]; k < cell_start[cn + 1]; ++k) {
              int64_t j = order[k];
              if (j == i) continue;
              double d[3];
              for (int q = 0; q < 3; ++q) d[q] = xi[q] - (x[3 * j + q] + sh[q]);
              double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
              double vs, f;
              mdref_pair(p, type[i], type[j], r, &vs, &f);
              if (f == 0.0 && vs == 0.0) continue;
              for (int q = 0; q < 3; ++q) fi[q] += f * d[q] / r;
              ui += 0.5 * vs;
              vi += 0.5 * f * r;
            }
          }
    }
    for (int q = 0; q < 3; ++q) F[3 * s + q] = fi[q];
    if (pe_i) pe_i[s] = ui;
    if (w_i) w_i[s] = vi;
  }
  return 0;
}

int mdref_rdf(int64_t n, double L, const double* x, double rmax,
              int32_t nbins, double* g) {
  if (n < 2 || nbins < 1 || !(rmax > 0.0) || rmax > 0.5 * L) return -1;
  double dr = rmax / nbins;
  long double* h = (long double*)calloc((size_t)nbins, sizeof(long double));
  if (!h) return -3;
  /* pair counts per bin: integers, so splitting the rows over threads and
     adding the per-thread counts gives exactly the serial histogram.  A
     thread whose count buffer cannot be allocated fails the whole call
     (no pair may go uncounted). */
  int failed = 0;
#pragma omp parallel
  {
    int64_t* hl = (int64_t*)calloc((size_t)nbins, sizeof(int64_t));
    if (!hl) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      if (!hl) continue;
      for (int64_t j = i + 1; j < n; ++j) {
        double d[3];
        for (int q = 0; q < 3; ++q) d[q] = min_image(x[3 * i + q] - x[3 * j + q], L);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r < rmax) {
          int32_t b = (int32_t)(r / dr);
          if (b >= nbins) b = nbins - 1;
          hl[b] += 1;
        }
      }
    }
    if (hl) {
#pragma omp critical
      for (int32_t b = 0; b < nbins; ++b) h[b] += (long double)hl[b];
      free(hl);
    }
  }
  if (failed) {
    free(h);
    return -3;
  }
  double V = L * L * L;
  const double pi = 3.14159265358979323846;
  for (int32_t b = 0; b < nbins; ++b) {
    double r0 = b * dr, r1 = (b + 1) * dr;
    double shell = 4.0 / 3.0 * pi * (r1 * r1 * r1 - r0 * r0 * r0);
    g[b] = (double)(2.0L * V * h[b] / ((long double)n * (long double)n * shell));
  }
  free(h);
  return 0;
}

/* ---- simulation: velocity Verlet with skin-triggered rebuilds ---------- */
struct mdref_sim {
  mdref_params p;
  int64_t n;
  double L, dt;
  int32_t brute, nc, cap, built;
  double inv_cell;
  double *x, *v, *F, *xref;
  int32_t *type, *img, *cell, *cell_start, *order, *count, *ids;
  double pe, w;
  int64_t rebuilds, step;
};

void mdref_sim_destroy(mdref_sim* s) {
  if (!s) return;
  free(s->x); free(s->v); free(s->F); free(s->xref);
  free(s->type); free(s->img); free(s->cell); free(s->cell_start);
  free(s->order); free(s->count); free(s->ids);
  free(s);
}

mdref_sim* mdref_sim_create(const mdref_params* p, int64_t n, double L,
                            double dt, int32_t brute) {
  if (!valid_params(p) || n < 2 || !(L >= 2.0 * (max_rc(p) + p->skin))) return NULL;
  mdref_sim* s = (mdref_sim*)calloc(1, sizeof(mdref_sim));
  if (!s) return NULL;
  s->p = *p;
  s->n = n;
  s->L = L;
  s->dt = dt;
  s->brute = brute;
  mdref_cell_grid(p, L, &s->nc, &s->inv_cell);
  size_t n3 = 3 * (size_t)n;
  int64_t ncell = (int64_t)s->nc * s->nc * s->nc;
  s->x = (double*)calloc(n3, sizeof(double));
  s->v = (double*)calloc(n3, sizeof(double));
  s->F = (double*)calloc(n3, sizeof(double));
  s->xref = (double*)calloc(n3, sizeof(double));
  s->type = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  s->img = (int32_t*)calloc(n3, sizeof(int32_t));
  s->cell = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  s->cell_start = (int32_t*)calloc((size_t)ncell + 1, sizeof(int32_t));
  s->order = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  s->count = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  s->cap = 64;
  s->ids = brute ? NULL : (int32_t*)calloc((size_t)n * s->cap, sizeof(int32_t));
  if (!s->x || !s->v || !s->F || !s->xref || !s->type || !s->img || !s->cell ||
      !s->cell_start || !s->order || !s->count || (!brute && !s->ids)) {
    mdref_sim_destroy(s);
    return NULL;
  }
  return s;
}

int mdref_sim_set_state(mdref_sim* s, const double* x, const double* v,
                        const int32_t* type) {
  size_t n3 = 3 * (size_t)s->n;
  memcpy(s->x, x, n3 * sizeof(double));
  memcpy(s->v, v, n3 * sizeof(double));
  memcpy(s->type, type, (size_t)s->n * sizeof(int32_t));
  memset(s->img, 0, n3 * sizeof(int32_t));
  for (int64_t i = 0; i < s->n; ++i)
    if (type[i] < 0 || type[i] >= s->p.ntypes) return -1;
  s->built = 0;
  s->step = 0;
  s->rebuilds = 0;
  return 0;
}

int mdref_sim_get_state(const mdref_sim* s, double* x, double* v, int32_t* img) {
  size_t n3 = 3 * (size_t)s->n;
  if (x) memcpy(x, s->x, n3 * sizeof(double));
  if (v) memcpy(v, s->v, n3 * sizeof(double));
  if (img) memcpy(img, s->img, n3 * sizeof(int32_t));
  return 0;
}

/* Wrap, bin, sort and (list mode) rebuild the neighbour list; x_ref = x. */
static int sim_rebuild(mdref_sim* s) {
  int rc = mdref_build_cells(s->n, s->L, s->nc, s->inv_cell, s->x, s->img,
                             s->cell, s->cell_start, s->order);
  if (rc) return rc;
  if (!s->brute) {
    for (;;) {
      rc = mdref_build_nlist(&s->p, s->n, s->L, s->nc, s->x, s->type, s->cell,
                             s->cell_start, s->order, s->cap, s->count, s->ids);
      if (rc < 0) return rc;
      if (rc == 0) break;
      int32_t m = 0;
      for (int64_t i = 0; i < s->n; ++i)
        if (s->count[i] > m) m = s->count[i];
      free(s->ids);
      s->cap = m + 16;
      s->ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)s->n * s->cap);
      if (!s->ids) return -3;
    }
  }
  memcpy(s->xref, s->x, 3 * (size_t)s->n * sizeof(double));
  s->rebuilds += 1;
  s->built = 1;
  return 0;
}

static int sim_forces(mdref_sim* s) {
  if (s->brute)
    return mdref_forces_brute(&s->p, s->n, s->L, s->x, s->type, s->F, &s->pe, &s->w);
  return mdref_forces_list(&s->p, s->n, s->L, s->x, s->type, s->cap, s->count,
                           s->ids, s->F, &s->pe, &s->w);
}

int mdref_sim_get_forces(mdref_sim* s, double* F, double* pe, double* w) {
  if (!s->built) {
    int rc = sim_rebuild(s);
    if (rc) return rc;
    rc = sim_forces(s);
    if (rc) return rc;
  }
  if (F) memcpy(F, s->F, 3 * (size_t)s->n * sizeof(double));
  if (pe) *pe = s->pe;
  if (w) *w = s->w;
  return 0;
}

static double kinetic(const mdref_sim* s) {
  long double k = 0.0L;
  for (int64_t i = 0; i < s->n; ++i) {
    double m = s->p.mass[s->type[i]];
    const double* v = &s->v[3 * i];
    k += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  }
  return (double)k;
}

int64_t mdref_sim_rebuilds(const mdref_sim* s) { return s->rebuilds; }

void mdref_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t mdref_max_threads(void) { return (int32_t)omp_get_max_threads(); }

int mdref_sim_step(mdref_sim* s, int32_t nsteps, int32_t thermostat,
                   double T0, double T1, int64_t ramp, mdref_obs* obs) {
  int rc;
  if (!s->built) {
    if ((rc = sim_rebuild(s))) return rc;
    if ((rc = sim_forces(s))) return rc;
  }
  const int64_t n = s->n;
  const double dt = s->dt, half = 0.5 * s->dt;
  const double h = 0.5 * s->p.skin;
  const double dof = 3.0 * (double)n - 3.0;
  const double V = s->L * s->L * s->L;
  for (int32_t k = 1; k <= nsteps; ++k) {
    /* first half kick and drift */
    for (int64_t i = 0; i < n; ++i) {
      double m = s->p.mass[s->type[i]];
      for (int q = 0; q < 3; ++q) {
        s->v[3 * i + q] += half * s->F[3 * i + q] / m;
        s->x[3 * i + q] += dt * s->v[3 * i + q];
      }
    }
    /* skin rule: rebuild once some particle moved more than skin/2 */
    double md2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double d0 = s->x[3 * i] - s->xref[3 * i];
      double d1 = s->x[3 * i + 1] - s->xref[3 * i + 1];
      double d2 = s->x[3 * i + 2] - s->xref[3 * i + 2];
      double d = d0 * d0 + d1 * d1 + d2 * d2;
      if (d > md2) md2 = d;
    }
    int rebuilt = 0;
    if (s->p.skin <= 0.0 || md2 > h * h) {
      if ((rc = sim_rebuild(s))) return rc;
      rebuilt = 1;
    }
    if ((rc = sim_forces(s))) return rc;
    /* second half kick */
    for (int64_t i = 0; i < n; ++i) {
      double m = s->p.mass[s->type[i]];
      for (int q = 0; q < 3; ++q) s->v[3 * i + q] += half * s->F[3 * i + q] / m;
    }
    double ke = kinetic(s);
    if (thermostat) {
      double frac = ramp > 0 ? (double)k / (double)ramp : 1.0;
      if (frac > 1.0) frac = 1.0;
      double tt = ramp > 0 ? T0 + (T1 - T0) * frac : T0;
      double ti = 2.0 * ke / dof;
      double lam = sqrt(tt / ti);
      for (int64_t i = 0; i < 3 * n; ++i) s->v[i] *= lam;
      ke = kinetic(s);
    }
    s->step += 1;
    if (obs) {
      mdref_obs* o = &obs[k - 1];
      o->ke = ke;
      o->pe = s->pe;
      o->w = s->w;
      o->T = 2.0 * ke / dof;
      o->P = (2.0 * ke + s->w) / (3.0 * V);
      o->E = ke + s->pe;
      o->max_disp2 = md2;
      o->step = s->step;
      o->rebuilt = rebuilt;
      o->pad = 0;
    }
  }
  return 0;
}
