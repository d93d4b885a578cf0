/*
 * cp_oracle.c -- plain FP64 reference for critical-point probabilities of
 * uncertain 2-D fields (Athawale et al., "Uncertainty Visualization of
 * Critical Points of 2D Scalar Fields for Parametric and Nonparametric
 * Probabilistic Models", arXiv 2407.18015).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never includes, links or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header or table with the
 * HIP path.
 *
 * What it computes (Sec. 3 problem setting; Eq. 3 for the minimum, the
 * negation argument of Sec. 4.1.2 / 4.2 for the maximum):
 *
 *   P_min(v) = Pr[X_v < X_n for every existing 4-neighbour n]
 *            = integral of pdf_v(x) * prod_n S_n(x) dx,   S_n = 1 - CDF_n
 *   P_max(v) = integral of pdf_v(x) * prod_n F_n(x) dx,   F_n = CDF_n
 *
 * With independent X_i (Sec. 3) every inner integral of Eq. 3 is a survival
 * function, so the 5-fold integral is a 1-D integral.  The oracle evaluates
 * that definition directly: it splits the vertex support at every support end
 * and bin edge of the (up to) five distributions, writes each factor on a
 * sub-interval as a polynomial in a piece-centred variable s in [-1, 1]
 * (x = c + h s), multiplies the polynomials in coefficient form and integrates
 * exactly.  No ordering of breakpoints, no templates, no quadrature.
 *
 * Models:
 *   uniform       pdf 1/(b-a) on [a,b]                         (Sec. 4.3)
 *   Epanechnikov  pdf 3/(4w) (1 - ((x-m)/w)^2) on [m-w, m+w]   (Sec. 4.3)
 *   histogram     mixture of uniform kernels, one per bin       (Sec. 4.4.1)
 *                 pdf = m_j / Delta on bin j; masses are taken as given
 *                 (unconstrained), so S(x) = integral_x^inf pdf, which equals
 *                 sum(masses) below the range; P is multilinear in the masses
 *                 exactly as in the h^5 sum of Eq. 5.
 *   independent Gaussian  N(mu, sigma^2) per vertex (the parametric
 *                 comparison model of Sec. 5.2, fitted from the member mean
 *                 and standard deviation).  No closed form exists (Sec. 4.3),
 *                 so the 1-D integral is evaluated by adaptive quadrature to
 *                 ~1e-15 (see gauss_* below).
 *   multivariate Gaussian over the 5-point stencil, Monte Carlo (Sec. 5.2,
 *                 5.3; prior work the paper compares against): Philox4x32-10
 *                 counters, Box-Muller normals, hit-count and conditional
 *                 (Rao-Blackwellised) estimators, pathwise gradient.
 *
 * Boundary (Sec. 3 leaves it open): a vertex uses only its existing
 * neighbours (3 on an edge, 2 at a corner, none for a 1x1 grid).
 *
 * Stencil slot order used for Jacobians and gathers: 0 = v (self),
 * 1 = e (x+1), 2 = n (y-1), 3 = w (x-1), 4 = s (y+1).
 *
 * Parameter planes are dense [n_param][H][W] doubles:
 *   uniform      (lo, hi)
 *   Epanechnikov (m, w)
 *   histogram    (lo, hi, mass_0 .. mass_{nb-1})   -- lo/hi not differentiated
 *   Gaussian     (mu, sigma)
 *   mvg          (mu, L_00, L_10, L_11, L_20, ... L_44) lower-triangular
 *                Cholesky factor over the variable order (e, n, w, s, v)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_UNIFORM = 0, OR_EPANECHNIKOV = 1, OR_HISTOGRAM = 2, OR_MVG = 3, OR_GAUSSIAN = 4 };

#define NSLOT 5
#define PCOEF 16 /* degree <= 15: pdf (2) + four cubic survival factors (12) */
#define MAXNB 64
#define MAXBREAK (5 * (MAXNB + 1) + 4)

static const int SLOT_DY[NSLOT] = {0, 0, -1, 0, 1};
static const int SLOT_DX[NSLOT] = {0, 1, 0, -1, 0};

/* ------------------------------------------------------------------------ */
/* polynomials in s, coefficient form                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int d;
  double c[PCOEF];
} poly_t;

static void p_set0(poly_t* p, double c0) {
  p->d = 0;
  p->c[0] = c0;
}
static void p_set1(poly_t* p, double c0, double c1) {
  p->d = 1;
  p->c[0] = c0;
  p->c[1] = c1;
}
static void p_mul(poly_t* r, const poly_t* a, const poly_t* b) {
  poly_t t;
  t.d = a->d + b->d;
  for (int k = 0; k <= t.d; ++k) t.c[k] = 0.0;
  for (int i = 0; i <= a->d; ++i)
    for (int j = 0; j <= b->d; ++j) t.c[i + j] += a->c[i] * b->c[j];
  *r = t;
}
static void p_scale(poly_t* p, double s) {
  for (int k = 0; k <= p->d; ++k) p->c[k] *= s;
}
static void p_add(poly_t* r, const poly_t* a, const poly_t* b) {
  poly_t t;
  t.d = a->d > b->d ? a->d : b->d;
  for (int k = 0; k <= t.d; ++k) {
    double va = k <= a->d ? a->c[k] : 0.0, vb = k <= b->d ? b->c[k] : 0.0;
    t.c[k] = va + vb;
  }
  *r = t;
}
/* integral over x of a polynomial in s, x = c + h s, s in [-1, 1] */
static double p_integrate(const poly_t* p, double h) {
  double acc = 0.0;
  for (int k = 0; k <= p->d; k += 2) acc += 2.0 * p->c[k] / (double)(k + 1);
  return acc * h;
}
/* compose a cubic in u, q(u) = q0 + q1 u + q2 u^2 + q3 u^3, with u = al + be s */
static void p_cubic_of_linear(poly_t* r, const double q[4], double al, double be) {
  poly_t u, u2, u3, acc, t;
  p_set1(&u, al, be);
  p_mul(&u2, &u, &u);
  p_mul(&u3, &u2, &u);
  p_set0(&acc, q[0]);
  t = u;
  p_scale(&t, q[1]);
  p_add(&acc, &acc, &t);
  t = u2;
  p_scale(&t, q[2]);
  p_add(&acc, &acc, &t);
  t = u3;
  p_scale(&t, q[3]);
  p_add(&acc, &acc, &t);
  *r = acc;
}

/* ------------------------------------------------------------------------ */
/* one distribution of the stencil                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int model;
  double lo, hi;      /* support */
  double m, w;        /* Epanechnikov centre, half-width */
  int nb;             /* histogram bins */
  double delta;       /* histogram bin width */
  const double* mass; /* histogram masses (strided in the parameter planes) */
  int64_t mstride;
  double total; /* sum of masses (histogram); 1 otherwise */
} dist_t;

static double d_mass(const dist_t* d, int j) { return d->mass[(int64_t)j * d->mstride]; }
static double d_edge(const dist_t* d, int j) {
  if (j <= 0) return d->lo;
  if (j >= d->nb) return d->hi;
  return d->lo + (double)j * d->delta;
}

enum { K_PDF = 0, K_SURV = 1, K_CDF = 2 };

/* Region of the piece with centre c: -1 below support, +1 above, 0 inside
 * (histogram: *bin receives the bin index). */
static int d_region(const dist_t* d, double c, int* bin) {
  if (c < d->lo) return -1;
  if (c > d->hi) return 1;
  if (d->model == OR_HISTOGRAM) {
    int j = 0;
    while (j + 1 < d->nb && d_edge(d, j + 1) <= c) ++j;
    *bin = j;
  }
  return 0;
}

/*
 * Polynomial (in s, x = c + h s) of pdf / survival / CDF of distribution d on
 * a piece that lies inside one smooth segment of d.  dp < 0: the function
 * itself; dp >= 0: its partial derivative w.r.t. parameter dp (uniform:
 * 0 = lo, 1 = hi; Epanechnikov: 0 = m, 1 = w; histogram: mass index).
 */
static void d_poly(const dist_t* d, int kind, int dp, double c, double h, poly_t* out) {
  int bin = 0;
  int reg = d_region(d, c, &bin);
  if (reg != 0) {
    /* outside the support: pdf 0; S = total below / 0 above; F = 0 / total */
    double v = 0.0;
    if (dp < 0) {
      if (kind == K_SURV && reg < 0) v = d->total;
      if (kind == K_CDF && reg > 0) v = d->total;
    } else if (d->model == OR_HISTOGRAM) {
      if (kind == K_SURV && reg < 0) v = 1.0;
      if (kind == K_CDF && reg > 0) v = 1.0;
    }
    p_set0(out, v);
    return;
  }
  if (d->model == OR_UNIFORM) {
    double L = d->hi - d->lo, L2 = L * L;
    double sv = (d->hi - c) / L, sh = -h / L; /* S = (hi - x)/L */
    double fv = (c - d->lo) / L, fh = h / L;  /* F = (x - lo)/L */
    if (kind == K_PDF) {
      if (dp < 0) p_set0(out, 1.0 / L);
      else p_set0(out, dp == 0 ? 1.0 / L2 : -1.0 / L2);
    } else if (kind == K_SURV) {
      if (dp < 0) p_set1(out, sv, sh);
      else if (dp == 0) p_set1(out, sv / L, sh / L); /* dS/dlo = (hi-x)/L^2 */
      else p_set1(out, fv / L, fh / L);              /* dS/dhi = (x-lo)/L^2 */
    } else {
      if (dp < 0) p_set1(out, fv, fh);
      else if (dp == 0) p_set1(out, -sv / L, -sh / L); /* dF/dlo = -(hi-x)/L^2 */
      else p_set1(out, -fv / L, -fh / L);              /* dF/dhi = -(x-lo)/L^2 */
    }
    return;
  }
  if (d->model == OR_EPANECHNIKOV) {
    double w = d->w, al = (c - d->m) / w, be = h / w;
    double k = 3.0 / (4.0 * w);
    /* pdf(u) = k (1 - u^2) */
    double q_pdf[4] = {k, 0.0, -k, 0.0};
    if (kind == K_PDF) {
      if (dp < 0) {
        p_cubic_of_linear(out, q_pdf, al, be);
      } else if (dp == 0) { /* d pdf / dm = 3/(2 w^2) u */
        double q[4] = {0.0, 3.0 / (2.0 * w * w), 0.0, 0.0};
        p_cubic_of_linear(out, q, al, be);
      } else { /* d pdf / dw = 3/(4 w^2) (3u^2 - 1) */
        double kk = 3.0 / (4.0 * w * w);
        double q[4] = {-kk, 0.0, 3.0 * kk, 0.0};
        p_cubic_of_linear(out, q, al, be);
      }
      return;
    }
    double sgn = (kind == K_SURV) ? 1.0 : -1.0;
    if (dp < 0) {
      /* S(u) = (2 - 3u + u^3)/4, F(u) = (2 + 3u - u^3)/4 */
      double q[4] = {0.5, -0.75 * sgn, 0.0, 0.25 * sgn};
      p_cubic_of_linear(out, q, al, be);
    } else if (dp == 0) { /* dS/dm = pdf, dF/dm = -pdf */
      double q[4] = {sgn * k, 0.0, -sgn * k, 0.0};
      p_cubic_of_linear(out, q, al, be);
    } else { /* dS/dw = u pdf, dF/dw = -u pdf */
      double q[4] = {0.0, sgn * k, 0.0, -sgn * k};
      p_cubic_of_linear(out, q, al, be);
    }
    return;
  }
  /* histogram: inside bin `bin` */
  {
    double D = d->delta;
    double e0 = d_edge(d, bin), e1 = d_edge(d, bin + 1);
    double mj = d_mass(d, bin);
    if (kind == K_PDF) {
      if (dp < 0) p_set0(out, mj / D);
      else p_set0(out, dp == bin ? 1.0 / D : 0.0);
      return;
    }
    if (kind == K_SURV) {
      if (dp < 0) {
        double tail = 0.0;
        for (int i = bin + 1; i < d->nb; ++i) tail += d_mass(d, i);
        p_set1(out, tail + mj * (e1 - c) / D, -mj * h / D);
      } else if (dp > bin) {
        p_set0(out, 1.0);
      } else if (dp == bin) {
        p_set1(out, (e1 - c) / D, -h / D);
      } else {
        p_set0(out, 0.0);
      }
      return;
    }
    if (dp < 0) {
      double head = 0.0;
      for (int i = 0; i < bin; ++i) head += d_mass(d, i);
      p_set1(out, head + mj * (c - e0) / D, mj * h / D);
    } else if (dp < bin) {
      p_set0(out, 1.0);
    } else if (dp == bin) {
      p_set1(out, (c - e0) / D, h / D);
    } else {
      p_set0(out, 0.0);
    }
  }
}

/* value of S or F of d at a point (used for the boundary terms) */
static double d_point(const dist_t* d, int kind, double x) {
  poly_t p;
  d_poly(d, kind, -1, x, 0.0, &p);
  return p.c[0];
}

/* ------------------------------------------------------------------------ */
/* grids                                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int model, H, W, nb;
  const double* par; /* [np][H][W] */
} grid_t;

static int n_param(int model, int nb) {
  if (model == OR_HISTOGRAM) return 2 + nb;
  if (model == OR_MVG) return 16;
  return 2;
}

static void grid_dist(const grid_t* g, int y, int x, dist_t* d) {
  int64_t plane = (int64_t)g->H * g->W, at = (int64_t)y * g->W + x;
  double p0 = g->par[at], p1 = g->par[plane + at];
  memset(d, 0, sizeof(*d));
  d->model = g->model;
  d->total = 1.0;
  if (g->model == OR_UNIFORM) {
    d->lo = p0;
    d->hi = p1;
  } else if (g->model == OR_EPANECHNIKOV) {
    d->m = p0;
    d->w = p1;
    d->lo = p0 - p1;
    d->hi = p0 + p1;
  } else {
    d->lo = p0;
    d->hi = p1;
    d->nb = g->nb;
    d->delta = (p1 - p0) / (double)g->nb;
    d->mass = g->par + 2 * plane + at;
    d->mstride = plane;
    d->total = 0.0;
    for (int j = 0; j < g->nb; ++j) d->total += d_mass(d, j);
  }
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* All breakpoints of the given distributions inside [lo, hi], sorted, unique. */
static int breakpoints(const dist_t* ds, int nd, double lo, double hi, double* out) {
  int n = 0;
  out[n++] = lo;
  out[n++] = hi;
  for (int k = 0; k < nd; ++k) {
    const dist_t* d = &ds[k];
    int ne = d->model == OR_HISTOGRAM ? d->nb : 1;
    for (int j = 0; j <= ne; ++j) {
      double e = d->model == OR_HISTOGRAM ? d_edge(d, j) : (j == 0 ? d->lo : d->hi);
      if (e > lo && e < hi) out[n++] = e;
    }
  }
  qsort(out, (size_t)n, sizeof(double), cmp_double);
  int u = 0;
  for (int i = 0; i < n; ++i)
    if (u == 0 || out[i] != out[u - 1]) out[u++] = out[i];
  return u;
}

/*
 * Per-vertex probabilities and (optionally) the Jacobian of P_min / P_max
 * with respect to every parameter of the five stencil members.
 * jmin/jmax: [NSLOT][np] (slot of an absent neighbour stays 0).
 */
static void cf_vertex(const grid_t* g, int y, int x, double* pmin, double* pmax, double* jmin,
                      double* jmax) {
  dist_t ds[NSLOT];
  int slot_of[NSLOT]; /* ds[k] sits in stencil slot slot_of[k] */
  int nd = 0;
  for (int s = 0; s < NSLOT; ++s) {
    int yy = y + SLOT_DY[s], xx = x + SLOT_DX[s];
    if (yy < 0 || yy >= g->H || xx < 0 || xx >= g->W) continue;
    grid_dist(g, yy, xx, &ds[nd]);
    slot_of[nd] = s;
    ++nd;
  }
  const dist_t* v = &ds[0]; /* slot 0 always exists */
  int np = n_param(g->model, g->nb);
  if (jmin) memset(jmin, 0, sizeof(double) * NSLOT * np);
  if (jmax) memset(jmax, 0, sizeof(double) * NSLOT * np);

  double bp[MAXBREAK];
  int nbp = breakpoints(ds, nd, v->lo, v->hi, bp);
  double smin = 0.0, smax = 0.0;
  for (int i = 0; i + 1 < nbp; ++i) {
    double c = 0.5 * (bp[i] + bp[i + 1]), h = 0.5 * (bp[i + 1] - bp[i]);
    if (!(h > 0.0)) continue;
    poly_t pdf, sv[NSLOT], fv[NSLOT], gs, gf, t;
    d_poly(v, K_PDF, -1, c, h, &pdf);
    p_set0(&gs, 1.0);
    p_set0(&gf, 1.0);
    for (int k = 1; k < nd; ++k) {
      d_poly(&ds[k], K_SURV, -1, c, h, &sv[k]);
      d_poly(&ds[k], K_CDF, -1, c, h, &fv[k]);
      p_mul(&gs, &gs, &sv[k]);
      p_mul(&gf, &gf, &fv[k]);
    }
    p_mul(&t, &pdf, &gs);
    smin += p_integrate(&t, h);
    p_mul(&t, &pdf, &gf);
    smax += p_integrate(&t, h);
    if (!jmin) continue;
    /* own parameters: d pdf / d theta times the product of the factors */
    int ownp = g->model == OR_HISTOGRAM ? g->nb : 2;
    int off = g->model == OR_HISTOGRAM ? 2 : 0;
    for (int q = 0; q < ownp; ++q) {
      poly_t dpdf;
      d_poly(v, K_PDF, q, c, h, &dpdf);
      p_mul(&t, &dpdf, &gs);
      jmin[0 * np + off + q] += p_integrate(&t, h);
      p_mul(&t, &dpdf, &gf);
      jmax[0 * np + off + q] += p_integrate(&t, h);
    }
    /* neighbour parameters: pdf * dS_k * prod_{j != k} S_j */
    for (int k = 1; k < nd; ++k) {
      poly_t los, lof; /* leave-one-out products */
      p_set0(&los, 1.0);
      p_set0(&lof, 1.0);
      for (int j = 1; j < nd; ++j) {
        if (j == k) continue;
        p_mul(&los, &los, &sv[j]);
        p_mul(&lof, &lof, &fv[j]);
      }
      p_mul(&los, &los, &pdf);
      p_mul(&lof, &lof, &pdf);
      for (int q = 0; q < ownp; ++q) {
        poly_t dq;
        d_poly(&ds[k], K_SURV, q, c, h, &dq);
        p_mul(&t, &dq, &los);
        jmin[slot_of[k] * np + off + q] += p_integrate(&t, h);
        d_poly(&ds[k], K_CDF, q, c, h, &dq);
        p_mul(&t, &dq, &lof);
        jmax[slot_of[k] * np + off + q] += p_integrate(&t, h);
      }
    }
  }
  /* Leibniz terms where the uniform vertex pdf jumps (its support ends) */
  if (jmin && g->model == OR_UNIFORM) {
    double L = v->hi - v->lo;
    double gs_lo = 1.0, gs_hi = 1.0, gf_lo = 1.0, gf_hi = 1.0;
    for (int k = 1; k < nd; ++k) {
      gs_lo *= d_point(&ds[k], K_SURV, v->lo);
      gs_hi *= d_point(&ds[k], K_SURV, v->hi);
      gf_lo *= d_point(&ds[k], K_CDF, v->lo);
      gf_hi *= d_point(&ds[k], K_CDF, v->hi);
    }
    jmin[0] += -gs_lo / L;
    jmin[1] += gs_hi / L;
    jmax[0] += -gf_lo / L;
    jmax[1] += gf_hi / L;
  }
  *pmin = smin;
  *pmax = smax;
}

/*
 * Saddle probability (Eq. 2 in 1-D, Eq. 4 on the 4-neighbour stencil):
 *   t1 = Pr[X_v < X_e, X_v > X_n, X_v < X_w, X_v > X_s]
 *      = integral pdf_v S_e F_n S_w F_s dx      (independence, Sec. 3)
 *   t2 = the same with every inequality reversed
 *      = integral pdf_v F_e S_n F_w S_s dx
 * Defined on interior vertices only: the alternating pattern needs the full
 * ring of four neighbours; a boundary vertex gets 0.
 */
static void cf_saddle_vertex(const grid_t* g, int y, int x, double* t1, double* t2) {
  *t1 = *t2 = 0.0;
  if (y < 1 || y > g->H - 2 || x < 1 || x > g->W - 2) return;
  dist_t ds[NSLOT];
  for (int s = 0; s < NSLOT; ++s) grid_dist(g, y + SLOT_DY[s], x + SLOT_DX[s], &ds[s]);
  const dist_t* v = &ds[0];
  double bp[MAXBREAK];
  int nbp = breakpoints(ds, NSLOT, v->lo, v->hi, bp);
  /* slot 1 = e, 2 = n, 3 = w, 4 = s */
  const int kind1[NSLOT] = {0, K_SURV, K_CDF, K_SURV, K_CDF};
  const int kind2[NSLOT] = {0, K_CDF, K_SURV, K_CDF, K_SURV};
  for (int i = 0; i + 1 < nbp; ++i) {
    double c = 0.5 * (bp[i] + bp[i + 1]), h = 0.5 * (bp[i + 1] - bp[i]);
    if (!(h > 0.0)) continue;
    poly_t pdf, a, b, f;
    d_poly(v, K_PDF, -1, c, h, &pdf);
    a = pdf;
    b = pdf;
    for (int k = 1; k < NSLOT; ++k) {
      d_poly(&ds[k], kind1[k], -1, c, h, &f);
      p_mul(&a, &a, &f);
      d_poly(&ds[k], kind2[k], -1, c, h, &f);
      p_mul(&b, &b, &f);
    }
    *t1 += p_integrate(&a, h);
    *t2 += p_integrate(&b, h);
  }
}

int or_saddle_at(int model, int H, int W, int nb, const double* params, int64_t nidx, const int64_t* idx,
                 double* t1, double* t2) {
  if (H < 1 || W < 1 || model < OR_UNIFORM || model > OR_HISTOGRAM) return 1;
  if (model == OR_HISTOGRAM && (nb < 1 || nb > MAXNB)) return 1;
  grid_t g = {model, H, W, nb, params};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nidx; ++i) cf_saddle_vertex(&g, (int)(idx[i] / W), (int)(idx[i] % W), &t1[i], &t2[i]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* public closed-form entry points                                            */
/* ------------------------------------------------------------------------ */
int or_n_param(int model, int nb) { return n_param(model, nb); }

static int check_grid(int model, int H, int W, int nb) {
  if (H < 1 || W < 1) return 1;
  if (model < OR_UNIFORM || model > OR_HISTOGRAM) return 1;
  if (model == OR_HISTOGRAM && (nb < 1 || nb > MAXNB)) return 1;
  return 0;
}

int or_forward(int model, int H, int W, int nb, const double* params, double* pmin, double* pmax) {
  if (check_grid(model, H, W, nb)) return 1;
  grid_t g = {model, H, W, nb, params};
  int64_t n = (int64_t)H * W;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) cf_vertex(&g, (int)(i / W), (int)(i % W), &pmin[i], &pmax[i], 0, 0);
  return 0;
}

int or_forward_at(int model, int H, int W, int nb, const double* params, int64_t nidx,
                  const int64_t* idx, double* pmin, double* pmax) {
  if (check_grid(model, H, W, nb)) return 1;
  grid_t g = {model, H, W, nb, params};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nidx; ++i)
    cf_vertex(&g, (int)(idx[i] / W), (int)(idx[i] % W), &pmin[i], &pmax[i], 0, 0);
  return 0;
}

/* Jacobians of the stencil centred at each listed vertex: [nidx][NSLOT][np] */
int or_jacobian_at(int model, int H, int W, int nb, const double* params, int64_t nidx,
                   const int64_t* idx, double* jmin, double* jmax) {
  if (check_grid(model, H, W, nb)) return 1;
  grid_t g = {model, H, W, nb, params};
  int np = n_param(model, nb);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nidx; ++i) {
    double a, b;
    cf_vertex(&g, (int)(idx[i] / W), (int)(idx[i] % W), &a, &b, jmin + i * NSLOT * np,
              jmax + i * NSLOT * np);
  }
  return 0;
}

/*
 * Adjoint: grad[k][u] = sum over stencils v containing u of
 *   g_min(v) dP_min(v)/dtheta_k(u) + g_max(v) dP_max(v)/dtheta_k(u).
 * Computed for the listed vertices u only (out: [nidx][np]).
 * absval != 0 sums the magnitudes of those ten terms instead (the scale of
 * the cancellation in the sum, used to state rounding tolerances).
 */
int or_grad_at(int model, int H, int W, int nb, const double* params, const double* gmin,
               const double* gmax, int64_t nidx, const int64_t* idx, double* out, int absval) {
  if (check_grid(model, H, W, nb)) return 1;
  grid_t g = {model, H, W, nb, params};
  int np = n_param(model, nb);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nidx; ++i) {
    int y = (int)(idx[i] / W), x = (int)(idx[i] % W);
    double* o = out + i * np;
    for (int k = 0; k < np; ++k) o[k] = 0.0;
    double jm[NSLOT * (2 + MAXNB)], jx[NSLOT * (2 + MAXNB)];
    /* u sits in slot 0 of its own stencil and in slot s of the stencil
       centred at u - offset(s) */
    for (int s = 0; s < NSLOT; ++s) {
      int vy = y - SLOT_DY[s], vx = x - SLOT_DX[s];
      if (vy < 0 || vy >= H || vx < 0 || vx >= W) continue;
      double a, b;
      cf_vertex(&g, vy, vx, &a, &b, jm, jx);
      int64_t at = (int64_t)vy * W + vx;
      for (int k = 0; k < np; ++k) {
        double a = gmin[at] * jm[s * np + k], b = gmax[at] * jx[s * np + k];
        o[k] += absval ? fabs(a) + fabs(b) : a + b;
      }
    }
  }
  return 0;
}

int or_grad(int model, int H, int W, int nb, const double* params, const double* gmin,
            const double* gmax, double* grad, int absval) {
  if (check_grid(model, H, W, nb)) return 1;
  int64_t n = (int64_t)H * W;
  int np = n_param(model, nb);
  double* tmp = (double*)malloc(sizeof(double) * n * np);
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * n);
  if (!tmp || !idx) {
    free(tmp);
    free(idx);
    return 2;
  }
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  int rc = or_grad_at(model, H, W, nb, params, gmin, gmax, n, idx, tmp, absval);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < np; ++k) grad[k * n + i] = tmp[i * np + k];
  free(tmp);
  free(idx);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* fitting per-vertex models from ensemble members (Sec. 5.1, 5.2, 5.3)      */
/* ------------------------------------------------------------------------ */
/*
 * members: [M][H][W] doubles.  single != 0 means the field is FP32: the
 * members are FP32 values, and every decision that floating point makes
 * (the widening of a degenerate range, the histogram bin of a member) is
 * taken in FP32 arithmetic, as the device does.  Statistics are FP64.
 *
 *  uniform       lo = min, hi = max                         (Sec. 5.1, 5.2)
 *  Epanechnikov  m = mean, w = bw * std(ddof) * M^(-1/5)     (Sec. 5.2: range
 *                from sample mean and standard deviation)
 *  histogram     lo = min, hi = max, nb equal-width bins, mass = count / M;
 *                member in bin floor((x - lo) / (hi - lo) * nb), the maximum
 *                in the last bin                             (Sec. 4.4)
 *  degenerate    (all members equal) lo/hi = x -/+ eps * max(1, |x|);
 *                Epanechnikov w = eps * max(1, |m|)
 */
int or_fit(int model, int single, const double* members, int M, int H, int W, int nb, int ddof,
           double bw, double eps, double* params) {
  if (H < 1 || W < 1 || M < 1) return 1;
  if (model < OR_UNIFORM || model > OR_GAUSSIAN || model == OR_MVG) return 1;
  if (model == OR_HISTOGRAM && (nb < 1 || nb > MAXNB)) return 1;
  int64_t n = (int64_t)H * W;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double mn = members[i], mx = members[i], sum = 0.0;
    for (int k = 0; k < M; ++k) {
      double xk = members[(int64_t)k * n + i];
      if (xk < mn) mn = xk;
      if (xk > mx) mx = xk;
      sum += xk;
    }
    double lo = mn, hi = mx;
    if (mn == mx) {
      if (single) {
        float e = (float)eps * fmaxf(1.0f, fabsf((float)mn));
        lo = (double)((float)mn - e);
        hi = (double)((float)mn + e);
      } else {
        double e = eps * fmax(1.0, fabs(mn));
        lo = mn - e;
        hi = mn + e;
      }
    }
    if (model == OR_UNIFORM) {
      params[i] = lo;
      params[n + i] = hi;
    } else if (model == OR_EPANECHNIKOV || model == OR_GAUSSIAN) {
      /* Epanechnikov half-width bw * sd * M^(-1/5); Gaussian sigma = sd */
      double mean = sum / (double)M, ss = 0.0;
      for (int k = 0; k < M; ++k) {
        double dk = members[(int64_t)k * n + i] - mean;
        ss += dk * dk;
      }
      double w;
      if (mn == mx) {
        w = eps * fmax(1.0, fabs(mean));
      } else {
        double sd = sqrt(ss / (double)(M - ddof));
        w = model == OR_GAUSSIAN ? sd : bw * sd * pow((double)M, -0.2);
      }
      params[i] = mean;
      params[n + i] = w;
    } else {
      params[i] = lo;
      params[n + i] = hi;
      int cnt[MAXNB];
      for (int j = 0; j < nb; ++j) cnt[j] = 0;
      for (int k = 0; k < M; ++k) {
        double xk = members[(int64_t)k * n + i];
        int j;
        if (single) {
          float d = (float)xk - (float)lo;
          float r = (float)hi - (float)lo;
          float t = d / r;
          float yb = t * (float)nb;
          j = (int)yb;
        } else {
          double t = (xk - lo) / (hi - lo);
          j = (int)(t * (double)nb);
        }
        if (j > nb - 1) j = nb - 1;
        if (j < 0) j = 0;
        cnt[j]++;
      }
      for (int j = 0; j < nb; ++j) params[(int64_t)(2 + j) * n + i] = (double)cnt[j] / (double)M;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* multivariate Gaussian over the stencil, Monte Carlo                         */
/* ------------------------------------------------------------------------ */
/*
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key; ten
 * rounds; each round multiplies counter words 0 and 2 by two fixed odd
 * constants, keeps high and low halves of the 64-bit products, xors the high
 * halves with the other two counter words and the key, and permutes; the key
 * is advanced by two Weyl constants between rounds.
 */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 24 high bits of a 32-bit word, centred in (0, 1): exact in FP64 */
static double u24(uint32_t r) { return ((double)(r >> 8) + 0.5) * (1.0 / 16777216.0); }

static double phi_cdf(double r) { return 0.5 * erfc(-r / sqrt(2.0)); }
static double phi_pdf(double r) { return exp(-0.5 * r * r) / sqrt(2.0 * M_PI); }

/* stencil variable order for the Gaussian model: e, n, w, s, v */
static const int MVG_SLOT[5] = {1, 2, 3, 4, 0}; /* variable -> stencil slot */
static int tri(int i, int j) { return i * (i + 1) / 2 + j; }

/*
 * Fit: mean plane; per vertex the 5x5 covariance of (e, n, w, s, v) across
 * members (ddof), plus jitter on the diagonal; FP64 Cholesky.  An absent
 * neighbour gets an identity row/column, which leaves the factor of the
 * present variables equal to the factor of their own covariance.
 * members [M][H][W]; params [16][H][W].  Returns 3 if a matrix is not
 * positive definite.
 */
int or_mvg_fit(const double* members, int M, int H, int W, int ddof, double jitter, double* params) {
  if (H < 1 || W < 1 || M < 2 || M - ddof < 1) return 1;
  int64_t n = (int64_t)H * W;
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = 0; k < M; ++k) s += members[(int64_t)k * n + i];
    params[i] = s / (double)M;
  }
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    int y = (int)(i / W), x = (int)(i % W);
    int64_t at[5];
    int present[5];
    double mu[5];
    for (int a = 0; a < 5; ++a) {
      int s = MVG_SLOT[a];
      int yy = y + SLOT_DY[s], xx = x + SLOT_DX[s];
      present[a] = !(yy < 0 || yy >= H || xx < 0 || xx >= W);
      at[a] = present[a] ? (int64_t)yy * W + xx : 0;
      mu[a] = 0.0;
      if (present[a]) {
        double sm = 0.0;
        for (int k = 0; k < M; ++k) sm += members[(int64_t)k * n + at[a]];
        mu[a] = sm / (double)M;
      }
    }
    double C[5][5];
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b) {
        if (!present[a] || !present[b]) {
          C[a][b] = (a == b) ? 1.0 : 0.0;
          continue;
        }
        double acc = 0.0;
        for (int k = 0; k < M; ++k)
          acc += (members[(int64_t)k * n + at[a]] - mu[a]) * (members[(int64_t)k * n + at[b]] - mu[b]);
        C[a][b] = acc / (double)(M - ddof) + (a == b ? jitter : 0.0);
      }
    double L[5][5];
    memset(L, 0, sizeof(L));
    for (int r = 0; r < 5; ++r) {
      for (int c = 0; c <= r; ++c) {
        double acc = C[r][c];
        for (int k = 0; k < c; ++k) acc -= L[r][k] * L[c][k];
        if (r == c) {
          if (!(acc > 0.0)) {
            bad |= 1;
            acc = 1.0;
          }
          L[r][c] = sqrt(acc);
        } else {
          L[r][c] = acc / L[c][c];
        }
      }
    }
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c <= r; ++c) params[(int64_t)(1 + tri(r, c)) * n + i] = L[r][c];
  }
  return bad ? 3 : 0;
}

typedef struct {
  double hit_min, hit_max, rb_min, rb_max;
  int amb_min, amb_max;
  double dmu_min[NSLOT], dmu_max[NSLOT]; /* by stencil slot */
  double dl_min[15], dl_max[15];
  /* near-tie slack per unit upstream gradient (see mvg_vertex) */
  double tmu_min[NSLOT], tmu_max[NSLOT], tl_min[15], tl_max[15];
} mvg_out_t;

/*
 * One vertex.  Sample i uses Philox counters (i, vertex id, field_id, 0) and
 * (i, vertex id, field_id, 1) under key (seed lo, seed hi).  Words of the
 * first block give the uniform pairs (u0,u1), (u2,u3); the first two words of
 * the second block give (u4,u5).  Box-Muller: z_2k = sqrt(-2 ln u_2k)
 * cos(2 pi u_2k+1), z_2k+1 = sqrt(-2 ln u_2k) sin(2 pi u_2k+1); z0..z4 drive
 * (e, n, w, s, v): x = mu + L z.
 *
 * Hit count: [x_v < min x_n] (resp. > max).  Conditional estimator: given
 * z0..z3 the vertex value is N(c, L44^2) with c = mu_v + sum_j<4 L4j z_j, so
 * Pr(min) = Phi((min_n x_n - c) / L44), Pr(max) = Phi((c - max_n x_n) / L44).
 * Gradient: pathwise derivative of the conditional estimator.
 * amb_*: samples whose hit decision has a margin below 1e-5 * max row norm of L.
 *
 * Near-tie slack (t*_min, t*_max): the gradient routes each sample's term to
 * the neighbour that attains the minimum (maximum).  A computation in lower
 * precision may pick another neighbour when two neighbour values lie within
 * its rounding of each other; then that sample's term moves between the two
 * neighbours' slots.  For every sample where more than one present neighbour
 * lies within tt = 2^-18 * max_r (|mu_r - mu_v| + sum_c |L_rc z_c|) of the
 * extreme (the operands of the neighbour values, about 64 FP32 units in the
 * last place of their magnitude), the magnitude of the term is added to the
 * slack of every such neighbour's components.  The slack is 0 wherever no
 * such near-tie occurs.
 */
static void mvg_vertex(const double* par, int H, int W, int y, int x, int ns, uint64_t seed,
                       uint32_t field_id, int want_grad, mvg_out_t* o) {
  int64_t n = (int64_t)H * W, at_v = (int64_t)y * W + x;
  double mu[5], L[5][5];
  int present[5];
  for (int a = 0; a < 5; ++a) {
    int s = MVG_SLOT[a];
    int yy = y + SLOT_DY[s], xx = x + SLOT_DX[s];
    present[a] = !(yy < 0 || yy >= H || xx < 0 || xx >= W);
    mu[a] = present[a] ? par[(int64_t)yy * W + xx] : 0.0;
  }
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) L[r][c] = c <= r ? par[(int64_t)(1 + tri(r, c)) * n + at_v] : 0.0;
  double rowmax = 0.0;
  for (int r = 0; r < 5; ++r) {
    if (!present[r]) continue;
    double s2 = 0.0;
    for (int c = 0; c <= r; ++c) s2 += L[r][c] * L[r][c];
    if (sqrt(s2) > rowmax) rowmax = sqrt(s2);
  }
  double tau = 1e-5 * rowmax;
  int nnb = present[0] + present[1] + present[2] + present[3];
  memset(o, 0, sizeof(*o));
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  double L44 = L[4][4];
  for (int i = 0; i < ns; ++i) {
    uint32_t c0[4] = {(uint32_t)i, (uint32_t)at_v, field_id, 0u}, r0[4];
    uint32_t c1[4] = {(uint32_t)i, (uint32_t)at_v, field_id, 1u}, r1[4];
    or_philox4x32_10(c0, key, r0);
    or_philox4x32_10(c1, key, r1);
    double u[6] = {u24(r0[0]), u24(r0[1]), u24(r0[2]), u24(r0[3]), u24(r1[0]), u24(r1[1])};
    double z[6];
    for (int k = 0; k < 3; ++k) {
      double rad = sqrt(-2.0 * log(u[2 * k]));
      z[2 * k] = rad * cos(2.0 * M_PI * u[2 * k + 1]);
      z[2 * k + 1] = rad * sin(2.0 * M_PI * u[2 * k + 1]);
    }
    double xv[5];
    for (int r = 0; r < 5; ++r) {
      double acc = mu[r];
      for (int c = 0; c <= r; ++c) acc += L[r][c] * z[c];
      xv[r] = acc;
    }
    if (nnb == 0) {
      o->hit_min += 1.0;
      o->hit_max += 1.0;
      o->rb_min += 1.0;
      o->rb_max += 1.0;
      continue;
    }
    int amin = -1, amax = -1;
    for (int r = 0; r < 4; ++r) {
      if (!present[r]) continue;
      if (amin < 0 || xv[r] < xv[amin]) amin = r;
      if (amax < 0 || xv[r] > xv[amax]) amax = r;
    }
    double lo = xv[amin], hi = xv[amax];
    double tmag = 0.0;
    for (int r = 0; r < 4; ++r) {
      if (!present[r]) continue;
      double m = fabs(mu[r] - mu[4]);
      for (int c = 0; c <= r; ++c) m += fabs(L[r][c] * z[c]);
      if (m > tmag) tmag = m;
    }
    double tt = 0x1p-18 * tmag;
    int tie_lo = 0, tie_hi = 0;
    for (int r = 0; r < 4; ++r) {
      if (!present[r]) continue;
      tie_lo += xv[r] - lo < tt;
      tie_hi += hi - xv[r] < tt;
    }
    o->hit_min += xv[4] < lo ? 1.0 : 0.0;
    o->hit_max += xv[4] > hi ? 1.0 : 0.0;
    if (fabs(xv[4] - lo) < tau) o->amb_min++;
    if (fabs(xv[4] - hi) < tau) o->amb_max++;
    double cmean = mu[4];
    for (int c = 0; c < 4; ++c) cmean += L[4][c] * z[c];
    double rmin = (lo - cmean) / L44, rmax = (cmean - hi) / L44;
    o->rb_min += phi_cdf(rmin);
    o->rb_max += phi_cdf(rmax);
    if (!want_grad) continue;
    /* d Phi(r) = phi(r) dr;  r_min = (x_amin - c) / L44 */
    double gmin = phi_pdf(rmin) / L44, gmax = phi_pdf(rmax) / L44;
    o->dmu_min[MVG_SLOT[amin]] += gmin;
    o->dmu_min[0] -= gmin;
    for (int c = 0; c <= amin; ++c) o->dl_min[tri(amin, c)] += gmin * z[c];
    for (int c = 0; c < 4; ++c) o->dl_min[tri(4, c)] -= gmin * z[c];
    o->dl_min[tri(4, 4)] -= gmin * rmin;
    /* r_max = (c - x_amax) / L44 */
    o->dmu_max[0] += gmax;
    o->dmu_max[MVG_SLOT[amax]] -= gmax;
    for (int c = 0; c < 4; ++c) o->dl_max[tri(4, c)] += gmax * z[c];
    for (int c = 0; c <= amax; ++c) o->dl_max[tri(amax, c)] -= gmax * z[c];
    o->dl_max[tri(4, 4)] -= gmax * rmax;
    for (int r = 0; r < 4; ++r) {
      if (!present[r]) continue;
      if (tie_lo > 1 && xv[r] - lo < tt) {
        o->tmu_min[MVG_SLOT[r]] += gmin;
        for (int c = 0; c <= r; ++c) o->tl_min[tri(r, c)] += gmin * fabs(z[c]);
      }
      if (tie_hi > 1 && hi - xv[r] < tt) {
        o->tmu_max[MVG_SLOT[r]] += gmax;
        for (int c = 0; c <= r; ++c) o->tl_max[tri(r, c)] += gmax * fabs(z[c]);
      }
    }
  }
  double inv = 1.0 / (double)ns;
  o->hit_min *= inv;
  o->hit_max *= inv;
  o->rb_min *= inv;
  o->rb_max *= inv;
  for (int k = 0; k < NSLOT; ++k) {
    o->dmu_min[k] *= inv;
    o->dmu_max[k] *= inv;
    o->tmu_min[k] *= inv;
    o->tmu_max[k] *= inv;
  }
  for (int k = 0; k < 15; ++k) {
    o->dl_min[k] *= inv;
    o->dl_max[k] *= inv;
    o->tl_min[k] *= inv;
    o->tl_max[k] *= inv;
  }
}

/* out: [nidx][4] = hit_min, hit_max, rb_min, rb_max; amb: [nidx][2] */
int or_mvg_forward_at(const double* params, int H, int W, int ns, uint64_t seed, uint32_t field_id,
                      int64_t nidx, const int64_t* idx, double* out, int32_t* amb) {
  if (H < 1 || W < 1 || ns < 1) return 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nidx; ++i) {
    mvg_out_t o;
    mvg_vertex(params, H, W, (int)(idx[i] / W), (int)(idx[i] % W), ns, seed, field_id, 0, &o);
    out[4 * i + 0] = o.hit_min;
    out[4 * i + 1] = o.hit_max;
    out[4 * i + 2] = o.rb_min;
    out[4 * i + 3] = o.rb_max;
    amb[2 * i + 0] = o.amb_min;
    amb[2 * i + 1] = o.amb_max;
  }
  return 0;
}

/*
 * Gradient of the conditional estimator: for listed vertices u,
 * out[i][0] = d/dmu(u) gathered over the stencils containing u,
 * out[i][1..15] = d/dL(u) (the factor is local to its stencil).
 * slack (may be NULL): [nidx][16], the near-tie slack of mvg_vertex gathered
 * the same way and weighted by |gmin|, |gmax|.
 */
int or_mvg_grad_at(const double* params, int H, int W, int ns, uint64_t seed, uint32_t field_id,
                   const double* gmin, const double* gmax, int64_t nidx, const int64_t* idx,
                   double* out, double* slack) {
  if (H < 1 || W < 1 || ns < 1) return 1;
#pragma omp parallel for schedule(dynamic, 2)
  for (int64_t i = 0; i < nidx; ++i) {
    int y = (int)(idx[i] / W), x = (int)(idx[i] % W);
    double* o = out + 16 * i;
    double* t = slack ? slack + 16 * i : NULL;
    for (int k = 0; k < 16; ++k) o[k] = 0.0;
    if (t)
      for (int k = 0; k < 16; ++k) t[k] = 0.0;
    for (int s = 0; s < NSLOT; ++s) {
      int vy = y - SLOT_DY[s], vx = x - SLOT_DX[s];
      if (vy < 0 || vy >= H || vx < 0 || vx >= W) continue;
      mvg_out_t r;
      mvg_vertex(params, H, W, vy, vx, ns, seed, field_id, 1, &r);
      int64_t at = (int64_t)vy * W + vx;
      o[0] += gmin[at] * r.dmu_min[s] + gmax[at] * r.dmu_max[s];
      if (s == 0)
        for (int k = 0; k < 15; ++k) o[1 + k] += gmin[at] * r.dl_min[k] + gmax[at] * r.dl_max[k];
      if (!t) continue;
      t[0] += fabs(gmin[at]) * r.tmu_min[s] + fabs(gmax[at]) * r.tmu_max[s];
      if (s == 0)
        for (int k = 0; k < 15; ++k) t[1 + k] += fabs(gmin[at]) * r.tl_min[k] + fabs(gmax[at]) * r.tl_max[k];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* independent Gaussian model                                                 */
/* ------------------------------------------------------------------------ */
/*
 * With X_i ~ N(mu_i, sigma_i^2) independent, the four classification
 * probabilities of an interior vertex are 1-D integrals (Eq. 3, Eq. 4):
 *   P_min = int pdf_v S_e S_n S_w S_s,  P_max = int pdf_v F_e F_n F_w F_s,
 *   t1 = int pdf_v S_e F_n S_w F_s,     t2 = int pdf_v F_e S_n F_w S_s,
 * S = 1 - CDF, F = CDF, evaluated with erfc so that both tails keep full
 * relative precision.  The integrals have no closed form; they are taken over
 * mu_v -/+ 12 sigma_v (the rest of pdf_v weighs < 1e-32), split at
 * mu_i + k sigma_i (k = 0, +-1, +-2, +-4, +-8) of the five distributions, and
 * each piece is refined by bisection until a 20-point and a 40-point
 * Gauss-Legendre rule agree to 1e-16 absolute (plus 1e-14 relative).
 * The Gauss-Legendre nodes are computed here by Newton's method on the
 * Legendre polynomial.  Absent neighbours contribute the factor 1; the
 * saddle terms are 0 unless all four neighbours exist.
 */
#define GQ_MAXN 40
static double gq_x[2][GQ_MAXN], gq_w[2][GQ_MAXN];
static const int gq_n[2] = {20, 40};
static int gq_ready = 0;

static void gq_init(void) {
  for (int r = 0; r < 2; ++r) {
    int n = gq_n[r];
    for (int i = 0; i < n; ++i) {
      double x = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        double dx = p1 / dp;
        x -= dx;
        if (fabs(dx) < 1e-17) break;
      }
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      gq_x[r][i] = x;
      gq_w[r][i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
  }
  gq_ready = 1;
}

typedef struct {
  double mu[NSLOT], sg[NSLOT];
  int pres[NSLOT];
} gstencil_t;

static double g_surv(double x, double mu, double sg) { return 0.5 * erfc((x - mu) / (sg * M_SQRT2)); }
static double g_cdf(double x, double mu, double sg) { return 0.5 * erfc((mu - x) / (sg * M_SQRT2)); }

/* the four integrands at x: out = (min, max, t1, t2) */
static void g_integrands(const gstencil_t* g, double x, double out[4]) {
  double z = (x - g->mu[0]) / g->sg[0];
  double pdf = exp(-0.5 * z * z) / (g->sg[0] * sqrt(2.0 * M_PI));
  double smin = pdf, smax = pdf, a = pdf, b = pdf;
  for (int k = 1; k < NSLOT; ++k) {
    if (!g->pres[k]) continue;
    double S = g_surv(x, g->mu[k], g->sg[k]), F = g_cdf(x, g->mu[k], g->sg[k]);
    smin *= S;
    smax *= F;
    /* slots 1 = e, 2 = n, 3 = w, 4 = s: t1 takes S for e, w and F for n, s */
    a *= (k == 1 || k == 3) ? S : F;
    b *= (k == 1 || k == 3) ? F : S;
  }
  out[0] = smin;
  out[1] = smax;
  out[2] = a;
  out[3] = b;
}

static void g_rule(const gstencil_t* g, int r, double lo, double hi, double out[4]) {
  double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo), f[4];
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int i = 0; i < gq_n[r]; ++i) {
    g_integrands(g, c + h * gq_x[r][i], f);
    for (int q = 0; q < 4; ++q) out[q] += gq_w[r][i] * f[q];
  }
  for (int q = 0; q < 4; ++q) out[q] *= h;
}

static void g_adapt(const gstencil_t* g, double lo, double hi, int depth, double acc[4]) {
  double a[4], b[4];
  g_rule(g, 0, lo, hi, a);
  g_rule(g, 1, lo, hi, b);
  int ok = 1;
  for (int q = 0; q < 4; ++q)
    if (fabs(a[q] - b[q]) > 1e-16 + 1e-14 * fabs(b[q])) ok = 0;
  if (ok || depth >= 50) {
    for (int q = 0; q < 4; ++q) acc[q] += b[q];
    return;
  }
  double m = 0.5 * (lo + hi);
  g_adapt(g, lo, m, depth + 1, acc);
  g_adapt(g, m, hi, depth + 1, acc);
}

static void gauss_load(const grid_t* gr, int y, int x, gstencil_t* g) {
  int64_t plane = (int64_t)gr->H * gr->W;
  for (int s = 0; s < NSLOT; ++s) {
    int yy = y + SLOT_DY[s], xx = x + SLOT_DX[s];
    g->pres[s] = yy >= 0 && yy < gr->H && xx >= 0 && xx < gr->W;
    g->mu[s] = g->sg[s] = 1.0;
    if (g->pres[s]) {
      int64_t at = (int64_t)yy * gr->W + xx;
      g->mu[s] = gr->par[at];
      g->sg[s] = gr->par[plane + at];
    }
  }
}

/* the forward's pieces: mu_v -/+ 12 sigma_v cut at mu_i + k sigma_i */
static int gauss_pieces(const gstencil_t* g, double* bp) {
  const double ks[9] = {-8, -4, -2, -1, 0, 1, 2, 4, 8};
  double lo = g->mu[0] - 12.0 * g->sg[0], hi = g->mu[0] + 12.0 * g->sg[0];
  int nbp = 0;
  bp[nbp++] = lo;
  bp[nbp++] = hi;
  for (int s = 0; s < NSLOT; ++s) {
    if (!g->pres[s]) continue;
    for (int k = 0; k < 9; ++k) {
      double p = g->mu[s] + ks[k] * g->sg[s];
      if (p > lo && p < hi) bp[nbp++] = p;
    }
  }
  qsort(bp, nbp, sizeof(double), cmp_double);
  return nbp;
}

static void gauss_vertex(const grid_t* gr, int y, int x, double out[4]) {
  gstencil_t g;
  gauss_load(gr, y, x, &g);
  double bp[2 + NSLOT * 9];
  int nbp = gauss_pieces(&g, bp);
  double acc[4] = {0, 0, 0, 0};
  for (int i = 0; i + 1 < nbp; ++i)
    if (bp[i + 1] > bp[i]) g_adapt(&g, bp[i], bp[i + 1], 0, acc);
  int interior = g.pres[1] && g.pres[2] && g.pres[3] && g.pres[4];
  out[0] = acc[0];
  out[1] = acc[1];
  out[2] = interior ? acc[2] : 0.0;
  out[3] = interior ? acc[3] : 0.0;
}

/*
 * Jacobian of P_min and P_max of one stencil with respect to (mu, sigma) of
 * its five slots (v, e, n, w, s), by differentiating the integrand:
 *   d pdf_v / d mu_v = pdf_v z_v / sigma_v,
 *   d pdf_v / d sigma_v = pdf_v (z_v^2 - 1) / sigma_v,       z_v = (x - mu_v)/sigma_v
 *   d S_k / d mu_k = pdf_k(x),  d S_k / d sigma_k = pdf_k(x) z_k,  d F_k = -d S_k,
 * and integrating each derivative of the product over the same pieces as the
 * forward.  A piece is accepted when the 20- and 40-point rules agree to
 * 1e-13 of (piece length x the largest magnitude of the integrand on it)
 * plus 1e-15 of (piece length x the largest magnitude over the whole range):
 * the vertex-slot integrands change sign (pdf_v (z_v^2 - 1) vanishes at
 * mu_v -/+ sigma_v, where it is known only to a rounding noise set by the
 * integrand's overall size), so neither their own value nor their local
 * size is a scale there; plus 1e-30 for far-tail pieces that underflow.
 */
#define GJ_N (2 * NSLOT * 2) /* (min, max) x slot x (mu, sigma) */

static void gj_integrands(const gstencil_t* g, double x, double out[GJ_N]) {
  double zv = (x - g->mu[0]) / g->sg[0];
  double pdf = exp(-0.5 * zv * zv) / (g->sg[0] * sqrt(2.0 * M_PI));
  double S[NSLOT], F[NSLOT], dS[NSLOT][2];
  for (int k = 1; k < NSLOT; ++k) {
    S[k] = F[k] = 1.0;
    dS[k][0] = dS[k][1] = 0.0;
    if (!g->pres[k]) continue;
    double zk = (x - g->mu[k]) / g->sg[k];
    double pk = exp(-0.5 * zk * zk) / (g->sg[k] * sqrt(2.0 * M_PI));
    S[k] = g_surv(x, g->mu[k], g->sg[k]);
    F[k] = g_cdf(x, g->mu[k], g->sg[k]);
    dS[k][0] = pk;
    dS[k][1] = pk * zk;
  }
  double PS = 1.0, PF = 1.0;
  for (int k = 1; k < NSLOT; ++k) {
    PS *= S[k];
    PF *= F[k];
  }
  /* slot 0: derivatives of the vertex density */
  double dv[2] = {pdf * zv / g->sg[0], pdf * (zv * zv - 1.0) / g->sg[0]};
  for (int q = 0; q < 2; ++q) {
    out[0 * NSLOT * 2 + 0 * 2 + q] = dv[q] * PS;
    out[1 * NSLOT * 2 + 0 * 2 + q] = dv[q] * PF;
  }
  for (int k = 1; k < NSLOT; ++k) {
    double ls = pdf, lf = pdf;
    for (int j = 1; j < NSLOT; ++j)
      if (j != k) {
        ls *= S[j];
        lf *= F[j];
      }
    for (int q = 0; q < 2; ++q) {
      out[0 * NSLOT * 2 + k * 2 + q] = ls * dS[k][q];
      out[1 * NSLOT * 2 + k * 2 + q] = -lf * dS[k][q];
    }
  }
}

/* out: the rule's value; mag: 2h max |f| over its nodes; absout: the rule
 * applied to |f| */
static void gj_rule(const gstencil_t* g, int r, double lo, double hi, double out[GJ_N], double mag[GJ_N],
                    double absout[GJ_N]) {
  double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo), f[GJ_N];
  for (int q = 0; q < GJ_N; ++q) out[q] = mag[q] = absout[q] = 0.0;
  for (int i = 0; i < gq_n[r]; ++i) {
    gj_integrands(g, c + h * gq_x[r][i], f);
    for (int q = 0; q < GJ_N; ++q) {
      out[q] += gq_w[r][i] * f[q];
      absout[q] += gq_w[r][i] * fabs(f[q]);
      mag[q] = fmax(mag[q], fabs(f[q]));
    }
  }
  for (int q = 0; q < GJ_N; ++q) {
    out[q] *= h;
    absout[q] *= h;
    mag[q] *= 2.0 * h;
  }
}

/* fs: the largest magnitude of each integrand over the stencil's range;
 * acc += the integrals, aacc += the integrals of the magnitudes (over the
 * pieces the integrals accept) */
static void gj_adapt(const gstencil_t* g, double lo, double hi, int depth, const double fs[GJ_N],
                     double acc[GJ_N], double aacc[GJ_N]) {
  double a[GJ_N], b[GJ_N], ma[GJ_N], mb[GJ_N], aa[GJ_N], ab[GJ_N];
  gj_rule(g, 0, lo, hi, a, ma, aa);
  gj_rule(g, 1, lo, hi, b, mb, ab);
  int ok = 1;
  for (int q = 0; q < GJ_N; ++q)
    if (fabs(a[q] - b[q]) > 1e-30 + 1e-13 * fmax(ma[q], mb[q]) + 1e-15 * (hi - lo) * fs[q]) ok = 0;
  if (ok || depth >= 30) {
    for (int q = 0; q < GJ_N; ++q) {
      acc[q] += b[q];
      aacc[q] += ab[q];
    }
    return;
  }
  double m = 0.5 * (lo + hi);
  gj_adapt(g, lo, m, depth + 1, fs, acc, aacc);
  gj_adapt(g, m, hi, depth + 1, fs, acc, aacc);
}

/* jm, jx: [NSLOT][2] derivatives of P_min, P_max; absent slots 0.
 * absval != 0: the integrals of the integrands' magnitudes instead, the
 * scale against which rounding in any quadrature of them is measured (the
 * vertex-slot integrands change sign, so their integral can be far smaller) */
static void gauss_jac_vertex(const grid_t* gr, int y, int x, double jm[NSLOT * 2], double jx[NSLOT * 2],
                             int absval) {
  gstencil_t g;
  gauss_load(gr, y, x, &g);
  double bp[2 + NSLOT * 9];
  int nbp = gauss_pieces(&g, bp);
  double acc[GJ_N], aacc[GJ_N], fs[GJ_N], tmp[GJ_N], mag[GJ_N], atmp[GJ_N];
  for (int q = 0; q < GJ_N; ++q) acc[q] = aacc[q] = fs[q] = 0.0;
  for (int i = 0; i + 1 < nbp; ++i)
    if (bp[i + 1] > bp[i]) {
      gj_rule(&g, 1, bp[i], bp[i + 1], tmp, mag, atmp);
      for (int q = 0; q < GJ_N; ++q) fs[q] = fmax(fs[q], mag[q] / (bp[i + 1] - bp[i]));
    }
  for (int i = 0; i + 1 < nbp; ++i)
    if (bp[i + 1] > bp[i]) gj_adapt(&g, bp[i], bp[i + 1], 0, fs, acc, aacc);
  const double* r = absval ? aacc : acc;
  for (int k = 0; k < NSLOT * 2; ++k) {
    int present = g.pres[k / 2];
    jm[k] = present ? r[k] : 0.0;
    jx[k] = present ? r[NSLOT * 2 + k] : 0.0;
  }
}

/* Jacobians of the stencils centred at idx: [nidx][NSLOT][2] each (absval:
 * the integrals of the integrands' magnitudes) */
int or_gauss_jacobian_at(int H, int W, const double* params, int64_t nidx, const int64_t* idx, double* jmin,
                         double* jmax, int absval) {
  if (H < 1 || W < 1) return 1;
  if (!gq_ready) gq_init();
  grid_t g = {OR_GAUSSIAN, H, W, 0, params};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nidx; ++i)
    gauss_jac_vertex(&g, (int)(idx[i] / W), (int)(idx[i] % W), jmin + i * NSLOT * 2, jmax + i * NSLOT * 2,
                     absval);
  return 0;
}

/* adjoint of the independent Gaussian at idx ([nidx][2]: mu, sigma), as
 * or_grad_at; absval != 0 sums |g| times the integrals of the integrands'
 * magnitudes */
int or_gauss_grad_at(int H, int W, const double* params, const double* gmin, const double* gmax, int64_t nidx,
                     const int64_t* idx, double* out, int absval) {
  if (H < 1 || W < 1) return 1;
  if (!gq_ready) gq_init();
  grid_t g = {OR_GAUSSIAN, H, W, 0, params};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nidx; ++i) {
    int y = (int)(idx[i] / W), x = (int)(idx[i] % W);
    double* o = out + i * 2;
    o[0] = o[1] = 0.0;
    double jm[NSLOT * 2], jx[NSLOT * 2];
    for (int s = 0; s < NSLOT; ++s) {
      int vy = y - SLOT_DY[s], vx = x - SLOT_DX[s];
      if (vy < 0 || vy >= H || vx < 0 || vx >= W) continue;
      gauss_jac_vertex(&g, vy, vx, jm, jx, absval);
      int64_t at = (int64_t)vy * W + vx;
      for (int k = 0; k < 2; ++k) {
        double a = gmin[at] * jm[s * 2 + k], b = gmax[at] * jx[s * 2 + k];
        o[k] += absval ? fabs(a) + fabs(b) : a + b;
      }
    }
  }
  return 0;
}

/* out [nidx][4] = (P_min, P_max, t1, t2) at flat indices idx */
int or_gauss_at(int H, int W, const double* params, int64_t nidx, const int64_t* idx, double* out) {
  if (H < 1 || W < 1) return 1;
  if (!gq_ready) gq_init();
  grid_t g = {OR_GAUSSIAN, H, W, 0, params};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nidx; ++i) gauss_vertex(&g, (int)(idx[i] / W), (int)(idx[i] % W), &out[4 * i]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* semianalytical histogram estimator (Sec. 4.4.2)                            */
/* ------------------------------------------------------------------------ */
/*
 * c samples x_i are drawn from the vertex histogram; for each sample the
 * probabilities that the neighbours lie above / below it are closed-form
 * (bin lookup plus the masses of the later / earlier bins), and their
 * products are averaged:
 *   P_min ~ T (1/c) sum_i prod_n S_n(x_i),   P_max ~ T (1/c) sum_i prod_n F_n(x_i),
 *   t1 ~ T (1/c) sum_i S_e F_n S_w F_s(x_i), t2 likewise with S and F swapped,
 * T = sum of the vertex masses (1 for a normalised histogram; with it the
 * expectation equals the closed-form integral of Eq. 3 / Eq. 4 for
 * unnormalised masses too).
 * Sampling: sample i uses word (i mod 4) of Philox4x32-10 with counter
 * (i / 4, y*W + x, field_id, 2) under key seed, u = ((word >> 8) + 1/2) 2^-24;
 * r = u T; with C_k = m_0 + ... + m_{k-1}, the bin is
 * j = #{k in 1..h-1 : C_k <= r}, the position in it
 * f = (r - C_j) / m_j clamped to [0, 1] (0 when m_j = 0), and
 * x = lo + Delta (j + f): the inverse of the histogram CDF.
 */
static void semi_vertex(const grid_t* g, int y, int x, int ns, uint64_t seed, uint32_t field_id, double out[4]) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  dist_t ds[NSLOT];
  int pres[NSLOT];
  for (int s = 0; s < NSLOT; ++s) {
    int yy = y + SLOT_DY[s], xx = x + SLOT_DX[s];
    pres[s] = yy >= 0 && yy < g->H && xx >= 0 && xx < g->W;
    if (pres[s]) grid_dist(g, yy, xx, &ds[s]);
  }
  const dist_t* v = &ds[0];
  int h = v->nb;
  double C[MAXNB + 1];
  C[0] = 0.0;
  for (int k = 0; k < h; ++k) C[k + 1] = C[k] + d_mass(v, k);
  double T = C[h];
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t at = (uint32_t)((int64_t)y * g->W + x);
  int interior = pres[1] && pres[2] && pres[3] && pres[4];
  double acc[4] = {0, 0, 0, 0};
  uint32_t words[4];
  for (int i = 0; i < ns; ++i) {
    if (i % 4 == 0) {
      uint32_t ctr[4] = {(uint32_t)(i / 4), at, field_id, 2u};
      or_philox4x32_10(ctr, key, words);
    }
    double r = u24(words[i % 4]) * T;
    int j = 0;
    for (int k = 1; k < h; ++k) j += C[k] <= r;
    double mj = d_mass(v, j), f = 0.0;
    if (mj > 0.0) {
      f = (r - C[j]) / mj;
      f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    }
    double xs = v->lo + v->delta * ((double)j + f);
    double pmin = 1.0, pmax = 1.0, a = 1.0, b = 1.0;
    for (int k = 1; k < NSLOT; ++k) {
      if (!pres[k]) continue;
      double S = d_point(&ds[k], K_SURV, xs), F = d_point(&ds[k], K_CDF, xs);
      pmin *= S;
      pmax *= F;
      a *= (k == 1 || k == 3) ? S : F;
      b *= (k == 1 || k == 3) ? F : S;
    }
    acc[0] += pmin;
    acc[1] += pmax;
    acc[2] += a;
    acc[3] += b;
  }
  for (int q = 0; q < 4; ++q) out[q] = ns > 0 ? T * acc[q] / (double)ns : 0.0;
  if (!interior) out[2] = out[3] = 0.0;
}

/* out [nidx][4] = (P_min, P_max, t1, t2) estimates at flat indices idx */
int or_semi_at(int H, int W, int nb, const double* params, int ns, uint64_t seed, uint32_t field_id, int64_t nidx,
               const int64_t* idx, double* out) {
  if (H < 1 || W < 1 || nb < 1 || nb > MAXNB || ns < 0) return 1;
  grid_t g = {OR_HISTOGRAM, H, W, nb, params};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nidx; ++i)
    semi_vertex(&g, (int)(idx[i] / W), (int)(idx[i] % W), ns, seed, field_id, &out[4 * i]);
  return 0;
}

/* the first ns sample positions of vertex (y, x) (for checking the sampler) */
int or_semi_samples(int H, int W, int nb, const double* params, int y, int x, int ns, uint64_t seed,
                    uint32_t field_id, double* xs) {
  if (H < 1 || W < 1 || nb < 1 || nb > MAXNB || ns < 0 || y < 0 || y >= H || x < 0 || x >= W) return 1;
  grid_t g = {OR_HISTOGRAM, H, W, nb, params};
  dist_t v;
  grid_dist(&g, y, x, &v);
  double C[MAXNB + 1];
  C[0] = 0.0;
  for (int k = 0; k < nb; ++k) C[k + 1] = C[k] + d_mass(&v, k);
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t words[4];
  for (int i = 0; i < ns; ++i) {
    if (i % 4 == 0) {
      uint32_t ctr[4] = {(uint32_t)(i / 4), (uint32_t)((int64_t)y * W + x), field_id, 2u};
      or_philox4x32_10(ctr, key, words);
    }
    double r = u24(words[i % 4]) * C[nb];
    int j = 0;
    for (int k = 1; k < nb; ++k) j += C[k] <= r;
    double mj = d_mass(&v, j), f = 0.0;
    if (mj > 0.0) {
      f = (r - C[j]) / mj;
      f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    }
    xs[i] = v.lo + v.delta * ((double)j + f);
  }
  return 0;
}
