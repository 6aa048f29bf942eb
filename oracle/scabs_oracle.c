/*
 * Oracle for the surface-conductivity-modified PMCHW system -- plain FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes (paper, Sec. II and Appendix A):
 *  - equivalent currents with exterior normal (eq6-eq9), L-surface reduction
 *    J_e = -J_i = J, M_e = -M_i = M (eq10, eq11), single M on the absorber
 *    (eq12) and the five unknown blocks x = [J^L, M^L, J_e^R, J_i^R, M^R];
 *  - RWG expansion (eqs RWGJ, RWGM) and Galerkin testing (testedLOp,
 *    testedKOp) of the MPIE operators E = -Z L(J) + K(M), H = -K(J) - L(M)/Z
 *    (eq15, eq16, LOp, KOp) with G = exp(-jkR)/(4 pi R);
 *  - rows eq1, eq2 on sigma-free edges and eq3, eq13, eq14 on absorber edges,
 *    with the sigma-weighted tests (testedSigLOp, testedSigKOp) evaluated at
 *    quadrature (target) points as the fast-solver appendix describes;
 *  - right-hand side b = [b_E^L, b_H^L, b_E^R, b_H^R, b_Esigma^R].
 * Readings of the paper used here (testing of eq13 rotated by n x, one-sided
 * limits, R-edge classification, quadrature rule) are listed in the design
 * notes; each function states the one it relies on.
 *
 * Also computes the pieces that define the pFFT approximation of the same
 * operator (Phillips-White precorrected FFT, cited by the paper as prior art):
 * Lagrange stencil weights, grid-kernel blocks for near pairs, and the grid
 * projection / interpolation maps used with an FFT convolution done in numpy.
 */
#include <complex.h>
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

#define PI 3.14159265358979323846
#define NQ 7

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline void sub3(const double *a, const double *b, double *c) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}
static inline double norm3(const double *a) { return sqrt(dot3(a, a)); }
/* complex vector (zc[3]) x real vector */
static inline void zcross_r(const zc *a, const double *b, zc *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
/* real vector x complex vector */
static inline void rcross_z(const double *a, const zc *b, zc *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline zc rdot_z(const double *a, const zc *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------ */
/* seven-point degree-5 triangle rule (Radon; tabulated by Dunavant)   */
/* ------------------------------------------------------------------ */
void or_rule7(double bary[NQ][3], double w[NQ]) {
  const double s15 = sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
  const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
  w[0] = 9.0 / 40.0;
  for (int i = 0; i < 3; i++) {
    for (int k = 0; k < 3; k++) {
      bary[1 + i][k] = (k == i) ? 1.0 - 2.0 * a1 : a1;
      bary[4 + i][k] = (k == i) ? 1.0 - 2.0 * a2 : a2;
    }
    w[1 + i] = w1;
    w[4 + i] = w2;
  }
}

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
  /* mesh (copied) */
  int nv, nt, ne, nbody;
  double *v;       /* nv*3 */
  int *t;          /* nt*3 */
  int *body;       /* nt */
  /* per triangle */
  double *area, *nrm, *cen, *rho; /* rho: largest centroid-vertex distance */
  double *qp, *qw;                /* nt*7*3, nt*7 */
  int *tedge, *tsign;             /* nt*3: edge opposite local vertex k, +1 if the triangle is T+ */
  /* per edge */
  int *ev, *et;                   /* ne*2 */
  double *elen;
  /* media */
  double omega, eps_in, eps_out, mu_in, mu_out;
  double k_e, k_i, Z_e, Z_i;
  double kappa_s;                 /* singular-subtraction radius factor */
  /* sigma at points */
  double *sigma;                  /* nt*7 */
  /* layout */
  int NL, NR, N;
  int *isR;                       /* ne */
  int *eidx;                      /* ne: index within its block */
  char err[256];
  /* grid (pFFT definition) */
  double h;
  int *anchor;                    /* nt*7*3 */
  double *gw;                     /* nt*7*27 value weights */
  double *gd;                     /* nt*7*27*3 gradient weights */
} Ctx;

/* host threads of the OpenMP loops (timing of the oracle on a given core count) */
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int or_get_threads(void) { return omp_get_max_threads(); }

static void set_err(Ctx *c, const char *m) { snprintf(c->err, sizeof c->err, "%s", m); }
const char *or_error(Ctx *c) { return c->err; }

typedef struct { int a, b, tri, k; } EdgeRec;
static int cmp_edge(const void *x, const void *y) {
  const EdgeRec *p = x, *q = y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  if (p->tri != q->tri) return p->tri < q->tri ? -1 : 1;
  return 0;
}

void or_free(Ctx *c) {
  if (!c) return;
  free(c->v); free(c->t); free(c->body); free(c->area); free(c->nrm); free(c->cen); free(c->rho);
  free(c->qp); free(c->qw); free(c->tedge); free(c->tsign); free(c->ev); free(c->et); free(c->elen);
  free(c->sigma); free(c->isR); free(c->eidx); free(c->anchor); free(c->gw); free(c->gd);
  free(c);
}

/* Build triangles, RWG edges (edges sorted by (v_min, v_max), T+ = lower
 * triangle index) and the quadrature points.  Returns NULL with *errout set on
 * a mesh that is not a closed, consistently oriented 2-manifold. */
Ctx *or_create(int nv, const double *v, int nt, const int *t, const int *body,
               double omega, double eps_in, double eps_out, double kappa_s, char *errout) {
  Ctx *c = calloc(1, sizeof(Ctx));
  c->nv = nv; c->nt = nt;
  c->v = malloc(sizeof(double) * 3 * nv); memcpy(c->v, v, sizeof(double) * 3 * nv);
  c->t = malloc(sizeof(int) * 3 * nt); memcpy(c->t, t, sizeof(int) * 3 * nt);
  c->body = malloc(sizeof(int) * nt); memcpy(c->body, body, sizeof(int) * nt);
  c->nbody = 0;
  for (int i = 0; i < nt; i++) if (body[i] + 1 > c->nbody) c->nbody = body[i] + 1;
  c->omega = omega; c->eps_in = eps_in; c->eps_out = eps_out; c->mu_in = 1.0; c->mu_out = 1.0;
  c->k_e = omega * sqrt(eps_out * c->mu_out); c->k_i = omega * sqrt(eps_in * c->mu_in);
  c->Z_e = sqrt(c->mu_out / eps_out); c->Z_i = sqrt(c->mu_in / eps_in);
  c->kappa_s = kappa_s;
  c->area = malloc(sizeof(double) * nt); c->nrm = malloc(sizeof(double) * 3 * nt);
  c->cen = malloc(sizeof(double) * 3 * nt); c->rho = malloc(sizeof(double) * nt);
  c->qp = malloc(sizeof(double) * nt * NQ * 3); c->qw = malloc(sizeof(double) * nt * NQ);
  double bary[NQ][3], wq[NQ];
  or_rule7(bary, wq);
  for (int i = 0; i < nt; i++) {
    const double *p0 = v + 3 * t[3 * i], *p1 = v + 3 * t[3 * i + 1], *p2 = v + 3 * t[3 * i + 2];
    double e1[3], e2[3], n[3];
    sub3(p1, p0, e1); sub3(p2, p0, e2); cross3(e1, e2, n);
    double nn = norm3(n);
    if (!(nn > 0)) { snprintf(errout, 256, "degenerate triangle %d", i); or_free(c); return NULL; }
    c->area[i] = 0.5 * nn;
    for (int k = 0; k < 3; k++) c->nrm[3 * i + k] = n[k] / nn;
    for (int k = 0; k < 3; k++) c->cen[3 * i + k] = (p0[k] + p1[k] + p2[k]) / 3.0;
    double r = 0;
    const double *P[3] = {p0, p1, p2};
    for (int a = 0; a < 3; a++) {
      double d[3]; sub3(P[a], c->cen + 3 * i, d);
      double dn = norm3(d); if (dn > r) r = dn;
    }
    c->rho[i] = r;
    for (int q = 0; q < NQ; q++) {
      for (int k = 0; k < 3; k++)
        c->qp[(i * NQ + q) * 3 + k] = bary[q][0] * p0[k] + bary[q][1] * p1[k] + bary[q][2] * p2[k];
      c->qw[i * NQ + q] = wq[q] * c->area[i];
    }
  }
  /* edges */
  EdgeRec *rec = malloc(sizeof(EdgeRec) * 3 * nt);
  for (int i = 0; i < nt; i++)
    for (int k = 0; k < 3; k++) {
      int a = t[3 * i + (k + 1) % 3], b = t[3 * i + (k + 2) % 3];
      rec[3 * i + k].a = a < b ? a : b; rec[3 * i + k].b = a < b ? b : a;
      rec[3 * i + k].tri = i; rec[3 * i + k].k = k;
    }
  qsort(rec, 3 * nt, sizeof(EdgeRec), cmp_edge);
  if ((3 * nt) % 2) { snprintf(errout, 256, "mesh is not closed"); free(rec); or_free(c); return NULL; }
  c->ne = 3 * nt / 2;
  c->ev = malloc(sizeof(int) * 2 * c->ne); c->et = malloc(sizeof(int) * 2 * c->ne); c->elen = malloc(sizeof(double) * c->ne);
  c->tedge = malloc(sizeof(int) * 3 * nt); c->tsign = malloc(sizeof(int) * 3 * nt);
  for (int e = 0; e < c->ne; e++) {
    EdgeRec *r0 = rec + 2 * e, *r1 = rec + 2 * e + 1;
    if (r0->a != r1->a || r0->b != r1->b || (e + 1 < c->ne && rec[2 * e + 2].a == r0->a && rec[2 * e + 2].b == r0->b) ||
        (e > 0 && rec[2 * e - 1].a == r0->a && rec[2 * e - 1].b == r0->b)) {
      snprintf(errout, 256, "mesh is not a closed 2-manifold near edge (%d,%d)", r0->a, r0->b);
      free(rec); or_free(c); return NULL;
    }
    /* orientation: the edge must run in opposite directions in its two triangles */
    int da = t[3 * r0->tri + (r0->k + 1) % 3], db = t[3 * r1->tri + (r1->k + 1) % 3];
    if (da == db) { snprintf(errout, 256, "inconsistent orientation at edge (%d,%d)", r0->a, r0->b); free(rec); or_free(c); return NULL; }
    c->ev[2 * e] = r0->a; c->ev[2 * e + 1] = r0->b;
    c->et[2 * e] = r0->tri; c->et[2 * e + 1] = r1->tri;   /* r0->tri < r1->tri by sort */
    double d[3]; sub3(v + 3 * r0->b, v + 3 * r0->a, d); c->elen[e] = norm3(d);
    c->tedge[3 * r0->tri + r0->k] = e; c->tsign[3 * r0->tri + r0->k] = +1;
    c->tedge[3 * r1->tri + r1->k] = e; c->tsign[3 * r1->tri + r1->k] = -1;
  }
  free(rec);
  /* outward orientation: signed volume of each body must be positive */
  for (int b = 0; b < c->nbody; b++) {
    double vol = 0;
    for (int i = 0; i < nt; i++) {
      if (body[i] != b) continue;
      const double *p0 = v + 3 * t[3 * i], *p1 = v + 3 * t[3 * i + 1], *p2 = v + 3 * t[3 * i + 2];
      double cr[3]; cross3(p1, p2, cr); vol += dot3(p0, cr) / 6.0;
    }
    if (!(vol > 0)) { snprintf(errout, 256, "body %d is not outward oriented (volume %g)", b, vol); or_free(c); return NULL; }
  }
  c->sigma = calloc(nt * NQ, sizeof(double));
  return c;
}

int or_counts(Ctx *c, int *out) {
  out[0] = c->nv; out[1] = c->nt; out[2] = c->ne; out[3] = c->nbody;
  out[4] = c->N; out[5] = c->NL; out[6] = c->NR;
  return 0;
}
void or_get_points(Ctx *c, double *qp, double *qw, double *nrm) {
  memcpy(qp, c->qp, sizeof(double) * c->nt * NQ * 3);
  memcpy(qw, c->qw, sizeof(double) * c->nt * NQ);
  memcpy(nrm, c->nrm, sizeof(double) * c->nt * 3);
}
void or_get_edges(Ctx *c, int *ev, int *et, double *elen, int *tedge, int *tsign) {
  memcpy(ev, c->ev, sizeof(int) * 2 * c->ne); memcpy(et, c->et, sizeof(int) * 2 * c->ne);
  memcpy(elen, c->elen, sizeof(double) * c->ne);
  memcpy(tedge, c->tedge, sizeof(int) * 3 * c->nt); memcpy(tsign, c->tsign, sizeof(int) * 3 * c->nt);
}

/* ------------------------------------------------------------------ */
/* surface conductivity at quadrature points (Sec. IV, eq60)           */
/* ------------------------------------------------------------------ */
void or_sigma_clear(Ctx *c) { memset(c->sigma, 0, sizeof(double) * c->nt * NQ); }

/* s = dir*(x_axis - x0)/L; u(s) = s^d on [0,1], 0 for s < 0; s > 1 is held at 1. */
static double profile_s(double xa, double x0, double L, int dir) {
  double s = dir * (xa - x0) / L;
  return s;
}
void or_sigma_add_monomial(Ctx *c, int axis, double x0, double L, int dir, int d, double sigma0) {
  for (int i = 0; i < c->nt * NQ; i++) {
    double s = profile_s(c->qp[3 * i + axis], x0, L, dir);
    if (s < 0) continue;
    if (s > 1) s = 1;
    c->sigma[i] += sigma0 * (d == 0 ? 1.0 : pow(s, d));
  }
}
/* piecewise-linear u with n control values at s_k = k/(n-1) (hat basis) */
static double hat(int k, int n, double s) {
  double sk = (double)k / (n - 1), hh = 1.0 / (n - 1);
  double a = fabs(s - sk) / hh;
  return a < 1 ? 1 - a : 0;
}
void or_sigma_add_pwl(Ctx *c, int axis, double x0, double L, int dir, int n, const double *ctrl) {
  for (int i = 0; i < c->nt * NQ; i++) {
    double s = profile_s(c->qp[3 * i + axis], x0, L, dir);
    if (s < 0) continue;
    if (s > 1) s = 1;
    double u = 0;
    for (int k = 0; k < n; k++) u += ctrl[k] * hat(k, n, s);
    c->sigma[i] += u;
  }
}
/* d sigma(q) / d ctrl_k for every point (np x n, row major) */
void or_sigma_pwl_jacobian(Ctx *c, int axis, double x0, double L, int dir, int n, double *J) {
  for (int i = 0; i < c->nt * NQ; i++) {
    double s = profile_s(c->qp[3 * i + axis], x0, L, dir);
    for (int k = 0; k < n; k++) J[(size_t)i * n + k] = 0;
    if (s < 0) continue;
    if (s > 1) s = 1;
    for (int k = 0; k < n; k++) J[(size_t)i * n + k] = hat(k, n, s);
  }
}
void or_sigma_set(Ctx *c, const double *s) { memcpy(c->sigma, s, sizeof(double) * c->nt * NQ); }
void or_sigma_get(Ctx *c, double *s) { memcpy(s, c->sigma, sizeof(double) * c->nt * NQ); }

/* ------------------------------------------------------------------ */
/* unknown layout: an edge is an absorber (R) edge when sigma > 0 at     */
/* some quadrature point of either of its triangles                     */
/* ------------------------------------------------------------------ */
int or_layout(Ctx *c, int force_all_R) {
  free(c->isR); free(c->eidx);
  c->isR = calloc(c->ne, sizeof(int)); c->eidx = malloc(sizeof(int) * c->ne);
  for (int e = 0; e < c->ne; e++) {
    int r = force_all_R;
    for (int s = 0; s < 2 && !r; s++) {
      int T = c->et[2 * e + s];
      for (int q = 0; q < NQ; q++) if (c->sigma[T * NQ + q] > 0) r = 1;
    }
    c->isR[e] = r;
  }
  int nl = 0, nr = 0;
  for (int e = 0; e < c->ne; e++) c->eidx[e] = c->isR[e] ? nr++ : nl++;
  c->NL = nl; c->NR = nr; c->N = 2 * nl + 3 * nr;
  return c->N;
}
void or_get_layout(Ctx *c, int *isR, int *eidx) {
  memcpy(isR, c->isR, sizeof(int) * c->ne); memcpy(eidx, c->eidx, sizeof(int) * c->ne);
}

/* half-RWG function of triangle T, local index k (edge opposite vertex k):
 * f(r) = s * l/(2A) * (r - v_k), div f = s * l / A  (eqs RWGJ/RWGM) */
static void half_rwg(const Ctx *c, int T, int k, const double *r, double *f, double *divf) {
  int e = c->tedge[3 * T + k];
  double s = c->tsign[3 * T + k], l = c->elen[e], A = c->area[T];
  const double *vk = c->v + 3 * c->t[3 * T + k];
  for (int a = 0; a < 3; a++) f[a] = s * l / (2 * A) * (r[a] - vk[a]);
  *divf = s * l / A;
}
void or_point_basis(Ctx *c, double *fv, double *fd) {
  for (int T = 0; T < c->nt; T++)
    for (int q = 0; q < NQ; q++)
      for (int k = 0; k < 3; k++)
        half_rwg(c, T, k, c->qp + 3 * (T * NQ + q), fv + ((T * NQ + q) * 3 + k) * 3, fd + (T * NQ + q) * 3 + k);
}

/* ------------------------------------------------------------------ */
/* static potential integrals over a flat triangle (Wilton et al. 1984, */
/* Graglia 1993):                                                       */
/*   I0 = int 1/R dS',  I1 = int (r'-r)/R dS',  Ig = int grad_r(1/R) dS' */
/* Ig is the principal value (no normal component for an in-plane r).   */
/* ------------------------------------------------------------------ */
void or_static_integrals(const double *r, const double *p0, const double *p1, const double *p2,
                         double *I0, double *I1, double *Ig) {
  const double *P[3] = {p0, p1, p2};
  double e1[3], e2[3], n[3];
  sub3(p1, p0, e1); sub3(p2, p0, e2); cross3(e1, e2, n);
  double nn = norm3(n);
  for (int a = 0; a < 3; a++) n[a] /= nn;
  double scale = sqrt(0.5 * nn);
  double rp[3]; sub3(r, p0, rp);
  double d = dot3(n, rp);
  if (fabs(d) < 1e-12 * scale) d = 0.0;
  double ad = fabs(d), sgn = d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0);
  double rho[3] = {r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2]};
  double sumP0f = 0, sumbeta = 0;
  double gin[3] = {0, 0, 0}, i1in[3] = {0, 0, 0};
  for (int i = 0; i < 3; i++) {
    const double *a = P[i], *b = P[(i + 1) % 3];
    double lv[3]; sub3(b, a, lv);
    double ll = norm3(lv);
    double lh[3] = {lv[0] / ll, lv[1] / ll, lv[2] / ll};
    double m[3]; cross3(lh, n, m);
    double bp[3], ap[3]; sub3(b, rho, bp); sub3(a, rho, ap);
    double lp = dot3(bp, lh), lm = dot3(ap, lh);
    double P0 = dot3(ap, m);
    double R02 = P0 * P0 + d * d;
    double Rp = sqrt(lp * lp + R02), Rm = sqrt(lm * lm + R02);
    double f2;
    if (lp + lm >= 0) {
      double num = Rp + lp;
      double den = lm >= 0 ? Rm + lm : R02 / (Rm - lm);
      f2 = log(num / den);
    } else {
      double num = Rm - lm;
      double den = lp <= 0 ? Rp - lp : R02 / (Rp + lp);
      f2 = log(num / den);
    }
    double beta = 0;
    if (fabs(P0) > 1e-14 * scale)
      beta = atan(P0 * lp / (R02 + ad * Rp)) - atan(P0 * lm / (R02 + ad * Rm));
    sumP0f += P0 * f2;
    sumbeta += beta;
    for (int k = 0; k < 3; k++) {
      gin[k] += m[k] * f2;
      i1in[k] += 0.5 * m[k] * (R02 * f2 + lp * Rp - lm * Rm);
    }
  }
  *I0 = sumP0f - ad * sumbeta;
  for (int k = 0; k < 3; k++) {
    Ig[k] = -gin[k] - sgn * n[k] * sumbeta;
    I1[k] = i1in[k] - d * n[k] * (*I0);
  }
}

/* ------------------------------------------------------------------ */
/* Green's function pieces                                             */
/* ------------------------------------------------------------------ */
/* G = exp(-jkR)/(4 pi R);  dG/dR */
static inline void green(double k, double R, zc *G, zc *dG) {
  zc e = cexp(-I * k * R);
  *G = e / (4 * PI * R);
  *dG = -(1.0 + I * k * R) * e / (4 * PI * R * R);
}
/* remainder Gr = (exp(-jkR) - 1)/(4 pi R) and dGr/dR, smooth at R = 0 */
static inline void green_rem(double k, double R, zc *G, zc *dG) {
  double x = k * R;
  if (x < 1e-3) {
    /* series: (e^{-jx}-1)/R = -jk - k^2 R/2 + j k^3 R^2/6 + k^4 R^3/24 */
    *G = (-I * k - k * k * R / 2 + I * k * k * k * R * R / 6 + k * k * k * k * R * R * R / 24) / (4 * PI);
    *dG = (-k * k / 2 + I * k * k * k * R / 3 + k * k * k * k * R * R / 8) / (4 * PI);
  } else {
    double sh = sin(0.5 * x);
    zc em1 = -2 * sh * sh - I * sin(x);          /* exp(-jx) - 1 */
    *G = em1 / (4 * PI * R);
    *dG = ((-I * x) * (em1 + 1.0) - em1) / (4 * PI * R * R);
  }
}

/* Inner integrals at observation point r over source triangle Tp for its
 * three half-RWG functions f_j:
 *   a_j = int G f_j,  phi_j = int G div f_j,  gphi_j = int grad G div f_j,
 *   c_j = int grad G x f_j   (so K(f_j) = -c_j, curl a_j = c_j).
 * singular != 0: static part analytic (above) plus 7-point quadrature of the
 * smooth remainder; otherwise plain 7-point quadrature of G. */
typedef struct { zc a[3][3], phi[3], gphi[3][3], c[3][3]; } Inner;

static void inner_exact(const Ctx *c, int Tp, const double *r, double k, int singular, Inner *o) {
  memset(o, 0, sizeof(Inner));
  const int *tv = c->t + 3 * Tp;
  double A = c->area[Tp];
  double coef[3], divf[3];
  const double *vj[3];
  for (int j = 0; j < 3; j++) {
    int e = c->tedge[3 * Tp + j];
    coef[j] = c->tsign[3 * Tp + j] * c->elen[e] / (2 * A);
    divf[j] = 2 * coef[j];
    vj[j] = c->v + 3 * tv[j];
  }
  zc S0 = 0, S1[3] = {0, 0, 0}, Sg[3] = {0, 0, 0};   /* int G, int G (r'-r), int grad G */
  zc Sc[3][3];                                       /* int grad G x (r' - v_j) */
  memset(Sc, 0, sizeof Sc);
  if (singular) {
    double I0, I1[3], Ig[3];
    or_static_integrals(r, c->v + 3 * tv[0], c->v + 3 * tv[1], c->v + 3 * tv[2], &I0, I1, Ig);
    S0 = I0 / (4 * PI);
    for (int a = 0; a < 3; a++) { S1[a] = I1[a] / (4 * PI); Sg[a] = Ig[a] / (4 * PI); }
    for (int j = 0; j < 3; j++) {
      double rv[3]; sub3(r, vj[j], rv);
      double cr[3]; cross3(Ig, rv, cr);
      for (int a = 0; a < 3; a++) Sc[j][a] = cr[a] / (4 * PI);
    }
  }
  for (int q = 0; q < NQ; q++) {
    const double *s = c->qp + 3 * (Tp * NQ + q);
    double w = c->qw[Tp * NQ + q];
    double d[3]; sub3(r, s, d);
    double R = norm3(d);
    zc G, dG;
    if (singular) green_rem(k, R, &G, &dG);
    else green(k, R, &G, &dG);
    S0 += w * G;
    for (int a = 0; a < 3; a++) S1[a] += w * G * (s[a] - r[a]);
    if (R > 1e-14) {
      zc g[3];
      for (int a = 0; a < 3; a++) { g[a] = dG * d[a] / R; Sg[a] += w * g[a]; }
      for (int j = 0; j < 3; j++) {
        double sv[3]; sub3(s, vj[j], sv);
        zc cr[3]; zcross_r(g, sv, cr);
        for (int a = 0; a < 3; a++) Sc[j][a] += w * cr[a];
      }
    }
  }
  for (int j = 0; j < 3; j++) {
    double rv[3]; sub3(r, vj[j], rv);
    for (int a = 0; a < 3; a++) {
      o->a[j][a] = coef[j] * (S1[a] + rv[a] * S0);       /* int G (r'-v) = int G (r'-r) + (r-v) int G */
      o->gphi[j][a] = divf[j] * Sg[a];
      o->c[j][a] = coef[j] * Sc[j][a];
    }
    o->phi[j] = divf[j] * S0;
  }
}

int or_singular_pair(const Ctx *c, int T, int Tp) {
  double d[3]; sub3(c->cen + 3 * T, c->cen + 3 * Tp, d);
  double thr = c->kappa_s * (c->rho[T] + c->rho[Tp]);
  return dot3(d, d) < thr * thr;
}

/* ------------------------------------------------------------------ */
/* tested blocks for a (test triangle T, source triangle Tp) pair       */
/* ------------------------------------------------------------------ */
typedef struct {
  zc L[3][3], K[3][3];           /* <g_i, L(f_j)>, <g_i, K(f_j)> (PV)               */
  zc Lrot[3][3], Krot[3][3];     /* sum w sigma (g_i x n).L(f_j)(q), same for K (PV)  */
  zc Lsig[3][3], Ksig[3][3];     /* sum w sigma g_i.L(f_j)(q),      same for K (PV)   */
} Blocks;

static void blocks_from_inner(const Ctx *c, int T, int q, double k, const Inner *in, Blocks *b) {
  const double *t = c->qp + 3 * (T * NQ + q);
  double w = c->qw[T * NQ + q], sg = c->sigma[T * NQ + q];
  const double *n = c->nrm + 3 * T;
  for (int i = 0; i < 3; i++) {
    double g[3], dg, gxn[3];
    half_rwg(c, T, i, t, g, &dg);
    cross3(g, n, gxn);
    for (int j = 0; j < 3; j++) {
      /* L(f_j)(t) = jk [a_j + k^-2 grad phi_j];  K(f_j)(t) = -c_j */
      zc Lv[3], Kv[3];
      for (int a = 0; a < 3; a++) {
        Lv[a] = I * k * (in->a[j][a] + in->gphi[j][a] / (k * k));
        Kv[a] = -in->c[j][a];
      }
      /* tested L by parts on the test side: jk [<g, a> - k^-2 <div g, phi>] */
      b->L[i][j] += w * I * k * (rdot_z(g, in->a[j]) - dg * in->phi[j] / (k * k));
      b->K[i][j] += w * rdot_z(g, Kv);
      if (sg != 0) {
        b->Lrot[i][j] += w * sg * rdot_z(gxn, Lv);
        b->Krot[i][j] += w * sg * rdot_z(gxn, Kv);
        b->Lsig[i][j] += w * sg * rdot_z(g, Lv);
        b->Ksig[i][j] += w * sg * rdot_z(g, Kv);
      }
    }
  }
}

void or_pair_blocks_exact(const Ctx *c, int T, int Tp, double k, Blocks *b) {
  memset(b, 0, sizeof(Blocks));
  int sing = or_singular_pair(c, T, Tp);
  for (int q = 0; q < NQ; q++) {
    Inner in;
    inner_exact(c, Tp, c->qp + 3 * (T * NQ + q), k, sing, &in);
    blocks_from_inner(c, T, q, k, &in, b);
  }
}

/* ------------------------------------------------------------------ */
/* stamping into the unknown/row layout                                */
/* ------------------------------------------------------------------ */
/* sink: dense (row-major N x N) or a triplet list */
typedef struct { zc *dense; int N; int *ri, *ci; zc *val; long cap, cnt; const int *rmap; } Sink;
static inline void sink_add(Sink *s, int r, int col, zc v) {
  if (v == 0) return;
  if (s->rmap) {   /* selected rows only: row r goes to block row rmap[r] */
    if (s->rmap[r] < 0) return;
    r = s->rmap[r];
  }
  if (s->dense) {
    double *p = (double *)&s->dense[(size_t)r * s->N + col];
#pragma omp atomic
    p[0] += creal(v);
#pragma omp atomic
    p[1] += cimag(v);
  } else {
    long i;
#pragma omp atomic capture
    i = s->cnt++;
    if (i < s->cap) { s->ri[i] = r; s->ci[i] = col; s->val[i] = v; }
  }
}
/* unknown / row indices of an edge.
 * cols: L edge -> (J, M) at (idx, NL+idx); R edge -> (Je, Ji, M) at 2NL + (idx, NR+idx, 2NR+idx)
 * rows: L edge -> (eq1, eq2); R edge -> (eq3, eq13, eq14), same offsets. */
static inline void edge_slots(const Ctx *c, int e, int *s0, int *s1, int *s2) {
  int id = c->eidx[e];
  if (!c->isR[e]) { *s0 = id; *s1 = c->NL + id; *s2 = -1; }
  else { int b = 2 * c->NL; *s0 = b + id; *s1 = b + c->NR + id; *s2 = b + 2 * c->NR + id; }
}

/* Stamp the operator blocks of one (T, Tp) pair.  be: exterior medium,
 * bi: interior medium (NULL when T and Tp are on different bodies).
 * Per source edge m: J_e, J_i, M_e = M, M_i = -M; L edges have J_i = -J_e.
 *  E row  : -Z_e L_e J_e + K_e M_e + Z_i L_i J_i - K_i M_i
 *  H row  : -K_e J_e - L_e M_e / Z_e + K_i J_i + L_i M_i / Z_i
 *           (+ on R rows)  sum w sigma (g x n).E_e(q)  = -Z_e Lrot_e J_e + Krot_e M_e
 *  eq14   : - sum w sigma g.E_i(q)(J_i, M_i) = Z_i Lsig_i J_i - Ksig_i M_i   */
static void stamp_pair(const Ctx *c, int T, int Tp, const Blocks *be, const Blocks *bi, double scale, Sink *s) {
  double Ze = c->Z_e, Zi = c->Z_i;
  for (int i = 0; i < 3; i++) {
    int n = c->tedge[3 * T + i];
    int rE, rH, r14; edge_slots(c, n, &rE, &rH, &r14);
    for (int j = 0; j < 3; j++) {
      int m = c->tedge[3 * Tp + j];
      int cA, cB, cC; edge_slots(c, m, &cA, &cB, &cC);
      /* coefficients on J_e, J_i, M */
      zc eJe = -Ze * be->L[i][j], eM = be->K[i][j];
      zc hJe = -be->K[i][j], hM = -be->L[i][j] / Ze;
      zc eJi = 0, hJi = 0;
      if (bi) { eJi = Zi * bi->L[i][j]; eM += bi->K[i][j]; hJi = bi->K[i][j]; hM += -bi->L[i][j] / Zi; }
      zc sJe = 0, sM = 0, tJi = 0, tM = 0;
      if (c->isR[n]) {
        sJe = -Ze * be->Lrot[i][j]; sM = be->Krot[i][j];
        if (bi) { tJi = Zi * bi->Lsig[i][j]; tM = bi->Ksig[i][j]; }   /* -Ksig * M_i = +Ksig * M */
      }
      if (!c->isR[m]) {
        int cJ = cA, cM = cB;   /* J_e = J, J_i = -J */
        sink_add(s, rE, cJ, scale * (eJe - eJi)); sink_add(s, rE, cM, scale * eM);
        sink_add(s, rH, cJ, scale * (hJe - hJi + sJe)); sink_add(s, rH, cM, scale * (hM + sM));
        if (r14 >= 0) { sink_add(s, r14, cJ, scale * (-tJi)); sink_add(s, r14, cM, scale * tM); }
      } else {
        int cJe = cA, cJi = cB, cM = cC;
        sink_add(s, rE, cJe, scale * eJe); sink_add(s, rE, cJi, scale * eJi); sink_add(s, rE, cM, scale * eM);
        sink_add(s, rH, cJe, scale * (hJe + sJe)); sink_add(s, rH, cJi, scale * hJi); sink_add(s, rH, cM, scale * (hM + sM));
        if (r14 >= 0) { sink_add(s, r14, cJi, scale * tJi); sink_add(s, r14, cM, scale * tM); }
      }
    }
  }
}

/* Local (same-triangle, exact for the 7-point rule) terms:
 *  H rows : one-sided limits leave -1/2 <g, n x (J_e + J_i)>
 *  R rows : sigma-rotated residue of E_e^+ (+1/2 n x M):  1/2 sum w sigma (g x n).(n x f) M
 *  eq14   : <g, J_e + J_i>  and  - sum w sigma g.(1/2 n x f) M  (E_i^- carries +1/2 n x M) */
static void stamp_local(const Ctx *c, int T, Sink *s) {
  const double *n = c->nrm + 3 * T;
  for (int i = 0; i < 3; i++) {
    int ne = c->tedge[3 * T + i];
    int rE, rH, r14; edge_slots(c, ne, &rE, &rH, &r14);
    for (int j = 0; j < 3; j++) {
      int m = c->tedge[3 * T + j];
      int cA, cB, cC; edge_slots(c, m, &cA, &cB, &cC);
      double gram = 0, nx = 0, srot = 0, snx = 0;
      for (int q = 0; q < NQ; q++) {
        const double *r = c->qp + 3 * (T * NQ + q);
        double w = c->qw[T * NQ + q], sg = c->sigma[T * NQ + q];
        double g[3], dg, f[3], df, nf[3], gxn[3];
        half_rwg(c, T, i, r, g, &dg); half_rwg(c, T, j, r, f, &df);
        cross3(n, f, nf); cross3(g, n, gxn);
        gram += w * dot3(g, f); nx += w * dot3(g, nf);
        srot += w * sg * dot3(gxn, nf); snx += w * sg * dot3(g, nf);
      }
      if (!c->isR[m]) continue;   /* J_e + J_i = 0 and M terms only on sigma points (R rows) */
      int cJe = cA, cJi = cB, cM = cC;
      sink_add(s, rH, cJe, -0.5 * nx); sink_add(s, rH, cJi, -0.5 * nx);
      if (r14 >= 0) {
        sink_add(s, rH, cM, 0.5 * srot);
        sink_add(s, r14, cJe, gram); sink_add(s, r14, cJi, gram);
        sink_add(s, r14, cM, -0.5 * snx);
      }
    }
    /* sigma residues from L source edges on R rows (M of an L edge is M_e = M) */
    if (r14 >= 0) {
      for (int j = 0; j < 3; j++) {
        int m = c->tedge[3 * T + j];
        if (c->isR[m]) continue;
        int cJ, cM, cX; edge_slots(c, m, &cJ, &cM, &cX);
        double srot = 0, snx = 0;
        for (int q = 0; q < NQ; q++) {
          const double *r = c->qp + 3 * (T * NQ + q);
          double w = c->qw[T * NQ + q], sg = c->sigma[T * NQ + q];
          double g[3], dg, f[3], df, nf[3], gxn[3];
          half_rwg(c, T, i, r, g, &dg); half_rwg(c, T, j, r, f, &df);
          cross3(n, f, nf); cross3(g, n, gxn);
          srot += w * sg * dot3(gxn, nf); snx += w * sg * dot3(g, nf);
        }
        sink_add(s, rH, cM, 0.5 * srot);
        sink_add(s, r14, cM, -0.5 * snx);
      }
    }
  }
}

/* Dense Galerkin matrix A (row-major, N x N), eq19. */
int or_dense(Ctx *c, zc *A) {
  if (!c->isR) { set_err(c, "layout not built"); return -1; }
  memset(A, 0, sizeof(zc) * (size_t)c->N * c->N);
  Sink s = {A, c->N, NULL, NULL, NULL, 0, 0};
#pragma omp parallel for schedule(dynamic, 4)
  for (int T = 0; T < c->nt; T++) {
    for (int Tp = 0; Tp < c->nt; Tp++) {
      Blocks be, bi;
      or_pair_blocks_exact(c, T, Tp, c->k_e, &be);
      int same = c->body[T] == c->body[Tp];
      if (same) or_pair_blocks_exact(c, T, Tp, c->k_i, &bi);
      stamp_pair(c, T, Tp, &be, same ? &bi : NULL, 1.0, &s);
    }
  }
  for (int T = 0; T < c->nt; T++) stamp_local(c, T, &s);
  return 0;
}

/* Selected rows of the dense Galerkin matrix (eq19), assembled exactly as
 * or_dense assembles them but only from the pairs whose test triangle carries
 * one of the rows' edges: out[k][N] = A[rows[k]][:] (row-major, nrows x N). */
int or_dense_rows(Ctx *c, int nrows, const int *rows, zc *out) {
  if (!c->isR) { set_err(c, "layout not built"); return -1; }
  int *rmap = malloc(sizeof(int) * c->N);
  for (int r = 0; r < c->N; r++) rmap[r] = -1;
  for (int k = 0; k < nrows; k++) {
    if (rows[k] < 0 || rows[k] >= c->N) { free(rmap); set_err(c, "row out of range"); return -1; }
    rmap[rows[k]] = k;
  }
  memset(out, 0, sizeof(zc) * (size_t)nrows * c->N);
  Sink s = {out, c->N, NULL, NULL, NULL, 0, 0, rmap};
  /* triangles testing a selected row */
  int *sel = calloc(c->nt, sizeof(int));
  for (int T = 0; T < c->nt; T++)
    for (int i = 0; i < 3; i++) {
      int rE, rH, r14; edge_slots(c, c->tedge[3 * T + i], &rE, &rH, &r14);
      if (rmap[rE] >= 0 || rmap[rH] >= 0 || (r14 >= 0 && rmap[r14] >= 0)) sel[T] = 1;
    }
  for (int T = 0; T < c->nt; T++) {
    if (!sel[T]) continue;
#pragma omp parallel for schedule(dynamic, 64)
    for (int Tp = 0; Tp < c->nt; Tp++) {
      Blocks be, bi;
      or_pair_blocks_exact(c, T, Tp, c->k_e, &be);
      int same = c->body[T] == c->body[Tp];
      if (same) or_pair_blocks_exact(c, T, Tp, c->k_i, &bi);
      stamp_pair(c, T, Tp, &be, same ? &bi : NULL, 1.0, &s);
    }
    stamp_local(c, T, &s);
  }
  free(sel);
  free(rmap);
  return nrows;
}

/* local terms only, as triplets (used by the pFFT operator) */
long or_local_coo(Ctx *c, int *ri, int *ci, zc *val, long cap) {
  Sink s = {NULL, c->N, ri, ci, val, cap, 0};
  for (int T = 0; T < c->nt; T++) stamp_local(c, T, &s);
  return s.cnt;
}

/* ------------------------------------------------------------------ */
/* incident field: electric dipole (current moment p = I l) in medium   */
/* (k, Z) -- the field of a point current in a homogeneous space        */
/* ------------------------------------------------------------------ */
void or_dipole_field(double k, double Z, const double *r0, const zc *p, const double *r, zc *E, zc *H) {
  double d[3]; sub3(r, r0, d);
  double R = norm3(d);
  double u[3] = {d[0] / R, d[1] / R, d[2] / R};
  zc e = cexp(-I * k * R);
  zc G = e / (4 * PI * R);
  zc G1 = -(1.0 + I * k * R) * e / (4 * PI * R * R);                 /* dG/dR */
  zc G2 = (2.0 + 2.0 * I * k * R - k * k * R * R) * e / (4 * PI * R * R * R); /* d2G/dR2 */
  zc up = rdot_z(u, p);
  /* H = curl(p G) = grad G x p;  E = -jkZ [p G + k^-2 grad(div(p G))] */
  zc g[3] = {G1 * u[0], G1 * u[1], G1 * u[2]};
  zc gx[3]; zc pz[3] = {p[0], p[1], p[2]};
  gx[0] = g[1] * pz[2] - g[2] * pz[1];
  gx[1] = g[2] * pz[0] - g[0] * pz[2];
  gx[2] = g[0] * pz[1] - g[1] * pz[0];
  for (int a = 0; a < 3; a++) {
    H[a] = gx[a];
    zc hess_p = G2 * up * u[a] + (G1 / R) * (p[a] - up * u[a]);
    E[a] = -I * k * Z * (p[a] * G + hess_p / (k * k));
  }
}

/* Gaussian beam of Sec. II as a dipole at a complex position (complex source
 * point): the dipole's closed form above with r0 replaced by r0 - j b dir,
 * i.e. d = r - r0 + j bd (bd = b dir), R = sqrt(d.d) on the principal branch
 * (csqrt), u = d / R, and the whole field scaled by exp(-k b).  b = 0 is the
 * point dipole. */
void or_source_field(double k, double Z, const double *r0, const double *bd, double b, const zc *p, const double *r,
                     zc *E, zc *H) {
  if (b == 0.0) { or_dipole_field(k, Z, r0, p, r, E, H); return; }
  zc d[3] = {r[0] - r0[0] + I * bd[0], r[1] - r0[1] + I * bd[1], r[2] - r0[2] + I * bd[2]};
  zc R = csqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  zc u[3] = {d[0] / R, d[1] / R, d[2] / R};
  zc e = cexp(-I * k * R - k * b);
  zc G = e / (4 * PI * R);
  zc G1 = -(1.0 + I * k * R) * e / (4 * PI * R * R);
  zc G2 = (2.0 + 2.0 * I * k * R - k * k * R * R) * e / (4 * PI * R * R * R);
  zc up = u[0] * p[0] + u[1] * p[1] + u[2] * p[2];
  H[0] = G1 * (u[1] * p[2] - u[2] * p[1]);
  H[1] = G1 * (u[2] * p[0] - u[0] * p[2]);
  H[2] = G1 * (u[0] * p[1] - u[1] * p[0]);
  for (int a = 0; a < 3; a++) {
    zc hess_p = G2 * up * u[a] + (G1 / R) * (p[a] - up * u[a]);
    E[a] = -I * k * Z * (p[a] * G + hess_p / (k * k));
  }
}

/* right-hand side of a source (dipole or beam) in the interior of `body` */
int or_rhs_source(Ctx *c, const double *r0, const double *bd, double b, const zc *p, int body, zc *rhs) {
  memset(rhs, 0, sizeof(zc) * c->N);
  for (int T = 0; T < c->nt; T++) {
    if (c->body[T] != body) continue;
    for (int q = 0; q < NQ; q++) {
      const double *r = c->qp + 3 * (T * NQ + q);
      double w = c->qw[T * NQ + q], sg = c->sigma[T * NQ + q];
      zc E[3], H[3];
      or_source_field(c->k_i, c->Z_i, r0, bd, b, p, r, E, H);
      for (int i = 0; i < 3; i++) {
        double g[3], dg; half_rwg(c, T, i, r, g, &dg);
        int n = c->tedge[3 * T + i];
        int rE, rH, r14; edge_slots(c, n, &rE, &rH, &r14);
        rhs[rE] += w * rdot_z(g, E);
        rhs[rH] += w * rdot_z(g, H);
        if (r14 >= 0) rhs[r14] += w * sg * rdot_z(g, E);
      }
    }
  }
  return 0;
}

/* b = [b_E^L, b_H^L, b_E^R, b_H^R, b_Esigma^R]; the incident field exists in
 * the interior medium of body `body` only (Sec. II: fields of the source in a
 * homogeneous space with the interior material). */
int or_rhs_dipole(Ctx *c, const double *r0, const zc *p, int body, zc *b) {
  memset(b, 0, sizeof(zc) * c->N);
  for (int T = 0; T < c->nt; T++) {
    if (c->body[T] != body) continue;
    for (int q = 0; q < NQ; q++) {
      const double *r = c->qp + 3 * (T * NQ + q);
      double w = c->qw[T * NQ + q], sg = c->sigma[T * NQ + q];
      zc E[3], H[3];
      or_dipole_field(c->k_i, c->Z_i, r0, p, r, E, H);
      for (int i = 0; i < 3; i++) {
        double g[3], dg; half_rwg(c, T, i, r, g, &dg);
        int n = c->tedge[3 * T + i];
        int rE, rH, r14; edge_slots(c, n, &rE, &rH, &r14);
        b[rE] += w * rdot_z(g, E);
        b[rH] += w * rdot_z(g, H);
        if (r14 >= 0) b[r14] += w * sg * rdot_z(g, E);
      }
    }
  }
  return 0;
}

/* incident field samples at every quadrature point (np x 3 each) */
void or_incident_at_points(Ctx *c, const double *r0, const zc *p, int body, zc *E, zc *H) {
  for (int T = 0; T < c->nt; T++)
    for (int q = 0; q < NQ; q++) {
      int iq = T * NQ + q;
      if (c->body[T] != body) { for (int a = 0; a < 3; a++) E[3 * iq + a] = H[3 * iq + a] = 0; continue; }
      or_dipole_field(c->k_i, c->Z_i, r0, p, c->qp + 3 * iq, E + 3 * iq, H + 3 * iq);
    }
}

/* per-edge source currents from x: (J_e, J_i, M) */
static void edge_currents(const Ctx *c, const zc *x, zc *Je, zc *Ji, zc *M) {
  for (int e = 0; e < c->ne; e++) {
    int s0, s1, s2; edge_slots(c, e, &s0, &s1, &s2);
    if (!c->isR[e]) { Je[e] = x[s0]; Ji[e] = -x[s0]; M[e] = x[s1]; }
    else { Je[e] = x[s0]; Ji[e] = x[s1]; M[e] = x[s2]; }
  }
}

/* ------------------------------------------------------------------ */
/* pointwise one-sided fields at every quadrature point:                */
/*   E_e^+ = E_e(J_e, M_e) + 1/2 n x M_e  (exterior limit)               */
/*   E_i^- = E_i(J_i, M_i) - 1/2 n x M_i  (interior limit, excl. E_inc)   */
/* with the same inner-integral rules as the dense matrix.               */
/* ------------------------------------------------------------------ */
void or_point_fields(Ctx *c, const zc *x, zc *Ee, zc *Ei) {
  zc *Je = malloc(sizeof(zc) * c->ne), *Ji = malloc(sizeof(zc) * c->ne), *M = malloc(sizeof(zc) * c->ne);
  edge_currents(c, x, Je, Ji, M);
#pragma omp parallel for schedule(dynamic, 4)
  for (int T = 0; T < c->nt; T++) {
    for (int q = 0; q < NQ; q++) {
      int iq = T * NQ + q;
      const double *r = c->qp + 3 * iq;
      zc ee[3] = {0, 0, 0}, ei[3] = {0, 0, 0};
      for (int Tp = 0; Tp < c->nt; Tp++) {
        int sing = or_singular_pair(c, T, Tp);
        int same = c->body[T] == c->body[Tp];
        for (int med = 0; med < (same ? 2 : 1); med++) {
          double k = med ? c->k_i : c->k_e, Z = med ? c->Z_i : c->Z_e;
          Inner in; inner_exact(c, Tp, r, k, sing, &in);
          for (int j = 0; j < 3; j++) {
            int m = c->tedge[3 * Tp + j];
            zc J = med ? Ji[m] : Je[m];
            zc Mm = med ? -M[m] : M[m];
            for (int a = 0; a < 3; a++) {
              zc val = -Z * I * k * (in.a[j][a] + in.gphi[j][a] / (k * k)) * J - in.c[j][a] * Mm;
              if (med) ei[a] += val; else ee[a] += val;
            }
          }
        }
      }
      /* residues from the currents on T itself */
      const double *n = c->nrm + 3 * T;
      zc Mq[3] = {0, 0, 0};
      for (int j = 0; j < 3; j++) {
        double f[3], df; half_rwg(c, T, j, r, f, &df);
        int m = c->tedge[3 * T + j];
        for (int a = 0; a < 3; a++) Mq[a] += f[a] * M[m];
      }
      zc nM[3]; rcross_z(n, Mq, nM);
      for (int a = 0; a < 3; a++) {
        Ee[3 * iq + a] = ee[a] + 0.5 * nM[a];
        Ei[3 * iq + a] = ei[a] + 0.5 * nM[a];   /* -1/2 n x M_i with M_i = -M */
      }
    }
  }
  free(Je); free(Ji); free(M);
}

/* Fields at off-surface points (plain 7-point quadrature; points must be
 * well away from the surface).  region < 0: exterior field of (J_e, M_e) in
 * the exterior medium; region = b: field of body b's interior currents in the
 * interior medium (scattered part, without E_inc). */
void or_fields_at(Ctx *c, const zc *x, int npts, const double *pts, int region, zc *E, zc *H) {
  zc *Je = malloc(sizeof(zc) * c->ne), *Ji = malloc(sizeof(zc) * c->ne), *M = malloc(sizeof(zc) * c->ne);
  edge_currents(c, x, Je, Ji, M);
  double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
#pragma omp parallel for
  for (int p = 0; p < npts; p++) {
    const double *r = pts + 3 * p;
    zc e[3] = {0, 0, 0}, hh[3] = {0, 0, 0};
    for (int T = 0; T < c->nt; T++) {
      if (region >= 0 && c->body[T] != region) continue;
      for (int q = 0; q < NQ; q++) {
        const double *s = c->qp + 3 * (T * NQ + q);
        double w = c->qw[T * NQ + q];
        zc Jq[3] = {0, 0, 0}, Mq[3] = {0, 0, 0}, rJ = 0, rM = 0;
        for (int j = 0; j < 3; j++) {
          double f[3], df; half_rwg(c, T, j, s, f, &df);
          int m = c->tedge[3 * T + j];
          zc J = region < 0 ? Je[m] : Ji[m], Mm = region < 0 ? M[m] : -M[m];
          for (int a = 0; a < 3; a++) { Jq[a] += f[a] * J; Mq[a] += f[a] * Mm; }
          rJ += df * J; rM += df * Mm;
        }
        double d[3]; sub3(r, s, d);
        double R = norm3(d);
        zc G, dG; green(k, R, &G, &dG);
        zc g[3] = {dG * d[0] / R, dG * d[1] / R, dG * d[2] / R};
        /* L(X) = jk [int X G + k^-2 int grad G div X];  K(X) = -int grad G x X */
        zc gJ[3], gM[3];
        gJ[0] = g[1] * Jq[2] - g[2] * Jq[1]; gJ[1] = g[2] * Jq[0] - g[0] * Jq[2]; gJ[2] = g[0] * Jq[1] - g[1] * Jq[0];
        gM[0] = g[1] * Mq[2] - g[2] * Mq[1]; gM[1] = g[2] * Mq[0] - g[0] * Mq[2]; gM[2] = g[0] * Mq[1] - g[1] * Mq[0];
        for (int a = 0; a < 3; a++) {
          zc LJ = I * k * (Jq[a] * G + g[a] * rJ / (k * k));
          zc LM = I * k * (Mq[a] * G + g[a] * rM / (k * k));
          e[a] += w * (-Z * LJ - gM[a]);
          hh[a] += w * (gJ[a] - LM / Z);
        }
      }
    }
    for (int a = 0; a < 3; a++) { E[3 * p + a] = e[a]; H[3 * p + a] = hh[a]; }
  }
  free(Je); free(Ji); free(M);
}

/* Fields at points close to the surface as well: per source triangle the
 * inner integrals of inner_exact, with the static part analytic when the
 * point lies within 5 triangle radii of the centroid (the near-field radius
 * of the exact evaluation), the plain rule otherwise. */
void or_fields_at_exact(Ctx *c, const zc *x, int npts, const double *pts, int region, zc *E, zc *H) {
  zc *Je = malloc(sizeof(zc) * c->ne), *Ji = malloc(sizeof(zc) * c->ne), *M = malloc(sizeof(zc) * c->ne);
  edge_currents(c, x, Je, Ji, M);
  double k = region < 0 ? c->k_e : c->k_i, Z = region < 0 ? c->Z_e : c->Z_i;
#pragma omp parallel for schedule(dynamic)
  for (int p = 0; p < npts; p++) {
    const double *r = pts + 3 * p;
    zc e[3] = {0, 0, 0}, hh[3] = {0, 0, 0};
    for (int T = 0; T < c->nt; T++) {
      if (region >= 0 && c->body[T] != region) continue;
      double d[3]; sub3(r, c->cen + 3 * T, d);
      double thr = 5.0 * c->rho[T];
      int near = dot3(d, d) < thr * thr;
      Inner in;
      inner_exact(c, T, r, k, near, &in);
      for (int j = 0; j < 3; j++) {
        int m = c->tedge[3 * T + j];
        zc J = region < 0 ? Je[m] : Ji[m], Mm = region < 0 ? M[m] : -M[m];
        for (int a = 0; a < 3; a++) {
          zc L = I * k * (in.a[j][a] + in.gphi[j][a] / (k * k));   /* L(f_j), K(f_j) = -c_j */
          e[a] += -Z * L * J - in.c[j][a] * Mm;
          hh[a] += in.c[j][a] * J - L * Mm / Z;
        }
      }
    }
    for (int a = 0; a < 3; a++) { E[3 * p + a] = e[a]; H[3 * p + a] = hh[a]; }
  }
  free(Je); free(Ji); free(M);
}

/* ------------------------------------------------------------------ */
/* pFFT definition pieces                                              */
/* lattice nodes at h * (i, j, k); anchor = nearest node; 3-point      */
/* Lagrange weights per axis on offsets -1, 0, +1.                      */
/* ------------------------------------------------------------------ */
static void lagr3(double u, double *L, double *dL) {
  L[0] = 0.5 * u * (u - 1); L[1] = 1 - u * u; L[2] = 0.5 * u * (u + 1);
  dL[0] = u - 0.5; dL[1] = -2 * u; dL[2] = u + 0.5;
}
static void stencil(double h, const double *r, int *anc, double *w, double *gw) {
  double L[3][3], dL[3][3];
  for (int a = 0; a < 3; a++) {
    double x = r[a] / h;
    anc[a] = (int)floor(x + 0.5);
    lagr3(x - anc[a], L[a], dL[a]);
  }
  int idx = 0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++, idx++) {
        w[idx] = L[0][i] * L[1][j] * L[2][k];
        gw[3 * idx + 0] = dL[0][i] * L[1][j] * L[2][k] / h;
        gw[3 * idx + 1] = L[0][i] * dL[1][j] * L[2][k] / h;
        gw[3 * idx + 2] = L[0][i] * L[1][j] * dL[2][k] / h;
      }
}
void or_stencil(double h, const double *r, int *anc, double *w, double *gw) { stencil(h, r, anc, w, gw); }

void or_grid_setup(Ctx *c, double h) {
  c->h = h;
  int np = c->nt * NQ;
  free(c->anchor); free(c->gw); free(c->gd);
  c->anchor = malloc(sizeof(int) * 3 * np); c->gw = malloc(sizeof(double) * 27 * np); c->gd = malloc(sizeof(double) * 81 * np);
  for (int i = 0; i < np; i++) stencil(h, c->qp + 3 * i, c->anchor + 3 * i, c->gw + 27 * i, c->gd + 81 * i);
}
void or_grid_weights(Ctx *c, int *anchor, double *w, double *gd) {
  int np = c->nt * NQ;
  memcpy(anchor, c->anchor, sizeof(int) * 3 * np);
  memcpy(w, c->gw, sizeof(double) * 27 * np);
  memcpy(gd, c->gd, sizeof(double) * 81 * np);
}

/* grid kernel H(offset) = G(h |offset|), H(0) = 0, tabulated over
 * |offset| components 0..D (the kernel depends on them only) */
typedef struct { zc *tab; int D; } HTab;
static HTab make_htab(double k, double h, int D) {
  HTab t; t.D = D; t.tab = malloc(sizeof(zc) * (size_t)(D + 1) * (D + 1) * (D + 1));
  for (int i = 0; i <= D; i++) for (int j = 0; j <= D; j++) for (int l = 0; l <= D; l++) {
    zc v = 0;
    if (i || j || l) {
      double R = h * sqrt((double)(i * i + j * j + l * l));
      v = cexp(-I * k * R) / (4 * PI * R);
    }
    t.tab[((size_t)i * (D + 1) + j) * (D + 1) + l] = v;
  }
  return t;
}
static inline zc htab_at(const HTab *t, int dx, int dy, int dz) {
  dx = abs(dx); dy = abs(dy); dz = abs(dz);
  return t->tab[((size_t)dx * (t->D + 1) + dy) * (t->D + 1) + dz];
}

/* grid-kernel inner "integrals" at test point (T, q) from source triangle Tp:
 *   Ht(t, s) = sum_{g in St(t), g' in St(s)} I_t(g) H(g - g') P_s(g'),
 * gradient via the derivative weights of the test stencil. */
static void inner_grid(const Ctx *c, int T, int q, int Tp, const HTab *ht, Inner *o) {
  memset(o, 0, sizeof(Inner));
  int it = T * NQ + q;
  const int *at = c->anchor + 3 * it;
  const double *wt = c->gw + 27 * it, *gt = c->gd + 81 * it;
  double A = c->area[Tp];
  double coef[3], divf[3];
  const double *vj[3];
  for (int j = 0; j < 3; j++) {
    int e = c->tedge[3 * Tp + j];
    coef[j] = c->tsign[3 * Tp + j] * c->elen[e] / (2 * A);
    divf[j] = 2 * coef[j];
    vj[j] = c->v + 3 * c->t[3 * Tp + j];
  }
  for (int sq = 0; sq < NQ; sq++) {
    int is = Tp * NQ + sq;
    const int *as = c->anchor + 3 * is;
    const double *ws = c->gw + 27 * is;
    const double *s = c->qp + 3 * is;
    double w = c->qw[is];
    zc Ht = 0, gH[3] = {0, 0, 0};
    int ia = 0;
    for (int i1 = -1; i1 <= 1; i1++) for (int j1 = -1; j1 <= 1; j1++) for (int k1 = -1; k1 <= 1; k1++, ia++) {
      zc phi = 0;   /* potential at test node from the projected source point */
      int ib = 0;
      for (int i2 = -1; i2 <= 1; i2++) for (int j2 = -1; j2 <= 1; j2++) for (int k2 = -1; k2 <= 1; k2++, ib++) {
        int dx = at[0] + i1 - as[0] - i2, dy = at[1] + j1 - as[1] - j2, dz = at[2] + k1 - as[2] - k2;
        phi += htab_at(ht, dx, dy, dz) * ws[ib];
      }
      Ht += wt[ia] * phi;
      for (int a = 0; a < 3; a++) gH[a] += gt[3 * ia + a] * phi;
    }
    for (int j = 0; j < 3; j++) {
      double f[3];
      for (int a = 0; a < 3; a++) f[a] = coef[j] * (s[a] - vj[j][a]);
      zc cr[3]; zcross_r(gH, f, cr);
      for (int a = 0; a < 3; a++) {
        o->a[j][a] += w * Ht * f[a];
        o->gphi[j][a] += w * gH[a] * divf[j];
        o->c[j][a] += w * cr[a];
      }
      o->phi[j] += w * Ht * divf[j];
    }
  }
}

static void pair_blocks_grid(const Ctx *c, int T, int Tp, double k, const HTab *ht, Blocks *b) {
  memset(b, 0, sizeof(Blocks));
  for (int q = 0; q < NQ; q++) {
    Inner in;
    inner_grid(c, T, q, Tp, ht, &in);
    blocks_from_inner(c, T, q, k, &in, b);
  }
}

/* near list: triangle pairs with centroid distance < r_near */
long or_near_pairs(Ctx *c, double r_near, int *pairs, long cap) {
  long cnt = 0;
  double r2 = r_near * r_near;
  for (int T = 0; T < c->nt; T++)
    for (int Tp = 0; Tp < c->nt; Tp++) {
      double d[3]; sub3(c->cen + 3 * T, c->cen + 3 * Tp, d);
      if (dot3(d, d) < r2) {
        if (cnt < cap) { pairs[2 * cnt] = T; pairs[2 * cnt + 1] = Tp; }
        cnt++;
      }
    }
  return cnt;
}
/* largest kappa_s * (rho_T + rho_T') over pairs that need singular
 * subtraction -- the near radius must exceed it */
double or_singular_radius(Ctx *c) {
  double m = 0;
  for (int T = 0; T < c->nt; T++)
    for (int Tp = 0; Tp < c->nt; Tp++)
      if (or_singular_pair(c, T, Tp)) {
        double d[3]; sub3(c->cen + 3 * T, c->cen + 3 * Tp, d);
        double dd = sqrt(dot3(d, d));
        if (dd > m) m = dd;
      }
  return m;
}

/* Precorrection (exact - grid) for the listed pairs, stamped as triplets.
 * mode 0: exact - grid; 1: exact only; 2: grid only. */
long or_pair_coo(Ctx *c, const int *pairs, long npairs, int mode, int *ri, int *ci, zc *val, long cap) {
  Sink s = {NULL, c->N, ri, ci, val, cap, 0};
  HTab hte = {NULL, 0}, hti = {NULL, 0};
  if (mode != 1) {
    int D = 0;
    for (long p = 0; p < npairs; p++)
      for (int q1 = 0; q1 < NQ; q1++) for (int q2 = 0; q2 < NQ; q2++)
        for (int a = 0; a < 3; a++) {
          int d = abs(c->anchor[3 * (pairs[2 * p] * NQ + q1) + a] - c->anchor[3 * (pairs[2 * p + 1] * NQ + q2) + a]);
          if (d > D) D = d;
        }
    D += 2;
    hte = make_htab(c->k_e, c->h, D);
    hti = make_htab(c->k_i, c->h, D);
  }
#pragma omp parallel for schedule(dynamic, 8)
  for (long p = 0; p < npairs; p++) {
    int T = pairs[2 * p], Tp = pairs[2 * p + 1];
    int same = c->body[T] == c->body[Tp];
    Blocks be, bi, ge, gi;
    memset(&be, 0, sizeof be); memset(&bi, 0, sizeof bi);
    if (mode != 2) {
      or_pair_blocks_exact(c, T, Tp, c->k_e, &be);
      if (same) or_pair_blocks_exact(c, T, Tp, c->k_i, &bi);
    }
    if (mode != 1) {
      pair_blocks_grid(c, T, Tp, c->k_e, &hte, &ge);
      if (same) pair_blocks_grid(c, T, Tp, c->k_i, &hti, &gi);
      zc *pb = (zc *)&be, *pg = (zc *)&ge, *qb = (zc *)&bi, *qg = (zc *)&gi;
      for (size_t i = 0; i < sizeof(Blocks) / sizeof(zc); i++) {
        pb[i] -= pg[i];
        if (same) qb[i] -= qg[i];
      }
    }
    stamp_pair(c, T, Tp, &be, same ? &bi : NULL, 1.0, &s);
  }
  free(hte.tab); free(hti.tab);
  return s.cnt;
}

/* ------------------------------------------------------------------ */
/* pFFT grid pipeline pieces (the FFT convolution is done by the caller) */
/* ------------------------------------------------------------------ */
/* Projection onto a node box [o, o+n) of the lattice.  which < 0: exterior
 * grid (all triangles, exterior currents J_e, M_e); which = b: interior grid
 * of body b (J_i, M_i).  Q has 8 fields [Jx, Jy, Jz, divJ, Mx, My, Mz, divM],
 * each n0*n1*n2 with the last index fastest; every source carries w_s. */
int or_grid_project(Ctx *c, const zc *x, int which, const int *o, const int *n, zc *Q) {
  zc *Je = malloc(sizeof(zc) * c->ne), *Ji = malloc(sizeof(zc) * c->ne), *M = malloc(sizeof(zc) * c->ne);
  edge_currents(c, x, Je, Ji, M);
  size_t G = (size_t)n[0] * n[1] * n[2];
  memset(Q, 0, sizeof(zc) * 8 * G);
  int bad = 0;
  for (int T = 0; T < c->nt; T++) {
    if (which >= 0 && c->body[T] != which) continue;
    for (int q = 0; q < NQ; q++) {
      int is = T * NQ + q;
      const double *s = c->qp + 3 * is;
      double w = c->qw[is];
      zc src[8] = {0};
      for (int j = 0; j < 3; j++) {
        double f[3], df; half_rwg(c, T, j, s, f, &df);
        int m = c->tedge[3 * T + j];
        zc J = which < 0 ? Je[m] : Ji[m], Mm = which < 0 ? M[m] : -M[m];
        for (int a = 0; a < 3; a++) { src[a] += w * f[a] * J; src[4 + a] += w * f[a] * Mm; }
        src[3] += w * df * J; src[7] += w * df * Mm;
      }
      const int *an = c->anchor + 3 * is;
      const double *ws = c->gw + 27 * is;
      int ib = 0;
      for (int i = -1; i <= 1; i++) for (int j = -1; j <= 1; j++) for (int k = -1; k <= 1; k++, ib++) {
        int gx = an[0] + i - o[0], gy = an[1] + j - o[1], gz = an[2] + k - o[2];
        if (gx < 0 || gy < 0 || gz < 0 || gx >= n[0] || gy >= n[1] || gz >= n[2]) { bad = 1; continue; }
        size_t g = ((size_t)gx * n[1] + gy) * n[2] + gz;
        for (int f = 0; f < 8; f++) Q[f * G + g] += ws[ib] * src[f];
      }
    }
  }
  free(Je); free(Ji); free(M);
  return bad ? -1 : 0;
}

/* Interpolation of grid potentials Phi (8 fields as above, convolved with the
 * grid kernel) at test points of the selected triangles, then the tested
 * rows they produce.  Adds into y (length N):
 *   E rows   +/- [ -Z jk (<g,a_J> - k^-2 <div g, phi_J>) - <g, curl a_M> ]
 *   H rows   +/- [ <g, curl a_J> - (jk/Z)(<g,a_M> - k^-2 <div g, phi_M>) ]
 *   R rows, exterior grid: + sum w sigma (g x n).E(q)
 *   eq14,   interior grid: - sum w sigma g.E(q)
 * sign + for the exterior grid, - for interior grids (E_e - E_i, H_e - H_i). */
int or_grid_interp_rows(Ctx *c, int which, const int *o, const int *n, const zc *Phi, zc *y) {
  double k = which < 0 ? c->k_e : c->k_i, Z = which < 0 ? c->Z_e : c->Z_i;
  double sgn = which < 0 ? 1.0 : -1.0;
  size_t G = (size_t)n[0] * n[1] * n[2];
  for (int T = 0; T < c->nt; T++) {
    if (which >= 0 && c->body[T] != which) continue;
    const double *nr = c->nrm + 3 * T;
    for (int q = 0; q < NQ; q++) {
      int it = T * NQ + q;
      const double *r = c->qp + 3 * it;
      double w = c->qw[it], sg = c->sigma[it];
      const int *an = c->anchor + 3 * it;
      const double *wt = c->gw + 27 * it, *gt = c->gd + 81 * it;
      zc val[8] = {0}, grad[8][3];
      memset(grad, 0, sizeof grad);
      int ib = 0;
      for (int i = -1; i <= 1; i++) for (int j = -1; j <= 1; j++) for (int kk = -1; kk <= 1; kk++, ib++) {
        int gx = an[0] + i - o[0], gy = an[1] + j - o[1], gz = an[2] + kk - o[2];
        if (gx < 0 || gy < 0 || gz < 0 || gx >= n[0] || gy >= n[1] || gz >= n[2]) return -1;
        size_t g = ((size_t)gx * n[1] + gy) * n[2] + gz;
        for (int f = 0; f < 8; f++) {
          zc p = Phi[f * G + g];
          val[f] += wt[ib] * p;
          for (int a = 0; a < 3; a++) grad[f][a] += gt[3 * ib + a] * p;
        }
      }
      zc aJ[3] = {val[0], val[1], val[2]}, aM[3] = {val[4], val[5], val[6]};
      zc phJ = val[3], phM = val[7];
      zc gphJ[3] = {grad[3][0], grad[3][1], grad[3][2]};
      /* curl a = (d_y a_z - d_z a_y, d_z a_x - d_x a_z, d_x a_y - d_y a_x) */
      zc cJ[3] = {grad[2][1] - grad[1][2], grad[0][2] - grad[2][0], grad[1][0] - grad[0][1]};
      zc cM[3] = {grad[6][1] - grad[5][2], grad[4][2] - grad[6][0], grad[5][0] - grad[4][1]};
      /* pointwise field of this medium (no residue) */
      zc Ep[3];
      for (int a = 0; a < 3; a++) Ep[a] = -Z * I * k * (aJ[a] + gphJ[a] / (k * k)) - cM[a];
      for (int i = 0; i < 3; i++) {
        double g[3], dg, gxn[3];
        half_rwg(c, T, i, r, g, &dg);
        cross3(g, nr, gxn);
        int ne = c->tedge[3 * T + i];
        int rE, rH, r14; edge_slots(c, ne, &rE, &rH, &r14);
        zc e = -Z * I * k * (rdot_z(g, aJ) - dg * phJ / (k * k)) - rdot_z(g, cM);
        zc hh = rdot_z(g, cJ) - (I * k / Z) * (rdot_z(g, aM) - dg * phM / (k * k));
        y[rE] += sgn * w * e;
        y[rH] += sgn * w * hh;
        if (r14 >= 0) {
          if (which < 0) y[rH] += w * sg * rdot_z(gxn, Ep);
          else y[r14] += -w * sg * rdot_z(g, Ep);
        }
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Transposed pFFT pieces (adjoint system A~^T l = g) and pointwise    */
/* one-sided fields of the pFFT operator (sigma derivative of A~ x).   */
/* ------------------------------------------------------------------ */

/* Transpose of or_grid_interp_rows.  Every tested quantity there is linear
 * in the grid potentials through the value weights W (a_J, phi_J, a_M, phi_M)
 * or the derivative weights grad W (curl a_J, curl a_M, grad phi_J).  Given a
 * row-space vector z, Src gets, per field, W times the coefficient of that
 * field's value plus grad W dotted with the coefficient of its gradient, so
 * that sum_f <Src_f, Phi_f> = z^T (rows added for Phi).  The coefficient of
 * grad A_c inside v . curl A is e_c x v. */
int or_grid_interp_rows_t(Ctx *c, int which, const int *o, const int *n, const zc *z, zc *Src) {
  double k = which < 0 ? c->k_e : c->k_i, Z = which < 0 ? c->Z_e : c->Z_i;
  double sgn = which < 0 ? 1.0 : -1.0;
  zc jk = I * k;
  size_t G = (size_t)n[0] * n[1] * n[2];
  memset(Src, 0, sizeof(zc) * 8 * G);
  for (int T = 0; T < c->nt; T++) {
    if (which >= 0 && c->body[T] != which) continue;
    const double *nr = c->nrm + 3 * T;
    for (int q = 0; q < NQ; q++) {
      int it = T * NQ + q;
      const double *r = c->qp + 3 * it;
      double w = c->qw[it], sg = c->sigma[it];
      zc tE[3] = {0, 0, 0}, tH[3] = {0, 0, 0}, sv[3] = {0, 0, 0}, dE = 0, dH = 0;
      for (int i = 0; i < 3; i++) {
        double g[3], dg, gxn[3];
        half_rwg(c, T, i, r, g, &dg);
        cross3(g, nr, gxn);
        int rE, rH, r14; edge_slots(c, c->tedge[3 * T + i], &rE, &rH, &r14);
        for (int a = 0; a < 3; a++) { tE[a] += z[rE] * g[a]; tH[a] += z[rH] * g[a]; }
        dE += z[rE] * dg; dH += z[rH] * dg;
        if (r14 >= 0) {
          for (int a = 0; a < 3; a++) {
            if (which < 0) sv[a] += w * sg * z[rH] * gxn[a];
            else sv[a] += -w * sg * z[r14] * g[a];
          }
        }
      }
      zc cv[8], gc[8][3], vJ[3], vM[3], gp[3];
      for (int a = 0; a < 3; a++) {
        cv[a] = -Z * jk * (sgn * w * tE[a] + sv[a]);
        cv[4 + a] = -(jk / Z) * sgn * w * tH[a];
        vJ[a] = sgn * w * tH[a];
        vM[a] = -(sgn * w * tE[a] + sv[a]);
        gp[a] = -Z * jk * sv[a] / (k * k);
      }
      cv[3] = sgn * w * Z * jk * dE / (k * k);
      cv[7] = (jk / Z) * sgn * w * dH / (k * k);
      const zc *vv[2] = {vJ, vM};
      for (int s = 0; s < 2; s++) {
        const zc *v = vv[s];
        int b = 4 * s;
        gc[b + 0][0] = 0;     gc[b + 0][1] = -v[2]; gc[b + 0][2] = v[1];
        gc[b + 1][0] = v[2];  gc[b + 1][1] = 0;     gc[b + 1][2] = -v[0];
        gc[b + 2][0] = -v[1]; gc[b + 2][1] = v[0];  gc[b + 2][2] = 0;
      }
      for (int a = 0; a < 3; a++) { gc[3][a] = gp[a]; gc[7][a] = 0; }
      const int *an = c->anchor + 3 * it;
      const double *wt = c->gw + 27 * it, *gt = c->gd + 81 * it;
      int ib = 0;
      for (int i = -1; i <= 1; i++) for (int j = -1; j <= 1; j++) for (int kk = -1; kk <= 1; kk++, ib++) {
        int gx = an[0] + i - o[0], gy = an[1] + j - o[1], gz = an[2] + kk - o[2];
        if (gx < 0 || gy < 0 || gz < 0 || gx >= n[0] || gy >= n[1] || gz >= n[2]) return -1;
        size_t gi = ((size_t)gx * n[1] + gy) * n[2] + gz;
        for (int f = 0; f < 8; f++)
          Src[f * G + gi] += wt[ib] * cv[f] + gt[3 * ib] * gc[f][0] + gt[3 * ib + 1] * gc[f][1] + gt[3 * ib + 2] * gc[f][2];
      }
    }
  }
  return 0;
}

/* transpose of edge_currents: adjoint currents per edge -> unknown space (adds) */
static void edge_currents_t(const Ctx *c, const zc *aJe, const zc *aJi, const zc *aM, zc *y) {
  for (int e = 0; e < c->ne; e++) {
    int s0, s1, s2; edge_slots(c, e, &s0, &s1, &s2);
    if (!c->isR[e]) { y[s0] += aJe[e] - aJi[e]; y[s1] += aM[e]; }
    else { y[s0] += aJe[e]; y[s1] += aJi[e]; y[s2] += aM[e]; }
  }
}

/* Transpose of or_grid_project: node values Phi (8 fields) -> unknown space
 * (adds into y).  Each source point reads Phi with its value weights and
 * hands w_s (f . Phi_vec + div f Phi_scalar) back to its half-RWG currents. */
int or_grid_project_t(Ctx *c, int which, const int *o, const int *n, const zc *Phi, zc *y) {
  zc *aJe = calloc(c->ne, sizeof(zc)), *aJi = calloc(c->ne, sizeof(zc)), *aM = calloc(c->ne, sizeof(zc));
  size_t G = (size_t)n[0] * n[1] * n[2];
  int bad = 0;
  for (int T = 0; T < c->nt && !bad; T++) {
    if (which >= 0 && c->body[T] != which) continue;
    for (int q = 0; q < NQ; q++) {
      int is = T * NQ + q;
      const double *s = c->qp + 3 * is;
      double w = c->qw[is];
      const int *an = c->anchor + 3 * is;
      const double *ws = c->gw + 27 * is;
      zc P[8] = {0};
      int ib = 0;
      for (int i = -1; i <= 1; i++) for (int j = -1; j <= 1; j++) for (int k = -1; k <= 1; k++, ib++) {
        int gx = an[0] + i - o[0], gy = an[1] + j - o[1], gz = an[2] + k - o[2];
        if (gx < 0 || gy < 0 || gz < 0 || gx >= n[0] || gy >= n[1] || gz >= n[2]) { bad = 1; continue; }
        size_t g = ((size_t)gx * n[1] + gy) * n[2] + gz;
        for (int f = 0; f < 8; f++) P[f] += ws[ib] * Phi[f * G + g];
      }
      for (int j = 0; j < 3; j++) {
        double f[3], df; half_rwg(c, T, j, s, f, &df);
        int m = c->tedge[3 * T + j];
        zc aj = w * (f[0] * P[0] + f[1] * P[1] + f[2] * P[2] + df * P[3]);
        zc am = w * (f[0] * P[4] + f[1] * P[5] + f[2] * P[6] + df * P[7]);
        if (which < 0) { aJe[m] += aj; aM[m] += am; }
        else { aJi[m] += aj; aM[m] -= am; }
      }
    }
  }
  edge_currents_t(c, aJe, aJi, aM, y);
  free(aJe); free(aJi); free(aM);
  return bad ? -1 : 0;
}

/* Pointwise field of one medium's grid potentials at the selected test points
 * (no residue): E = -Z jk (a_J + k^-2 grad phi_J) - curl a_M, added into Ep. */
int or_grid_point_fields(Ctx *c, int which, const int *o, const int *n, const zc *Phi, zc *Ep) {
  double k = which < 0 ? c->k_e : c->k_i, Z = which < 0 ? c->Z_e : c->Z_i;
  size_t G = (size_t)n[0] * n[1] * n[2];
  for (int T = 0; T < c->nt; T++) {
    if (which >= 0 && c->body[T] != which) continue;
    for (int q = 0; q < NQ; q++) {
      int it = T * NQ + q;
      const int *an = c->anchor + 3 * it;
      const double *wt = c->gw + 27 * it, *gt = c->gd + 81 * it;
      zc val[8] = {0}, grad[8][3];
      memset(grad, 0, sizeof grad);
      int ib = 0;
      for (int i = -1; i <= 1; i++) for (int j = -1; j <= 1; j++) for (int kk = -1; kk <= 1; kk++, ib++) {
        int gx = an[0] + i - o[0], gy = an[1] + j - o[1], gz = an[2] + kk - o[2];
        if (gx < 0 || gy < 0 || gz < 0 || gx >= n[0] || gy >= n[1] || gz >= n[2]) return -1;
        size_t g = ((size_t)gx * n[1] + gy) * n[2] + gz;
        for (int f = 0; f < 8; f++) {
          zc p = Phi[f * G + g];
          val[f] += wt[ib] * p;
          for (int a = 0; a < 3; a++) grad[f][a] += gt[3 * ib + a] * p;
        }
      }
      zc cM[3] = {grad[6][1] - grad[5][2], grad[4][2] - grad[6][0], grad[5][0] - grad[4][1]};
      for (int a = 0; a < 3; a++)
        Ep[3 * it + a] += -Z * I * k * (val[a] + grad[3][a] / (k * k)) - cM[a];
    }
  }
  return 0;
}

/* Near-pair correction of the pointwise fields: for every listed pair
 * (T, T') and test point of T, (exact - grid) field of the currents of T'
 * (exterior medium always, interior medium when both lie on one body) added
 * into Ee / Ei.  Pairs must be grouped by test triangle. */
int or_point_near_corr(Ctx *c, const zc *x, const int *pairs, long npairs, zc *Ee, zc *Ei) {
  for (long p = 1; p < npairs; p++) if (pairs[2 * p] < pairs[2 * (p - 1)]) return -1;
  zc *Je = malloc(sizeof(zc) * c->ne), *Ji = malloc(sizeof(zc) * c->ne), *M = malloc(sizeof(zc) * c->ne);
  edge_currents(c, x, Je, Ji, M);
  int D = 0;
  for (long p = 0; p < npairs; p++)
    for (int q1 = 0; q1 < NQ; q1++) for (int q2 = 0; q2 < NQ; q2++)
      for (int a = 0; a < 3; a++) {
        int d = abs(c->anchor[3 * (pairs[2 * p] * NQ + q1) + a] - c->anchor[3 * (pairs[2 * p + 1] * NQ + q2) + a]);
        if (d > D) D = d;
      }
  D += 2;
  HTab hte = make_htab(c->k_e, c->h, D), hti = make_htab(c->k_i, c->h, D);
  long *start = malloc(sizeof(long) * (c->nt + 1));
  for (int T = 0; T <= c->nt; T++) start[T] = 0;
  for (long p = 0; p < npairs; p++) start[pairs[2 * p] + 1]++;
  for (int T = 0; T < c->nt; T++) start[T + 1] += start[T];
#pragma omp parallel for schedule(dynamic, 4)
  for (int T = 0; T < c->nt; T++) {
    for (long p = start[T]; p < start[T + 1]; p++) {
      int Tp = pairs[2 * p + 1];
      int sing = or_singular_pair(c, T, Tp);
      int same = c->body[T] == c->body[Tp];
      for (int q = 0; q < NQ; q++) {
        int iq = T * NQ + q;
        const double *r = c->qp + 3 * iq;
        for (int med = 0; med < (same ? 2 : 1); med++) {
          double k = med ? c->k_i : c->k_e, Z = med ? c->Z_i : c->Z_e;
          Inner ex, gr;
          inner_exact(c, Tp, r, k, sing, &ex);
          inner_grid(c, T, q, Tp, med ? &hti : &hte, &gr);
          for (int j = 0; j < 3; j++) {
            int m = c->tedge[3 * Tp + j];
            zc J = med ? Ji[m] : Je[m], Mm = med ? -M[m] : M[m];
            for (int a = 0; a < 3; a++) {
              zc da = ex.a[j][a] - gr.a[j][a], dg = ex.gphi[j][a] - gr.gphi[j][a], dc = ex.c[j][a] - gr.c[j][a];
              zc val = -Z * I * k * (da + dg / (k * k)) * J - dc * Mm;
              if (med) Ei[3 * iq + a] += val; else Ee[3 * iq + a] += val;
            }
          }
        }
      }
    }
  }
  free(start); free(hte.tab); free(hti.tab);
  free(Je); free(Ji); free(M);
  return 0;
}
