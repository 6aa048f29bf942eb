// Exact-interaction math shared by the near-pair setup, the block-Toeplitz
// setup and the near-surface field evaluation (FP64): small vector types, the
// potential integrals of the static kernel over a flat triangle (Wilton et al.
// 1984 / Graglia 1993), the Helmholtz kernel or its smooth remainder, and the
// inner integrals of one half-RWG function at an observation point.
#pragma once
#include <cmath>

#include "device_common.h"
#include "internal.h"

namespace scabs {

struct D3 {
  double x, y, z;
};
__device__ inline D3 d3(const double *p) { return {p[0], p[1], p[2]}; }
__device__ inline D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dotd(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 crossd(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// complex 3-vector helpers
struct Z3 {
  cx<double> x, y, z;
};
__device__ inline Z3 zscale(cx<double> s, D3 v) { return {s * v.x, s * v.y, s * v.z}; }
__device__ inline Z3 zcross(Z3 a, D3 b) {   // a x b
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline Z3 zadd(Z3 a, Z3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline cx<double> zdot(D3 a, Z3 b) {
  cx<double> r = a.x * b.x;
  axpy(r, a.y, b.y);
  axpy(r, a.z, b.z);
  return r;
}

// Potential integrals of 1/R over the flat triangle p0 p1 p2 at r:
// J0 = int 1/R, J1 = int (r' - r)/R, Jg = int grad_r (1/R) (principal value).
__device__ void tri_potentials(D3 r, D3 p0, D3 p1, D3 p2, double &J0, D3 &J1, D3 &Jg) {
  D3 P[3] = {p0, p1, p2};
  D3 nv = crossd(p1 - p0, p2 - p0);
  double twoA = sqrt(dotd(nv, nv));
  D3 n = (1.0 / twoA) * nv;
  double scale = sqrt(0.5 * twoA);
  double hgt = dotd(n, r - p0);
  if (fabs(hgt) < 1e-12 * scale) hgt = 0.0;
  double ah = fabs(hgt);
  double sg = hgt > 0 ? 1.0 : (hgt < 0 ? -1.0 : 0.0);
  D3 rho = r - hgt * n;
  double omega = 0, sum0 = 0;
  D3 glog = {0, 0, 0}, lin = {0, 0, 0};
  for (int i = 0; i < 3; i++) {
    D3 a = P[i], b = P[(i + 1) % 3];
    D3 sv = b - a;
    D3 sh = (1.0 / sqrt(dotd(sv, sv))) * sv;
    D3 m = crossd(sh, n);                    // outward in-plane edge normal
    double lm = dotd(a - rho, sh), lp = dotd(b - rho, sh);
    double t0 = dotd(a - rho, m);
    double r02 = t0 * t0 + hgt * hgt;
    double Rm = sqrt(lm * lm + r02), Rp = sqrt(lp * lp + r02);
    double f;   // int_edge dl / R = ln((Rp + lp)/(Rm + lm)), cancellation-free
    if (lp + lm >= 0) {
      double den = lm >= 0 ? Rm + lm : r02 / (Rm - lm);
      f = log((Rp + lp) / den);
    } else {
      double den = lp <= 0 ? Rp - lp : r02 / (Rp + lp);
      f = log((Rm - lm) / den);
    }
    double beta = 0;
    if (fabs(t0) > 1e-14 * scale) beta = atan(t0 * lp / (r02 + ah * Rp)) - atan(t0 * lm / (r02 + ah * Rm));
    omega += beta;
    sum0 += t0 * f;
    glog = glog + f * m;
    lin = lin + (0.5 * (r02 * f + lp * Rp - lm * Rm)) * m;
  }
  J0 = sum0 - ah * omega;
  Jg = (-1.0) * glog - (sg * omega) * n;
  J1 = lin - (hgt * J0) * n;
}

// G and dG/dR (full kernel) or its smooth remainder G - 1/(4 pi R)
__device__ inline void kernel_val(double k, double R, bool remainder, cx<double> &G, cx<double> &dG) {
  const double c4 = 1.0 / (4.0 * PI);
  if (!remainder) {
    double sn, cs;
    sincos(k * R, &sn, &cs);
    cx<double> e = {cs, -sn};
    G = e * (c4 / R);
    dG = (cx<double>{1.0, k * R} * e) * (-c4 / (R * R));
    return;
  }
  double x = k * R;
  if (x < 1e-3) {
    double k2 = k * k, k3 = k2 * k, k4 = k2 * k2;
    G = cx<double>{-k2 * R / 2 + k4 * R * R * R / 24, -k + k3 * R * R / 6} * c4;
    dG = cx<double>{-k2 / 2 + k4 * R * R / 8, k3 * R / 3} * c4;
  } else {
    double sh = sin(0.5 * x);
    cx<double> em1 = {-2.0 * sh * sh, -sin(x)};            // exp(-jx) - 1
    G = em1 * (c4 / R);
    cx<double> ex = em1 + cx<double>{1.0, 0.0};
    // d/dR [(e^{-jkR} - 1)/R] = (-jkR e^{-jkR} - (e^{-jkR} - 1)) / R^2
    cx<double> num = mul_j(ex) * (-x) - em1;
    dG = num * (c4 / (R * R));
  }
}

// ---------------------------------------------------------------------------
// exact inner integrals of one half-RWG function at an observation point
// (the near-pair, block-Toeplitz and near-surface field paths)
// ---------------------------------------------------------------------------
__device__ inline D3 tri_vertex(const TriD *A, int k, double sx) {
  return {A->v[3 * k] + sx, A->v[3 * k + 1], A->v[3 * k + 2]};
}
__device__ inline D3 tri_point(const TriD *A, int q, double sx) {
  return {A->qp[3 * q] + sx, A->qp[3 * q + 1], A->qp[3 * q + 2]};
}
__device__ inline bool singular_pair(const TriD *A, double sa, const TriD *B, double sb, double kappa) {
  const double dx = A->cen[0] + sa - B->cen[0] - sb, dy = A->cen[1] - B->cen[1], dz = A->cen[2] - B->cen[2];
  const double thr = kappa * (A->rho + B->rho);
  return dx * dx + dy * dy + dz * dz < thr * thr;
}

struct StaticJ {
  double J0;
  D3 J1, Jg;
};

// half function j of the source triangle B (shifted by sb along x), at r, in
// medium k: a = int G f_j, phi = int G div f_j, gphi = int grad G div f_j,
// c = int grad G x f_j.  Singular pairs: static part from st (analytic), 7-point
// rule on the smooth remainder; otherwise the plain rule on G.
struct InnerJ {
  Z3 a, gphi, c;
  cx<double> phi;
};
__device__ inline void inner_j(D3 r, const TriD *B, double sb, int j, bool sing, const StaticJ &st, double k, InnerJ &o) {
  cx<double> S0 = {0, 0};
  Z3 S1 = {{0, 0}, {0, 0}, {0, 0}}, Sg = S1, Sc = S1;
  const D3 vj = tri_vertex(B, j, sb);
  for (int s = 0; s < NQ; s++) {
    const D3 sp = tri_point(B, s, sb);
    const double w = B->qw[s];
    const D3 dv = r - sp;
    const double R = sqrt(dotd(dv, dv));
    cx<double> G = {0, 0}, dG = {0, 0};
    if (R > 0 || sing) kernel_val(k, R, sing, G, dG);
    Z3 gr = {{0, 0}, {0, 0}, {0, 0}};
    if (R > 1e-14) gr = zscale(dG * (1.0 / R), dv);
    S0 += G * w;
    S1 = zadd(S1, zscale(G * w, sp - r));
    const Z3 grw = {gr.x * w, gr.y * w, gr.z * w};
    Sg = zadd(Sg, grw);
    Sc = zadd(Sc, zcross(grw, sp - vj));
  }
  if (sing) {
    const double c4 = 1.0 / (4.0 * PI);
    S0.x += c4 * st.J0;
    S1.x.x += c4 * st.J1.x;
    S1.y.x += c4 * st.J1.y;
    S1.z.x += c4 * st.J1.z;
    Sg.x.x += c4 * st.Jg.x;
    Sg.y.x += c4 * st.Jg.y;
    Sg.z.x += c4 * st.Jg.z;
    const D3 cr = crossd(st.Jg, r - vj);
    Sc.x.x += c4 * cr.x;
    Sc.y.x += c4 * cr.y;
    Sc.z.x += c4 * cr.z;
  }
  const double cf = B->coef[j], dv = 2.0 * cf;
  const D3 rv = r - vj;
  const Z3 a = zadd(S1, zscale(S0, rv));
  o.a = {a.x * cf, a.y * cf, a.z * cf};
  o.phi = S0 * dv;
  o.gphi = {Sg.x * dv, Sg.y * dv, Sg.z * dv};
  o.c = {Sc.x * cf, Sc.y * cf, Sc.z * cf};
}

__device__ inline StaticJ static_of(D3 r, const TriD *B, double sb) {
  StaticJ st;
  tri_potentials(r, tri_vertex(B, 0, sb), tri_vertex(B, 1, sb), tri_vertex(B, 2, sb), st.J0, st.J1, st.Jg);
  return st;
}

}  // namespace scabs
