// Field post-processing along and across a guide (host arithmetic on field
// samples the GPU evaluates): the standing-wave ratio and reflection
// coefficient on the axis (Sec. I, Table I), the standing-wave fit, the
// exponential decay fit of the field in an absorber (Sec. III) and the
// pieces of the Poynting decay-rate formula (Sec. III, eq_alpha_power):
// Gauss-Legendre rules and the surface currents at points of the surface.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace scabs {

typedef std::complex<double> zd;

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's iteration on P_n
// from the Chebyshev-like first guesses cos(pi (i + 3/4) / (n + 1/2))
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; i++) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;   // P_0, P_1
      for (int k = 2; k <= n; k++) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);   // P_n'
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// triangle of `body` containing the surface point r (within tol of its plane
// and inside up to tol), or -1
int locate_surface_point(const Geometry &g, const double *r, int body, double tol) {
  int best = -1;
  double bestd = 1e300;
  for (int T = 0; T < g.nt; T++) {
    if (body >= 0 && g.body[T] != body) continue;
    const double *n = g.nrm.data() + 3 * T;
    const double *a = g.v.data() + 3 * g.t[3 * T];
    const double h = (r[0] - a[0]) * n[0] + (r[1] - a[1]) * n[1] + (r[2] - a[2]) * n[2];
    if (std::fabs(h) > tol) continue;
    // barycentric coordinates of the projection
    const double *b = g.v.data() + 3 * g.t[3 * T + 1], *c = g.v.data() + 3 * g.t[3 * T + 2];
    double lam[3];
    const double *P[3] = {a, b, c};
    bool inside = true;
    double out = 0;
    for (int k = 0; k < 3; k++) {
      const double *p1 = P[(k + 1) % 3], *p2 = P[(k + 2) % 3];
      const double u[3] = {p1[0] - r[0], p1[1] - r[1], p1[2] - r[2]}, v[3] = {p2[0] - r[0], p2[1] - r[1], p2[2] - r[2]};
      const double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
      lam[k] = 0.5 * (cr[0] * n[0] + cr[1] * n[1] + cr[2] * n[2]) / g.area[T];
      if (lam[k] < -tol / std::sqrt(g.area[T])) inside = false;
      out = std::max(out, -lam[k]);
    }
    if (inside && out < bestd) {
      bestd = out;
      best = T;
    }
  }
  return best;
}

// surface currents (J on the side of region: exterior J_e, interior J_i;
// and M = E x n) at a point r of triangle T from the unknowns x (host)
void surface_currents_at(const Geometry &g, const Layout &L, const double *x, int T, const double *r, bool interior,
                         zd J[3], zd M[3]) {
  for (int a = 0; a < 3; a++) J[a] = M[a] = 0.0;
  for (int k = 0; k < 3; k++) {
    const int e = g.tedge[3 * T + k];
    const double cf = g.tsign[3 * T + k] * g.elen[e] / (2.0 * g.area[T]);
    const double *v = g.v.data() + 3 * g.t[3 * T + k];
    const int id = L.eidx[e];
    zd Jv, Mv;
    if (!L.isR[e]) {
      Jv = zd(x[2 * id], x[2 * id + 1]);
      if (interior) Jv = -Jv;
      Mv = zd(x[2 * (L.NL + id)], x[2 * (L.NL + id) + 1]);
    } else {
      const int b0 = 2 * L.NL;
      const int s = interior ? b0 + L.NR + id : b0 + id;
      Jv = zd(x[2 * s], x[2 * s + 1]);
      Mv = zd(x[2 * (b0 + 2 * L.NR + id)], x[2 * (b0 + 2 * L.NR + id) + 1]);
    }
    for (int a = 0; a < 3; a++) {
      const double f = cf * (r[a] - v[a]);
      J[a] += f * Jv;
      M[a] += f * Mv;
    }
  }
}

}  // namespace scabs

using scabs::zd;

extern "C" {

int scabs_swr(const double *E, int n, double out[2]) {
  if (!E || !out || n < 2) return SCABS_E_ARG;
  double mx = 0, mn = 1e300;
  for (int i = 0; i < n; i++) {
    const double a = std::hypot(E[2 * i], E[2 * i + 1]);
    mx = std::max(mx, a);
    mn = std::min(mn, a);
  }
  if (!(mn > 0)) return SCABS_E_ARG;
  out[0] = mx / mn;
  out[1] = (out[0] - 1.0) / (out[0] + 1.0);
  return SCABS_OK;
}

// least-squares fit of E(x) = a e^{-j beta x} + c e^{+j beta x} at fixed beta:
// 2x2 complex normal equations; returns the relative residual
static double sw_fit(const double *xs, const zd *E, int n, double beta, zd &a, zd &c) {
  zd g11 = 0, g12 = 0, g22 = 0, r1 = 0, r2 = 0;
  for (int i = 0; i < n; i++) {
    const zd f = std::exp(zd(0, -beta * xs[i])), h = std::conj(f);   // forward, backward
    g11 += std::conj(f) * f;
    g12 += std::conj(f) * h;
    g22 += std::conj(h) * h;
    r1 += std::conj(f) * E[i];
    r2 += std::conj(h) * E[i];
  }
  const zd g21 = std::conj(g12), det = g11 * g22 - g12 * g21;
  if (std::abs(det) < 1e-300) {
    a = c = 0;
    return 1.0;
  }
  a = (g22 * r1 - g12 * r2) / det;
  c = (g11 * r2 - g21 * r1) / det;
  double num = 0, den = 0;
  for (int i = 0; i < n; i++) {
    const zd fit = a * std::exp(zd(0, -beta * xs[i])) + c * std::exp(zd(0, beta * xs[i]));
    num += std::norm(E[i] - fit);
    den += std::norm(E[i]);
  }
  return den > 0 ? std::sqrt(num / den) : 1.0;
}

int scabs_standing_wave_fit(const double *xs, const double *E, int n, double beta_lo, double beta_hi,
                            double out[6]) {
  if (!xs || !E || !out || n < 4 || !(beta_lo > 0) || !(beta_hi >= beta_lo)) return SCABS_E_ARG;
  const zd *Ez = reinterpret_cast<const zd *>(E);
  zd a, c;
  double beta = beta_lo;
  if (beta_hi > beta_lo) {
    // scan, then golden-section refinement of the residual around the best
    const int ns = 400;
    double best = 1e300;
    for (int i = 0; i <= ns; i++) {
      const double b = beta_lo + (beta_hi - beta_lo) * i / ns;
      const double r = sw_fit(xs, Ez, n, b, a, c);
      if (r < best) {
        best = r;
        beta = b;
      }
    }
    const double step = (beta_hi - beta_lo) / ns;
    double lo = std::max(beta_lo, beta - step), hi = std::min(beta_hi, beta + step);
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = sw_fit(xs, Ez, n, x1, a, c), f2 = sw_fit(xs, Ez, n, x2, a, c);
    for (int it = 0; it < 80; it++) {
      if (f1 < f2) {
        hi = x2;
        x2 = x1;
        f2 = f1;
        x1 = hi - gr * (hi - lo);
        f1 = sw_fit(xs, Ez, n, x1, a, c);
      } else {
        lo = x1;
        x1 = x2;
        f1 = f2;
        x2 = lo + gr * (hi - lo);
        f2 = sw_fit(xs, Ez, n, x2, a, c);
      }
    }
    beta = 0.5 * (lo + hi);
  }
  const double res = sw_fit(xs, Ez, n, beta, a, c);
  if (!(std::abs(a) > 0)) return SCABS_E_ARG;
  out[0] = beta;
  out[1] = std::abs(c) / std::abs(a);
  out[2] = res;
  out[3] = std::abs(a);
  out[4] = std::abs(c);
  out[5] = std::arg(c / a);
  return SCABS_OK;
}

int scabs_decay_fit(const double *xs, const double *E, int n, double out[4]) {
  if (!xs || !E || !out || n < 3) return SCABS_E_ARG;
  // ln|E| = c0 - alpha x and unwrapped phase = p0 - beta x, least squares
  double sx = 0, sxx = 0, sl = 0, sxl = 0, sp = 0, sxp = 0, prev = 0, turn = 0;
  std::vector<double> lg(n), ph(n);
  for (int i = 0; i < n; i++) {
    const double m = std::hypot(E[2 * i], E[2 * i + 1]);
    if (!(m > 0)) return SCABS_E_ARG;
    lg[i] = std::log(m);
    double p = std::atan2(E[2 * i + 1], E[2 * i]);
    if (i > 0) {
      while (p + turn - prev > M_PI) turn -= 2 * M_PI;
      while (p + turn - prev < -M_PI) turn += 2 * M_PI;
    }
    ph[i] = p + turn;
    prev = ph[i];
  }
  for (int i = 0; i < n; i++) {
    sx += xs[i];
    sxx += xs[i] * xs[i];
    sl += lg[i];
    sxl += xs[i] * lg[i];
    sp += ph[i];
    sxp += xs[i] * ph[i];
  }
  const double den = n * sxx - sx * sx;
  if (!(std::fabs(den) > 0)) return SCABS_E_ARG;
  const double sl_ = (n * sxl - sx * sl) / den, sp_ = (n * sxp - sx * sp) / den;
  const double c0 = (sl - sl_ * sx) / n;
  double rr = 0, tt = 0;
  for (int i = 0; i < n; i++) {
    const double f = c0 + sl_ * xs[i];
    rr += (lg[i] - f) * (lg[i] - f);
    tt += lg[i] * lg[i];
  }
  out[0] = -sl_;
  out[1] = -sp_;
  out[2] = tt > 0 ? std::sqrt(rr / tt) : 0.0;
  out[3] = c0;
  return SCABS_OK;
}

}  // extern "C"
