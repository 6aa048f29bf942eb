// Host-side setup: RWG edges, quadrature points, surface conductivity,
// unknown layout, lattice boxes and the near-pair structure.
#include <algorithm>
#include <limits>
#include <array>
#include <cmath>
#include <cstdio>
#include <numeric>

#include "internal.h"

namespace scabs {

namespace {
struct V3 {
  double x, y, z;
};
inline V3 at(const std::vector<double> &a, size_t i) { return {a[3 * i], a[3 * i + 1], a[3 * i + 2]}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// Radon's degree-5 seven-point rule (Dunavant's table): barycentric
// coordinates and weights from their closed forms.
void seven_point_rule(double bary[NQ][3], double wt[NQ]) {
  const double r15 = std::sqrt(15.0);
  const double a[2] = {(6.0 - r15) / 21.0, (6.0 + r15) / 21.0};
  const double w[2] = {(155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0};
  bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
  wt[0] = 9.0 / 40.0;
  for (int g = 0; g < 2; g++)
    for (int p = 0; p < 3; p++) {
      int q = 1 + 3 * g + p;
      for (int c = 0; c < 3; c++) bary[q][c] = (c == p) ? 1.0 - 2.0 * a[g] : a[g];
      wt[q] = w[g];
    }
}
}  // namespace

std::string build_geometry(const std::vector<double> &v, const std::vector<int> &t, const std::vector<int> &body,
                           Geometry &g) {
  g = Geometry();
  g.nv = (int)(v.size() / 3);
  g.nt = (int)(t.size() / 3);
  g.v = v;
  g.t = t;
  g.body = body;
  if (g.nt == 0) return "empty mesh";
  for (int i = 0; i < 3 * g.nt; i++)
    if (t[i] < 0 || t[i] >= g.nv) return "triangle vertex index out of range";
  g.nbody = 0;
  for (int b : body) {
    if (b < 0) return "negative body index";
    g.nbody = std::max(g.nbody, b + 1);
  }
  double bary[NQ][3], wt[NQ];
  seven_point_rule(bary, wt);
  g.area.resize(g.nt);
  g.nrm.resize(3 * g.nt);
  g.cen.resize(3 * g.nt);
  g.rho.resize(g.nt);
  g.qp.resize((size_t)g.nt * NQ * 3);
  g.qw.resize((size_t)g.nt * NQ);
  for (int i = 0; i < g.nt; i++) {
    V3 p[3] = {at(v, t[3 * i]), at(v, t[3 * i + 1]), at(v, t[3 * i + 2])};
    V3 n = cross(p[1] - p[0], p[2] - p[0]);
    double nn = std::sqrt(dot(n, n));
    if (!(nn > 0)) return "degenerate triangle " + std::to_string(i);
    g.area[i] = 0.5 * nn;
    g.nrm[3 * i] = n.x / nn;
    g.nrm[3 * i + 1] = n.y / nn;
    g.nrm[3 * i + 2] = n.z / nn;
    V3 c = {(p[0].x + p[1].x + p[2].x) / 3.0, (p[0].y + p[1].y + p[2].y) / 3.0, (p[0].z + p[1].z + p[2].z) / 3.0};
    g.cen[3 * i] = c.x;
    g.cen[3 * i + 1] = c.y;
    g.cen[3 * i + 2] = c.z;
    double r = 0;
    for (int a = 0; a < 3; a++) r = std::max(r, std::sqrt(dot(p[a] - c, p[a] - c)));
    g.rho[i] = r;
    for (int q = 0; q < NQ; q++) {
      double *o = &g.qp[((size_t)i * NQ + q) * 3];
      o[0] = bary[q][0] * p[0].x + bary[q][1] * p[1].x + bary[q][2] * p[2].x;
      o[1] = bary[q][0] * p[0].y + bary[q][1] * p[1].y + bary[q][2] * p[2].y;
      o[2] = bary[q][0] * p[0].z + bary[q][1] * p[1].z + bary[q][2] * p[2].z;
      g.qw[(size_t)i * NQ + q] = wt[q] * g.area[i];
    }
  }
  // edges: each undirected vertex pair must occur in exactly two triangles,
  // traversed in opposite directions (closed, consistently oriented)
  struct HalfEdge {
    int a, b, tri, k;
  };
  std::vector<HalfEdge> he(3 * (size_t)g.nt);
  for (int i = 0; i < g.nt; i++)
    for (int k = 0; k < 3; k++) {
      int a = t[3 * i + (k + 1) % 3], b = t[3 * i + (k + 2) % 3];
      he[3 * i + k] = {std::min(a, b), std::max(a, b), i, k};
    }
  std::sort(he.begin(), he.end(), [](const HalfEdge &p, const HalfEdge &q) {
    if (p.a != q.a) return p.a < q.a;
    if (p.b != q.b) return p.b < q.b;
    return p.tri < q.tri;
  });
  g.ne = 0;
  g.tedge.assign(3 * g.nt, -1);
  g.tsign.assign(3 * g.nt, 0);
  for (size_t s = 0; s < he.size();) {
    size_t e = s;
    while (e < he.size() && he[e].a == he[s].a && he[e].b == he[s].b) e++;
    if (e - s != 2) {
      char buf[128];
      snprintf(buf, sizeof buf, "edge (%d,%d) is shared by %d triangles (mesh not closed 2-manifold)", he[s].a,
               he[s].b, (int)(e - s));
      return buf;
    }
    const HalfEdge &p = he[s], &q = he[s + 1];
    int dp = t[3 * p.tri + (p.k + 1) % 3], dq = t[3 * q.tri + (q.k + 1) % 3];
    if (dp == dq) return "inconsistent triangle orientation at edge (" + std::to_string(p.a) + "," + std::to_string(p.b) + ")";
    int id = g.ne++;
    g.ev.push_back(p.a);
    g.ev.push_back(p.b);
    g.et.push_back(p.tri);   // lower triangle index: T+
    g.et.push_back(q.tri);
    V3 d = at(v, p.b) - at(v, p.a);
    g.elen.push_back(std::sqrt(dot(d, d)));
    g.tedge[3 * p.tri + p.k] = id;
    g.tsign[3 * p.tri + p.k] = +1;
    g.tedge[3 * q.tri + q.k] = id;
    g.tsign[3 * q.tri + q.k] = -1;
    s = e;
  }
  for (int b = 0; b < g.nbody; b++) {
    double vol = 0;
    for (int i = 0; i < g.nt; i++) {
      if (body[i] != b) continue;
      V3 p0 = at(v, t[3 * i]), p1 = at(v, t[3 * i + 1]), p2 = at(v, t[3 * i + 2]);
      vol += dot(p0, cross(p1, p2)) / 6.0;
    }
    if (!(vol > 0)) return "body " + std::to_string(b) + " is not outward oriented";
  }
  return "";
}

// sigma = sum of sigma0 * u(s) over absorbers (eq60), s = dir (x - x0) / L
// conductivity of one profile end (not a raw end) at coordinate xa along its
// axis: sigma0 s^d or the hat interpolant of the control values, s =
// dir (xa - x0) / L, zero for s < 0 and held at s = 1 beyond the end
static double profile_value(const SigmaEnd &e, double xa) {
  double s = e.dir * (xa - e.x0) / e.length;
  if (s < 0) return 0.0;
  s = std::min(s, 1.0);
  if (e.ctrl.empty()) return e.sigma0 * (e.degree == 0 ? 1.0 : std::pow(s, e.degree));
  int n = (int)e.ctrl.size();
  double step = 1.0 / (n - 1), acc = 0;
  for (int k = 0; k < n; k++) {
    double a = std::fabs(s - (double)k / (n - 1)) / step;
    if (a < 1) acc += e.ctrl[k] * (1 - a);
  }
  return acc;
}

void eval_sigma(const Geometry &g, const std::vector<SigmaEnd> &ends, std::vector<double> &sigma) {
  size_t np = (size_t)g.nt * NQ;
  sigma.assign(np, 0.0);
  for (const SigmaEnd &e : ends) {
    if (!e.pts.empty()) {
      for (size_t i = 0; i < np; i++) sigma[i] += e.pts[i];
      continue;
    }
    for (size_t i = 0; i < np; i++) sigma[i] += profile_value(e, g.qp[3 * i + e.axis]);
  }
}

double sigma_at(const Geometry &g, const std::vector<SigmaEnd> &ends, const double *r, int T) {
  double acc = 0.0;
  for (const SigmaEnd &e : ends) {
    if (e.pts.empty()) {
      acc += profile_value(e, r[e.axis]);
      continue;
    }
    int best = 0;
    double bd = 1e300;
    for (int q = 0; q < NQ; q++) {
      const double *p = g.qp.data() + 3 * ((size_t)T * NQ + q);
      const double d = (p[0] - r[0]) * (p[0] - r[0]) + (p[1] - r[1]) * (p[1] - r[1]) + (p[2] - r[2]) * (p[2] - r[2]);
      if (d < bd) {
        bd = d;
        best = q;
      }
    }
    acc += e.pts[(size_t)T * NQ + best];
  }
  return acc;
}

// d sigma_q / d p per quadrature point (CSR over points): parameters are, end
// by end, sigma0 of a monomial end or the control values of a piecewise-linear
// end, in the order the ends were added
void sigma_param_jacobian(const Geometry &g, const std::vector<SigmaEnd> &ends, std::vector<int64_t> &ptr,
                          std::vector<int> &idx, std::vector<double> &val, int64_t *npar) {
  size_t np = (size_t)g.nt * NQ;
  std::vector<std::vector<std::pair<int, double>>> rows(np);
  int base = 0;
  for (const SigmaEnd &e : ends) {
    if (!e.pts.empty()) {
      for (size_t i = 0; i < np; i++) rows[i].push_back({base + (int)i, 1.0});
      base += (int)np;
      continue;
    }
    const int n = e.ctrl.empty() ? 1 : (int)e.ctrl.size();
    for (size_t i = 0; i < np; i++) {
      double s = e.dir * (g.qp[3 * i + e.axis] - e.x0) / e.length;
      if (s < 0) continue;
      s = std::min(s, 1.0);
      if (e.ctrl.empty()) {
        rows[i].push_back({base, e.degree == 0 ? 1.0 : std::pow(s, e.degree)});
      } else {
        double step = 1.0 / (n - 1);
        for (int k = 0; k < n; k++) {
          double a = std::fabs(s - (double)k / (n - 1)) / step;
          if (a < 1) rows[i].push_back({base + k, 1 - a});
        }
      }
    }
    base += n;
  }
  *npar = base;
  ptr.assign(np + 1, 0);
  idx.clear();
  val.clear();
  for (size_t i = 0; i < np; i++) {
    for (auto &pr : rows[i]) {
      idx.push_back(pr.first);
      val.push_back(pr.second);
    }
    ptr[i + 1] = (int64_t)idx.size();
  }
}

void build_layout(const Geometry &g, Layout &L) {
  L.isR.assign(g.ne, 0);
  L.eidx.assign(g.ne, 0);
  for (int e = 0; e < g.ne; e++)
    for (int s = 0; s < 2; s++) {
      int T = g.et[2 * e + s];
      for (int q = 0; q < NQ; q++)
        if (L.sigma[(size_t)T * NQ + q] > 0) L.isR[e] = 1;
    }
  L.NL = L.NR = 0;
  for (int e = 0; e < g.ne; e++) L.eidx[e] = L.isR[e] ? L.NR++ : L.NL++;
  L.N = 2 * L.NL + 3 * L.NR;
}

// smallest 2^a or 3 * 2^a >= 2n - 1 (sizes the mixed-radix FFT handles)
static int fft_size(int n) {
  int need = std::max(2 * n - 1, 2), best = 1 << 30;
  for (int m = 1; m < (1 << 30); m *= 2) {
    if (m >= need) best = std::min(best, m);
    if (3 * m >= need) best = std::min(best, 3 * m);
    if (m >= need) break;
  }
  return best;
}

std::string build_grids(const Geometry &g, double h, double k_e, double k_i, std::vector<GridDesc> &grids,
                        std::vector<int> &anchor, std::vector<double> &u) {
  size_t np = (size_t)g.nt * NQ;
  anchor.resize(3 * np);
  u.resize(3 * np);
  for (size_t i = 0; i < np; i++)
    for (int a = 0; a < 3; a++) {
      double xh = g.qp[3 * i + a] / h;
      int an = (int)std::floor(xh + 0.5);
      anchor[3 * i + a] = an;
      u[3 * i + a] = xh - an;
    }
  grids.clear();
  for (int which = -1; which < g.nbody; which++) {
    GridDesc d;
    d.which = which;
    d.k = which < 0 ? k_e : k_i;
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (int T = 0; T < g.nt; T++) {
      if (which >= 0 && g.body[T] != which) continue;
      for (int q = 0; q < NQ; q++)
        for (int a = 0; a < 3; a++) {
          int an = anchor[3 * ((size_t)T * NQ + q) + a];
          lo[a] = std::min(lo[a], an);
          hi[a] = std::max(hi[a], an);
        }
    }
    for (int a = 0; a < 3; a++) {
      d.o[a] = lo[a] - 1;
      d.n[a] = hi[a] - lo[a] + 3;
      d.N[a] = fft_size(d.n[a]);
    }
    if (d.n[0] >= (1 << 14) || d.n[1] >= (1 << 9) || d.n[2] >= (1 << 9))
      return "grid too large for the anchor packing (x < 16384, y,z < 512 nodes)";
    if (d.n[1] * d.n[2] > 1024) return "grid cross-section too large for the projection tile (n_y n_z <= 1024)";
    if (d.N[0] > 4096 || d.N[1] * d.N[2] > 4096)
      return "FFT sizes beyond the supported range (N_x <= 4096, N_y N_z <= 4096)";
    grids.push_back(d);
  }
  return "";
}

std::string build_near(const Geometry &g, double r_near, double kappa_s, NearList &nl) {
  int nt = g.nt;
  double rho_max = *std::max_element(g.rho.begin(), g.rho.end());
  double search = std::max(r_near, 2.0 * kappa_s * rho_max) * (1.0 + 1e-9);
  // bin centroids into cubic cells of side `search`
  double lo[3] = {1e300, 1e300, 1e300};
  for (int i = 0; i < nt; i++)
    for (int a = 0; a < 3; a++) lo[a] = std::min(lo[a], g.cen[3 * i + a]);
  auto cell_of = [&](int i, int *c) {
    for (int a = 0; a < 3; a++) c[a] = (int)std::floor((g.cen[3 * i + a] - lo[a]) / search);
  };
  int nc[3] = {0, 0, 0};
  std::vector<int> cell(3 * nt);
  for (int i = 0; i < nt; i++) {
    cell_of(i, &cell[3 * i]);
    for (int a = 0; a < 3; a++) nc[a] = std::max(nc[a], cell[3 * i + a] + 1);
  }
  auto cid = [&](int x, int y, int z) { return ((int64_t)x * nc[1] + y) * nc[2] + z; };
  std::vector<int> order(nt);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int64_t> key(nt);
  for (int i = 0; i < nt; i++) key[i] = cid(cell[3 * i], cell[3 * i + 1], cell[3 * i + 2]);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] != key[b] ? key[a] < key[b] : a < b; });
  std::vector<int64_t> skey(nt);
  for (int i = 0; i < nt; i++) skey[i] = key[order[i]];
  const double r2 = r_near * r_near;
  std::vector<std::vector<int>> lists(nt);
  std::vector<std::vector<uint8_t>> sflags(nt);
  int bad = -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int T = 0; T < nt; T++) {
    std::vector<int> &L = lists[T];
    std::vector<uint8_t> &S = sflags[T];
    const int *c = &cell[3 * T];
    for (int dx = -1; dx <= 1; dx++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dz = -1; dz <= 1; dz++) {
          int x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= nc[0] || y >= nc[1] || z >= nc[2]) continue;
          int64_t k = cid(x, y, z);
          auto it = std::lower_bound(skey.begin(), skey.end(), k);
          for (size_t s = it - skey.begin(); s < (size_t)nt && skey[s] == k; s++) {
            int Tp = order[s];
            double ddx = g.cen[3 * T] - g.cen[3 * Tp], ddy = g.cen[3 * T + 1] - g.cen[3 * Tp + 1],
                   ddz = g.cen[3 * T + 2] - g.cen[3 * Tp + 2];
            double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            double thr = kappa_s * (g.rho[T] + g.rho[Tp]);
            bool sing = d2 < thr * thr;
            if (d2 < r2) {
              L.push_back(Tp);
              S.push_back(sing ? 1 : 0);
            } else if (sing) {
#pragma omp critical
              bad = T;
            }
          }
        }
    // sort by source triangle
    std::vector<int> idx(L.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return L[a] < L[b]; });
    std::vector<int> L2(L.size());
    std::vector<uint8_t> S2(L.size());
    for (size_t i = 0; i < idx.size(); i++) {
      L2[i] = L[idx[i]];
      S2[i] = S[idx[i]];
    }
    L.swap(L2);
    S.swap(S2);
  }
  if (bad >= 0) return "r_near is smaller than the singular-pair radius (kappa_s (rho_T + rho_T'))";
  nl.tptr.assign(nt + 1, 0);
  for (int T = 0; T < nt; T++) nl.tptr[T + 1] = nl.tptr[T] + (int64_t)lists[T].size();
  nl.src.resize(nl.tptr[nt]);
  nl.sing.resize(nl.tptr[nt]);
  for (int T = 0; T < nt; T++) {
    std::copy(lists[T].begin(), lists[T].end(), nl.src.begin() + nl.tptr[T]);
    std::copy(sflags[T].begin(), sflags[T].end(), nl.sing.begin() + nl.tptr[T]);
  }
  // edge-pair CSR: entry (n, m) collects every near pair (T, T') with T in
  // supp(n), T' in supp(m)
  int ne = g.ne;
  struct Contrib {
    int m, pair;
    uint8_t ij;
  };
  std::vector<std::vector<Contrib>> rows(ne);
#pragma omp parallel for schedule(dynamic, 64)
  for (int n = 0; n < ne; n++) {
    std::vector<Contrib> &R = rows[n];
    for (int s = 0; s < 2; s++) {
      int T = g.et[2 * n + s];
      int i = (g.tedge[3 * T] == n) ? 0 : (g.tedge[3 * T + 1] == n ? 1 : 2);
      for (int64_t p = nl.tptr[T]; p < nl.tptr[T + 1]; p++) {
        int Tp = nl.src[p];
        for (int j = 0; j < 3; j++) R.push_back({g.tedge[3 * Tp + j], (int)p, (uint8_t)(3 * i + j)});
      }
    }
    std::sort(R.begin(), R.end(), [](const Contrib &a, const Contrib &b) { return a.m != b.m ? a.m < b.m : a.pair < b.pair; });
  }
  nl.rowptr.assign(ne + 1, 0);
  std::vector<int64_t> cnt(ne + 1, 0);
  for (int n = 0; n < ne; n++) {
    int64_t u = 0;
    for (size_t k = 0; k < rows[n].size(); k++)
      if (k == 0 || rows[n][k].m != rows[n][k - 1].m) u++;
    nl.rowptr[n + 1] = nl.rowptr[n] + u;
    cnt[n + 1] = cnt[n] + (int64_t)rows[n].size();
  }
  int64_t nnz = nl.rowptr[ne];
  nl.col.resize(nnz);
  nl.cptr.resize(nnz + 1);
  nl.cpair.resize(cnt[ne]);
  nl.cij.resize(cnt[ne]);
#pragma omp parallel for schedule(dynamic, 64)
  for (int n = 0; n < ne; n++) {
    int64_t e = nl.rowptr[n] - 1, c = cnt[n];
    for (size_t k = 0; k < rows[n].size(); k++, c++) {
      if (k == 0 || rows[n][k].m != rows[n][k - 1].m) {
        e++;
        nl.col[e] = rows[n][k].m;
        nl.cptr[e] = c;
      }
      nl.cpair[c] = rows[n][k].pair;
      nl.cij[c] = rows[n][k].ij;
    }
  }
  nl.cptr[nnz] = cnt[ne];
  return "";
}

// unknown slots of an edge: L -> (J, M), R -> (J_e, J_i, M) (Appendix A order)
void edge_slots(const Layout &L, int e, int *slots, int *nslots) {
  int id = L.eidx[e];
  if (!L.isR[e]) {
    slots[0] = id;
    slots[1] = L.NL + id;
    *nslots = 2;
  } else {
    int b = 2 * L.NL;
    slots[0] = b + id;
    slots[1] = b + L.NR + id;
    slots[2] = b + 2 * L.NR + id;
    *nslots = 3;
  }
}

std::string build_clusters(const Geometry &g, const Layout &L, double cell, double overlap, Clusters &cl,
                           bool *too_large, const std::vector<int> *mask) {
  *too_large = false;
  if (!(cell > 0) || overlap < 0 || overlap > cell) return "preconditioner cell must be > 0 and overlap in [0, cell]";
  const int ne = g.ne;
  std::vector<double> mid(3 * ne);
  double lo[3] = {1e300, 1e300, 1e300};
  for (int e = 0; e < ne; e++)
    for (int a = 0; a < 3; a++) {
      mid[3 * e + a] = 0.5 * (g.v[3 * g.ev[2 * e] + a] + g.v[3 * g.ev[2 * e + 1] + a]);
      lo[a] = std::min(lo[a], mid[3 * e + a]);
    }
  std::vector<std::array<int, 3>> key(ne);
  int nc3[3] = {0, 0, 0};
  for (int e = 0; e < ne; e++)
    for (int a = 0; a < 3; a++) {
      key[e][a] = (int)std::floor((mid[3 * e + a] - lo[a]) / cell);
      nc3[a] = std::max(nc3[a], key[e][a] + 1);
    }
  auto cid = [&](int x, int y, int z) { return ((int64_t)x * nc3[1] + y) * nc3[2] + z; };
  // edges outside the mask take part in no cluster (sorted to the end)
  std::vector<int> order(ne);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int64_t> k1(ne);
  const int64_t none = std::numeric_limits<int64_t>::max();
  for (int e = 0; e < ne; e++) k1[e] = (mask && !(*mask)[e]) ? none : cid(key[e][0], key[e][1], key[e][2]);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return k1[a] != k1[b] ? k1[a] < k1[b] : a < b; });
  std::vector<int64_t> sk(ne);
  for (int i = 0; i < ne; i++) sk[i] = k1[order[i]];
  // one cluster per non-empty cell
  std::vector<int64_t> cells;
  for (int i = 0; i < ne; i++)
    if (sk[i] != none && (i == 0 || sk[i] != sk[i - 1])) cells.push_back(sk[i]);
  cl = Clusters();
  cl.nc = (int)cells.size();
  std::vector<std::vector<int>> ext(cl.nc), core(cl.nc);
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < cl.nc; c++) {
    int64_t k = cells[c];
    int cx_ = (int)(k / ((int64_t)nc3[1] * nc3[2])), cy = (int)((k / nc3[2]) % nc3[1]), cz = (int)(k % nc3[2]);
    int ck[3] = {cx_, cy, cz};
    double blo[3], bhi[3];
    for (int a = 0; a < 3; a++) {
      blo[a] = lo[a] + ck[a] * cell - overlap;
      bhi[a] = lo[a] + (ck[a] + 1) * cell + overlap;
    }
    std::vector<int> ee, cc;
    for (int dx = -1; dx <= 1; dx++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dz = -1; dz <= 1; dz++) {
          int x = cx_ + dx, y = cy + dy, z = cz + dz;
          if (x < 0 || y < 0 || z < 0 || x >= nc3[0] || y >= nc3[1] || z >= nc3[2]) continue;
          int64_t kk = cid(x, y, z);
          auto it = std::lower_bound(sk.begin(), sk.end(), kk);
          for (size_t i = it - sk.begin(); i < (size_t)ne && sk[i] == kk; i++) {
            int e = order[i];
            bool in = true;
            for (int a = 0; a < 3; a++) in &= mid[3 * e + a] >= blo[a] && mid[3 * e + a] < bhi[a];
            if (in) ee.push_back(e);
            if (kk == k) cc.push_back(e);
          }
        }
    std::vector<int> es, cs;
    int sl[3], ns;
    for (int e : ee) {
      edge_slots(L, e, sl, &ns);
      es.insert(es.end(), sl, sl + ns);
    }
    for (int e : cc) {
      edge_slots(L, e, sl, &ns);
      cs.insert(cs.end(), sl, sl + ns);
    }
    std::sort(es.begin(), es.end());
    std::sort(cs.begin(), cs.end());
    ext[c].swap(es);
    core[c].swap(cs);
  }
  cl.ext_ptr.assign(cl.nc + 1, 0);
  cl.core_ptr.assign(cl.nc + 1, 0);
  cl.a_off.assign(cl.nc + 1, 0);
  cl.r_off.assign(cl.nc + 1, 0);
  size_t maxext = 0, maxcore = 0;
  for (int c = 0; c < cl.nc; c++) {
    size_t ne_c = ext[c].size(), nc_c = core[c].size();
    maxext = std::max(maxext, ne_c);
    maxcore = std::max(maxcore, nc_c);
    cl.ext_ptr[c + 1] = cl.ext_ptr[c] + ne_c;
    cl.core_ptr[c + 1] = cl.core_ptr[c] + nc_c;
    cl.a_off[c + 1] = cl.a_off[c] + (int64_t)(ne_c * ne_c);
    cl.r_off[c + 1] = cl.r_off[c] + rt_cols((int64_t)ne_c) * rt_stride((int64_t)nc_c);
  }
  if (maxext > (size_t)PC_MAX_EXT || maxcore > (size_t)PC_MAX_CORE) {
    *too_large = true;
    return "preconditioner cluster too large (extended set > 8192 or core > 4096 unknowns); reduce the cell size";
  }
  cl.ext_slot.resize(cl.ext_ptr[cl.nc]);
  cl.core_pos.resize(cl.core_ptr[cl.nc]);
  cl.core_slot.resize(cl.core_ptr[cl.nc]);
  for (int c = 0; c < cl.nc; c++) {
    std::copy(ext[c].begin(), ext[c].end(), cl.ext_slot.begin() + cl.ext_ptr[c]);
    for (size_t i = 0; i < core[c].size(); i++) {
      int s = core[c][i];
      cl.core_slot[cl.core_ptr[c] + i] = s;
      cl.core_pos[cl.core_ptr[c] + i] = (int)(std::lower_bound(ext[c].begin(), ext[c].end(), s) - ext[c].begin());
    }
  }
  return "";
}

void build_local_terms(const Geometry &g, const Layout &L, LocalTerms &lt) {
  // per edge row: up to 5 neighbours (itself and the other edges of its two triangles)
  std::vector<std::vector<std::pair<int, std::array<double, 4>>>> rows(g.ne);
  for (int T = 0; T < g.nt; T++) {
    const double *n = &g.nrm[3 * T];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        std::array<double, 4> acc = {0, 0, 0, 0};
        for (int q = 0; q < NQ; q++) {
          size_t ip = (size_t)T * NQ + q;
          const double *r = &g.qp[3 * ip];
          double w = g.qw[ip], sg = L.sigma[ip];
          double gi[3], fj[3];
          int ei = g.tedge[3 * T + i], ej = g.tedge[3 * T + j];
          double ci = g.tsign[3 * T + i] * g.elen[ei] / (2 * g.area[T]);
          double cj = g.tsign[3 * T + j] * g.elen[ej] / (2 * g.area[T]);
          for (int a = 0; a < 3; a++) {
            gi[a] = ci * (r[a] - g.v[3 * g.t[3 * T + i] + a]);
            fj[a] = cj * (r[a] - g.v[3 * g.t[3 * T + j] + a]);
          }
          double nf[3] = {n[1] * fj[2] - n[2] * fj[1], n[2] * fj[0] - n[0] * fj[2], n[0] * fj[1] - n[1] * fj[0]};
          double gn[3] = {gi[1] * n[2] - gi[2] * n[1], gi[2] * n[0] - gi[0] * n[2], gi[0] * n[1] - gi[1] * n[0]};
          acc[0] += w * (gi[0] * fj[0] + gi[1] * fj[1] + gi[2] * fj[2]);
          acc[1] += w * (gi[0] * nf[0] + gi[1] * nf[1] + gi[2] * nf[2]);
          acc[2] += w * sg * (gn[0] * nf[0] + gn[1] * nf[1] + gn[2] * nf[2]);
          acc[3] += w * sg * (gi[0] * nf[0] + gi[1] * nf[1] + gi[2] * nf[2]);
        }
        int ne_ = g.tedge[3 * T + i], me = g.tedge[3 * T + j];
        auto &R = rows[ne_];
        bool found = false;
        for (auto &pr : R)
          if (pr.first == me) {
            for (int a = 0; a < 4; a++) pr.second[a] += acc[a];
            found = true;
          }
        if (!found) R.push_back({me, acc});
      }
  }
  lt.ptr.assign(g.ne + 1, 0);
  for (int e = 0; e < g.ne; e++) lt.ptr[e + 1] = lt.ptr[e] + (int64_t)rows[e].size();
  lt.col.resize(lt.ptr[g.ne]);
  lt.val.resize(4 * lt.ptr[g.ne]);
  for (int e = 0; e < g.ne; e++) {
    std::sort(rows[e].begin(), rows[e].end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    for (size_t k = 0; k < rows[e].size(); k++) {
      lt.col[lt.ptr[e] + k] = rows[e][k].first;
      for (int a = 0; a < 4; a++) lt.val[4 * (lt.ptr[e] + k) + a] = rows[e][k].second[a];
    }
  }
}

}  // namespace scabs
