// Periodic unit of a guide mesh along x for the block-Toeplitz product
// (fast-solver appendix, Fig. period_WG): rings of identical triangles and
// RWG edges repeated at a fixed pitch, plus the non-periodic remainder.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <unordered_map>

#include "internal.h"

namespace scabs {

namespace {

struct QKey {
  long long x, y, z;
  bool operator==(const QKey &o) const { return x == o.x && y == o.y && z == o.z; }
};
struct QHash {
  size_t operator()(const QKey &k) const {
    return (size_t)(k.x * 73856093LL) ^ (size_t)(k.y * 19349663LL) ^ (size_t)(k.z * 83492791LL);
  }
};

// vertex lookup by position: quantised cells, neighbouring cells searched
struct VertexIndex {
  double q, tol;
  std::unordered_map<QKey, std::vector<int>, QHash> cells;
  const std::vector<double> *v;
  QKey key(double x, double y, double z) const {
    return {(long long)std::floor(x / q), (long long)std::floor(y / q), (long long)std::floor(z / q)};
  }
  void add(int i) {
    const double *p = v->data() + 3 * i;
    cells[key(p[0], p[1], p[2])].push_back(i);
  }
  int find(double x, double y, double z) const {
    QKey k = key(x, y, z);
    for (int a = -1; a <= 1; a++)
      for (int b = -1; b <= 1; b++)
        for (int c = -1; c <= 1; c++) {
          auto it = cells.find({k.x + a, k.y + b, k.z + c});
          if (it == cells.end()) continue;
          for (int i : it->second) {
            const double *p = v->data() + 3 * i;
            if (std::fabs(p[0] - x) <= tol && std::fabs(p[1] - y) <= tol && std::fabs(p[2] - z) <= tol) return i;
          }
        }
    return -1;
  }
};

}  // namespace

int smooth_length(int n) {
  int best = 1 << 30;
  for (long long p2 = 1; p2 < (1LL << 31); p2 *= 2)
    for (long long p = p2; p < (1LL << 31); p *= 3) {
      if (p >= n && p < best) best = (int)p;
      if (p >= n) break;
    }
  return best;
}

void make_tri_records(const Geometry &g, std::vector<TriD> &out) {
  out.assign(g.nt, TriD{});
  for (int T = 0; T < g.nt; T++) {
    TriD &r = out[T];
    for (int k = 0; k < 3; k++)
      for (int c = 0; c < 3; c++) r.v[3 * k + c] = g.v[3 * g.t[3 * T + k] + c];
    for (int i = 0; i < 21; i++) r.qp[i] = g.qp[21 * (size_t)T + i];
    for (int q = 0; q < NQ; q++) r.qw[q] = g.qw[NQ * (size_t)T + q];
    double e1[3], len = 0;
    for (int c = 0; c < 3; c++) {
      r.nrm[c] = g.nrm[3 * T + c];
      r.cen[c] = g.cen[3 * T + c];
      e1[c] = r.v[3 + c] - r.v[c];
      len += e1[c] * e1[c];
    }
    len = std::sqrt(len);
    for (int c = 0; c < 3; c++) r.t1[c] = e1[c] / len;
    r.t2[0] = r.nrm[1] * r.t1[2] - r.nrm[2] * r.t1[1];
    r.t2[1] = r.nrm[2] * r.t1[0] - r.nrm[0] * r.t1[2];
    r.t2[2] = r.nrm[0] * r.t1[1] - r.nrm[1] * r.t1[0];
    r.rho = g.rho[T];
    for (int k = 0; k < 3; k++) {
      const int e = g.tedge[3 * T + k];
      r.coef[k] = g.tsign[3 * T + k] * g.elen[e] / (2.0 * g.area[T]);
    }
    r.body = g.body[T];
  }
}

std::string build_rings(const Geometry &g, RingTemplate &rt) {
  rt = RingTemplate();
  rt.nbody = g.nbody;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = 0; i < g.nv; i++)
    for (int c = 0; c < 3; c++) {
      lo[c] = std::min(lo[c], g.v[3 * i + c]);
      hi[c] = std::max(hi[c], g.v[3 * i + c]);
    }
  const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  const double tol = 1e-9 * ext;
  // pitch: the smallest gap between distinct vertex x coordinates
  std::vector<double> xs(g.nv);
  for (int i = 0; i < g.nv; i++) xs[i] = g.v[3 * i];
  std::sort(xs.begin(), xs.end());
  double dx = 0;
  for (int i = 1; i < g.nv; i++) {
    const double d = xs[i] - xs[i - 1];
    if (d > 1e3 * tol && (dx == 0 || d < dx)) dx = d;
  }
  if (!(dx > 0)) return "the mesh has no periodic unit along x";
  rt.dx = dx;
  VertexIndex vi;
  vi.q = 1e-6 * ext;
  vi.tol = 1e3 * tol;
  vi.v = &g.v;
  for (int i = 0; i < g.nv; i++) vi.add(i);
  // triangles by vertex set; next[T] = the triangle translated by +dx
  std::map<std::array<int, 3>, int> tmap;
  for (int T = 0; T < g.nt; T++) {
    std::array<int, 3> k = {g.t[3 * T], g.t[3 * T + 1], g.t[3 * T + 2]};
    std::sort(k.begin(), k.end());
    tmap[k] = T;
  }
  std::vector<int> next(g.nt, -1), prev(g.nt, -1);
  for (int T = 0; T < g.nt; T++) {
    int w[3];
    bool ok = true;
    for (int k = 0; k < 3 && ok; k++) {
      const double *p = g.v.data() + 3 * g.t[3 * T + k];
      w[k] = vi.find(p[0] + dx, p[1], p[2]);
      ok = w[k] >= 0;
    }
    if (!ok) continue;
    std::array<int, 3> k = {w[0], w[1], w[2]};
    std::sort(k.begin(), k.end());
    auto it = tmap.find(k);
    if (it == tmap.end()) continue;
    const int U = it->second;
    // U's vertices are the translates of T's in the same order (not only the
    // same cyclic order): the quadrature points and local edges of U are then
    // the translates of T's with the same indices, as the ring template needs
    if (g.t[3 * U] != w[0] || g.t[3 * U + 1] != w[1] || g.t[3 * U + 2] != w[2]) continue;
    next[T] = U;
    prev[U] = T;
  }
  // chains of translates; each covers the rings [s, s + len) counted from
  // the smallest x of the mesh.  The periodic part is the ring window [a, b)
  // that the most triangles cover: chains spanning the window, cut to it,
  // maximising (chains) x (b - a), at least 3 rings (ties: the longer window)
  auto xmin_of = [&](int T) {
    double m = 1e300;
    for (int k = 0; k < 3; k++) m = std::min(m, g.v[3 * g.t[3 * T + k]]);
    return m;
  };
  std::vector<std::vector<int>> chains;
  std::vector<int> cstart;
  for (int T = 0; T < g.nt; T++) {
    if (prev[T] >= 0) continue;
    std::vector<int> c;
    for (int U = T; U >= 0 && (int)c.size() <= g.nt; U = next[U]) c.push_back(U);
    cstart.push_back((int)std::lround((xmin_of(c[0]) - lo[0]) / dx));
    chains.push_back(std::move(c));
  }
  std::vector<int> starts, ends;
  for (size_t i = 0; i < chains.size(); i++) {
    starts.push_back(cstart[i]);
    ends.push_back(cstart[i] + (int)chains[i].size());
  }
  std::sort(starts.begin(), starts.end());
  starts.erase(std::unique(starts.begin(), starts.end()), starts.end());
  std::sort(ends.begin(), ends.end());
  ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
  long long best = 0;
  int wa = 0, wb = 0;
  for (int a : starts)
    for (int b : ends) {
      if (b - a < 3) continue;
      long long n = 0;
      for (size_t i = 0; i < chains.size(); i++)
        n += cstart[i] <= a && cstart[i] + (int)chains[i].size() >= b;
      const long long score = n * (b - a);
      if (score > best || (score == best && b - a > wb - wa)) {
        best = score;
        wa = a;
        wb = b;
      }
    }
  if (best == 0) return "the mesh has fewer than three periodic rings along x";
  const int nr = wb - wa;
  std::vector<std::vector<int>> per;
  for (size_t i = 0; i < chains.size(); i++)
    if (cstart[i] <= wa && cstart[i] + (int)chains[i].size() >= wb)
      per.emplace_back(chains[i].begin() + (wa - cstart[i]), chains[i].begin() + (wb - cstart[i]));
  std::stable_sort(per.begin(), per.end(), [&](const std::vector<int> &a, const std::vector<int> &b) {
    if (g.body[a[0]] != g.body[b[0]]) return g.body[a[0]] < g.body[b[0]];
    return a[0] < b[0];
  });
  rt.nr = nr;
  rt.nt_r = (int)per.size();
  rt.tri_loc.assign(g.nt, -1);
  rt.tri_ring.assign(g.nt, -1);
  std::vector<int> &tri_ring = rt.tri_ring;
  rt.pmap.assign((size_t)rt.nt_r * nr, -1);
  for (int lt = 0; lt < rt.nt_r; lt++)
    for (int j = 0; j < nr; j++) {
      const int T = per[lt][j];
      rt.tri_loc[T] = lt;
      tri_ring[T] = j;
      rt.pmap[(size_t)lt * nr + j] = T;
    }
  // periodic edges: both triangles periodic, halves at ring offsets 0 / -1
  rt.edge_loc.assign(g.ne, -1);
  rt.edge_ring.assign(g.ne, 0);
  rt.edge_sgn.assign(g.ne, 0);
  std::map<std::array<int, 6>, int> emap;
  std::vector<std::array<int, 6>> keys;
  for (int e = 0; e < g.ne; e++) {
    const int T0 = g.et[2 * e], T1 = g.et[2 * e + 1];
    if (rt.tri_loc[T0] < 0 || rt.tri_loc[T1] < 0) continue;
    const int r0 = tri_ring[T0], r1 = tri_ring[T1], re = std::max(r0, r1);
    const int o0 = r0 - re, o1 = r1 - re;
    if (o0 < -1 || o1 < -1) continue;
    int k0 = -1, k1 = -1;
    for (int k = 0; k < 3; k++) {
      if (g.tedge[3 * T0 + k] == e) k0 = k;
      if (g.tedge[3 * T1 + k] == e) k1 = k;
    }
    std::array<int, 6> A = {rt.tri_loc[T0], k0, o0, rt.tri_loc[T1], k1, o1};
    std::array<int, 6> B = {rt.tri_loc[T1], k1, o1, rt.tri_loc[T0], k0, o0};
    const bool a_first = A < B;
    const std::array<int, 6> &K = a_first ? A : B;
    auto it = emap.find(K);
    int id;
    if (it == emap.end()) {
      id = (int)keys.size();
      emap[K] = id;
      keys.push_back(K);
    } else {
      id = it->second;
    }
    rt.edge_loc[e] = id;
    rt.edge_ring[e] = re;
    rt.edge_sgn[e] = a_first ? 1 : -1;   // actual T+ is the template's + side
  }
  // order local edges by body
  const int ne_r = (int)keys.size();
  if (ne_r == 0) return "the periodic rings along x share no RWG edge";
  std::vector<int> order(ne_r);
  for (int i = 0; i < ne_r; i++) order[i] = i;
  auto ebody = [&](int id) { return g.body[per[keys[id][0]][0]]; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ebody(a) < ebody(b); });
  std::vector<int> newid(ne_r);
  for (int i = 0; i < ne_r; i++) newid[order[i]] = i;
  rt.ne_r = ne_r;
  rt.e_tri.resize(2 * ne_r);
  rt.e_k.resize(2 * ne_r);
  rt.e_off.resize(2 * ne_r);
  for (int i = 0; i < ne_r; i++) {
    const auto &K = keys[order[i]];
    for (int s = 0; s < 2; s++) {
      rt.e_tri[2 * i + s] = K[3 * s];
      rt.e_k[2 * i + s] = K[3 * s + 1];
      rt.e_off[2 * i + s] = K[3 * s + 2];
    }
  }
  rt.ringmap.assign((size_t)ne_r * nr, -1);
  for (int e = 0; e < g.ne; e++) {
    if (rt.edge_loc[e] < 0) continue;
    const int a = newid[rt.edge_loc[e]];
    rt.edge_loc[e] = a;
    int &slot = rt.ringmap[(size_t)a * nr + rt.edge_ring[e]];
    if (slot >= 0) return "two periodic edges share one local edge and ring";
    slot = e;
  }
  // body ranges
  rt.body_e0.assign(g.nbody + 1, 0);
  rt.body_t0.assign(g.nbody + 1, 0);
  for (int lt = 0; lt < rt.nt_r; lt++) rt.body_t0[g.body[per[lt][0]] + 1]++;
  for (int a = 0; a < ne_r; a++) rt.body_e0[g.body[per[rt.e_tri[2 * a]][0]] + 1]++;
  for (int b = 0; b < g.nbody; b++) {
    rt.body_t0[b + 1] += rt.body_t0[b];
    rt.body_e0[b + 1] += rt.body_e0[b];
  }
  // template triangles (ring 0) with the template's half-function signs
  std::vector<TriD> all;
  make_tri_records(g, all);
  rt.tri.resize(rt.nt_r);
  for (int lt = 0; lt < rt.nt_r; lt++) rt.tri[lt] = all[per[lt][0]];
  for (int a = 0; a < ne_r; a++)
    for (int s = 0; s < 2; s++) {
      TriD &t = rt.tri[rt.e_tri[2 * a + s]];
      const int k = rt.e_k[2 * a + s];
      t.coef[k] = (s == 0 ? 1.0 : -1.0) * std::fabs(t.coef[k]);
    }
  rt.P = smooth_length(2 * nr - 1);
  return "";
}

}  // namespace scabs
