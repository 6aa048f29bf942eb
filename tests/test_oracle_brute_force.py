"""Brute-force pin of the oracle's dense Galerkin matrix on tiny closed meshes.

The five-current system of Appendix A (eq19) is assembled here a second time,
independently of the oracle's C code, straight from its definition:

* RWG half functions on every triangle (edges sorted by vertex pair, the
  lower-numbered triangle carrying the + half), the degree-5 seven-point rule
  on test and source triangles (pinned separately), unknowns
  [J^L, M^L, J_e^R, J_i^R, M^R] and rows [eq1, eq2, eq3, eq13, eq14];
* one-sided fields E^+/- = PV +/- 1/2 n x M, H^+/- = PV -/+ 1/2 n x J, the
  L operator tested by parts on the test side, the sigma-weighted tests of
  eq13 (rotated by n x) and eq14 taken pointwise at the quadrature points;
* for singular pairs (centroid distance below kappa_s (rho + rho')) the static
  kernel 1/(4 pi R) integrated over the source triangle by brute force --
  Duffy-transformed tensor Gauss-Legendre for int 1/R and int (r' - r)/R, the
  tangential part of int grad(1/R) as the edge line integrals of Gauss's
  theorem (Gauss-Legendre on each edge, split at the foot point), the normal
  part as h * int 1/R^3 by Duffy quadrature -- plus the seven-point rule on
  the smooth remainder G - 1/(4 pi R); the plain seven-point rule otherwise.

None of this shares code with the oracle's closed-form potential integrals
(Wilton/Graglia), its inner-integral routine or its stamping.  The meshes
(a tetrahedron, an octahedron, a one-cell box) produce coincident,
edge-adjacent (coplanar and at an angle), vertex-adjacent and disjoint pairs;
some triangles carry a random conductivity so L and R edges and every row type
appear.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import synth

NQ = 7


def _rule7():
    """Barycentric points and weights (sum 1) of the seven-point rule, read
    from the oracle's table, which test_rule7_exact_to_degree_5 pins."""
    b = np.zeros((7, 3))
    w = np.zeros(7)
    oracle.lib().or_rule7.argtypes = [np.ctypeslib.ndpointer(np.float64), np.ctypeslib.ndpointer(np.float64)]
    oracle.lib().or_rule7(b, w)
    return b, w


# ---------------------------------------------------------------------------
# brute-force static integrals over a flat triangle
# ---------------------------------------------------------------------------
_GL = {}


def _gl(n):
    if n not in _GL:
        x, w = np.polynomial.legendre.leggauss(n)
        _GL[n] = (0.5 * (x + 1), 0.5 * w)
    return _GL[n]


def _adaptive_rect(fun, rtol=1e-13, ng=8, max_depth=30):
    """Adaptive tensor Gauss-Legendre over the unit square: a cell is accepted
    when its ng x ng estimate and the sum over its four children agree to
    rtol times the integral's magnitude, scaled by the cell's area (norm of
    the vector-valued integrand)."""
    g, gw = _gl(ng)
    G1, G2 = np.meshgrid(g, g, indexing="ij")
    W = np.outer(gw, gw).ravel()

    def est(cells, absval=False):
        # cells: (m, 4) = (u0, v0, du, dv)
        u = cells[:, 0:1] + cells[:, 2:3] * G1.ravel()[None, :]
        v = cells[:, 1:2] + cells[:, 3:4] * G2.ravel()[None, :]
        vals = fun(u.ravel(), v.ravel())
        vals = vals.reshape(cells.shape[0], W.size, -1)
        if absval:
            vals = np.abs(vals)
        return np.einsum("mqk,q->mk", vals, W) * (cells[:, 2] * cells[:, 3])[:, None]

    def split(cells):
        h = cells[:, 2:4] * 0.5
        return np.concatenate([np.column_stack([cells[:, 0] + a * h[:, 0], cells[:, 1] + b * h[:, 1], h])
                               for a in (0, 1) for b in (0, 1)])

    cells = split(split(np.array([[0.0, 0.0, 1.0, 1.0]])))
    coarse = est(cells)
    # the scale is the integral of |f| (a sum that does not cancel)
    tol = rtol * max(np.linalg.norm(est(cells, absval=True).sum(axis=0)), 1e-300)
    total = 0
    for _ in range(max_depth):
        kids = split(cells)
        fine = est(kids).reshape(4, cells.shape[0], -1)
        fsum = fine.sum(axis=0)
        area = cells[:, 2] * cells[:, 3]
        ok = np.linalg.norm(fsum - coarse, axis=1) <= tol * np.maximum(area, 1e-3)
        total = total + fsum[ok].sum(axis=0)
        if ok.all():
            return total
        bad = ~ok
        cells = np.concatenate([kids.reshape(4, -1, 4)[k][bad] for k in range(4)])
        coarse = fine[:, bad].reshape(-1, fine.shape[2])
        if cells.shape[0] > 20000:
            break
    raise RuntimeError("adaptive quadrature did not converge")


def _duffy(fun, r, P3):
    """int over the triangle P3 of fun(q) (q: (m, 3) points -> (m, k)), split
    at the foot point of r into three (signed) sub-triangles, each mapped to
    the unit square by Duffy's transform (which removes an integrable 1/R at
    the foot point) and integrated adaptively."""
    p0, p1, p2 = P3
    n = np.cross(p1 - p0, p2 - p0)
    n /= np.linalg.norm(n)
    P = r - np.dot(r - p0, n) * n
    tot = 0
    for B, C in ((p0, p1), (p1, p2), (p2, p0)):
        cr = np.cross(B - P, C - P)
        jac = np.linalg.norm(cr) * np.sign(np.dot(cr, n))
        if abs(jac) < 1e-300:
            continue

        def f(u, v, B=B, C=C, jac=jac):
            q = P + u[:, None] * (B - P) + (u * v)[:, None] * (C - B)
            return fun(q).reshape(u.size, -1) * (u * jac)[:, None]

        tot = tot + _adaptive_rect(f)
    return tot


def _edge_line_1_over_R(r, a, b, ng=48):
    """int over the segment a-b of 1/|r - s| ds, split at the foot point."""
    L = np.linalg.norm(b - a)
    t = (b - a) / L
    s0 = np.clip(np.dot(r - a, t), 0.0, L)
    g, gw = _gl(ng)
    tot = 0.0
    for lo, hi in ((0.0, s0), (s0, L)):
        if hi - lo <= 0:
            continue
        # cluster the nodes toward the foot point with s = foot +- (dist) u^2
        s = lo + (hi - lo) * (g ** 2 if lo == s0 else 1 - g ** 2)
        ds = (hi - lo) * 2 * g
        pts = a + s[:, None] * t
        tot += np.sum(gw * ds / np.linalg.norm(r - pts, axis=1))
    return tot


def static_parts(r, P3):
    """(int 1/R, int (r' - r)/R, int grad_r (1/R)) over the triangle P3 at r;
    the last is the principal value (zero normal part for r in the plane)."""
    p0, p1, p2 = P3
    n = np.cross(p1 - p0, p2 - p0)
    A2 = np.linalg.norm(n)
    n /= A2
    R = lambda q: np.linalg.norm(r - q, axis=1)
    both = _duffy(lambda q: np.column_stack([1.0 / R(q), (q - r) / R(q)[:, None]]), r, P3)
    I0, I1 = both[0], both[1:]
    # tangential part: grad_r (1/R) = -grad' (1/R); Gauss on the surface gives
    # int grad'_t (1/R) = sum over edges of m_e int_e 1/R (m_e outward in-plane)
    gt = np.zeros(3)
    for a, b in ((p0, p1), (p1, p2), (p2, p0)):
        e = b - a
        m = np.cross(e, n)
        m /= np.linalg.norm(m)
        gt -= m * _edge_line_1_over_R(r, a, b)
    h = np.dot(r - p0, n)
    gn = 0.0
    if abs(h) > 1e-12 * math.sqrt(A2):
        gn = -h * _duffy(lambda q: 1.0 / R(q) ** 3, r, P3)[0]
    return I0, I1, gt + gn * n


# ---------------------------------------------------------------------------
# independent assembly of the dense system
# ---------------------------------------------------------------------------
class Brute:
    def __init__(self, mesh, omega, eps_in, eps_out=1.0, kappa_s=1.37, sigma=None):
        self.v = np.asarray(mesh.verts, float)
        self.t = np.asarray(mesh.tris, int)
        self.body = np.asarray(mesh.body, int)
        nt = self.nt = self.t.shape[0]
        self.k = {"e": omega * math.sqrt(eps_out), "i": omega * math.sqrt(eps_in)}
        self.Z = {"e": 1 / math.sqrt(eps_out), "i": 1 / math.sqrt(eps_in)}
        self.kappa_s = kappa_s
        self._static = {}   # static parts are independent of the medium
        P = self.v[self.t]                                  # (nt, 3, 3)
        cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.nrm = cr / (2 * self.area[:, None])
        self.cen = P.mean(axis=1)
        self.rho = np.max(np.linalg.norm(P - self.cen[:, None, :], axis=2), axis=1)
        b, w = _rule7()
        self.qp = np.einsum("qk,tkc->tqc", b, P)            # (nt, 7, 3)
        self.qw = w[None, :] * self.area[:, None]
        # edges: sorted vertex pairs; local index k = edge opposite vertex k
        pairs = {}
        for T in range(nt):
            for k in range(3):
                a, c = self.t[T, (k + 1) % 3], self.t[T, (k + 2) % 3]
                pairs.setdefault((min(a, c), max(a, c)), []).append((T, k))
        keys = sorted(pairs)
        self.ne = len(keys)
        self.tedge = np.zeros((nt, 3), int)
        self.tsign = np.zeros((nt, 3), int)
        self.elen = np.zeros(self.ne)
        self.etri = np.zeros((self.ne, 2), int)
        for e, key in enumerate(keys):
            (T0, k0), (T1, k1) = sorted(pairs[key])
            self.tedge[T0, k0], self.tsign[T0, k0] = e, +1
            self.tedge[T1, k1], self.tsign[T1, k1] = e, -1
            self.etri[e] = (T0, T1)
            self.elen[e] = np.linalg.norm(self.v[key[0]] - self.v[key[1]])
        self.sigma = np.zeros((nt, NQ)) if sigma is None else np.asarray(sigma, float).reshape(nt, NQ)
        isR = np.array([np.any(self.sigma[list(self.etri[e])] > 0) for e in range(self.ne)])
        self.isR = isR
        self.NL, self.NR = int(np.sum(~isR)), int(np.sum(isR))
        self.N = 2 * self.NL + 3 * self.NR
        idx = np.zeros(self.ne, int)
        idx[~isR] = np.arange(self.NL)
        idx[isR] = np.arange(self.NR)
        self.idx = idx

    # half RWG function k of triangle T at points r (m, 3) and its divergence
    def half(self, T, k, r):
        e = self.tedge[T, k]
        c = self.tsign[T, k] * self.elen[e] / (2 * self.area[T])
        return c * (r - self.v[self.t[T, k]]), 2 * c

    def singular(self, T, Tp):
        return np.linalg.norm(self.cen[T] - self.cen[Tp]) < self.kappa_s * (self.rho[T] + self.rho[Tp])

    def inner(self, r, Tp, kk, sing):
        """a_j = int G f_j, phi_j = int G div f_j, gphi_j = int grad G div f_j,
        c_j = int grad G x f_j over source triangle Tp at the point r."""
        sp, sw = self.qp[Tp], self.qw[Tp]
        d = r[None, :] - sp
        R = np.linalg.norm(d, axis=1)
        x = kk * R
        with np.errstate(divide="ignore", invalid="ignore"):
            if sing:
                em1 = -2 * np.sin(0.5 * x) ** 2 - 1j * np.sin(x)        # exp(-jx) - 1
                G = np.where(R > 0, em1 / (4 * math.pi * R), -1j * kk / (4 * math.pi))
                dG = np.where(R > 0, (-1j * x * (em1 + 1) - em1) / (4 * math.pi * R * R), 0)
            else:
                e = np.exp(-1j * x)
                G = e / (4 * math.pi * R)
                dG = -(1 + 1j * x) * e / (4 * math.pi * R * R)
            gG = np.where(R[:, None] > 1e-14, dG[:, None] * d / R[:, None], 0)   # grad_r G
        # int G q' and int grad G x q' (q' the source point) by the rule
        S0 = np.sum(sw * G)
        Sq = np.sum((sw * G)[:, None] * sp, axis=0)
        Sg = np.sum(sw[:, None] * gG, axis=0)
        Sx = np.sum(sw[:, None] * np.cross(gG, sp), axis=0)
        if sing:
            key = (tuple(r), Tp)
            if key not in self._static:
                self._static[key] = static_parts(r, self.v[self.t[Tp]])
            I0, I1, Ig = self._static[key]
            c4 = 1 / (4 * math.pi)
            S0 = S0 + c4 * I0
            Sq = Sq + c4 * (I1 + r * I0)                        # int q'/R = int (q' - r)/R + r int 1/R
            Sg = Sg + c4 * Ig
            # int grad(1/R) x q' = int grad(1/R) x (q' - r) + Ig x r; the first
            # integrand vanishes (grad_r(1/R) is parallel to r - q')
            Sx = Sx + c4 * np.cross(Ig, r)
        out = []
        for j in range(3):
            e = self.tedge[Tp, j]
            cj = self.tsign[Tp, j] * self.elen[e] / (2 * self.area[Tp])
            vj = self.v[self.t[Tp, j]]
            a = cj * (Sq - vj * S0)
            phi = 2 * cj * S0
            gphi = 2 * cj * Sg
            cc = cj * (Sx - np.cross(Sg, vj))
            out.append((a, phi, gphi, cc))
        return out

    def dense(self):
        """The five-current matrix A (rows eq1, eq2, eq3, eq13, eq14)."""
        ne, N = self.ne, self.N
        # per (row edge, column edge): tested fields of the source currents
        # Ee[n, m, c]: <X_n, E_e(c_m)>, c in (J, M); likewise He, Ei, Hi;
        # sig_rot[n, m, c]: sum w sigma (X_n x n).E_e^{PV}(c_m); sig[n, m, c]: sum w sigma X_n.E_i^{PV}(c_m)
        F = {key: np.zeros((ne, ne, 2), complex) for key in ("Ee", "He", "Ei", "Hi", "Srot", "Ssig")}
        for T in range(self.nt):
            for Tp in range(self.nt):
                sing = self.singular(T, Tp)
                meds = ["e"] + (["i"] if self.body[T] == self.body[Tp] else [])
                for med in meds:
                    kk, Z = self.k[med], self.Z[med]
                    for q in range(NQ):
                        r, w, sg = self.qp[T, q], self.qw[T, q], self.sigma[T, q]
                        inn = self.inner(r, Tp, kk, sing)
                        for i in range(3):
                            g, dg = self.half(T, i, r[None, :])
                            g = g[0]
                            n = self.tedge[T, i]
                            gxn = np.cross(g, self.nrm[T])
                            for j, (a, phi, gphi, cc) in enumerate(inn):
                                m = self.tedge[Tp, j]
                                Lt = 1j * kk * (np.dot(g, a) - dg * phi / kk ** 2)     # tested L, by parts
                                Kv = -cc                                                  # K(f)(r)
                                Lv = 1j * kk * (a + gphi / kk ** 2)                       # L(f)(r)
                                Kt = np.dot(g, Kv)
                                # E = -Z L(J) + K(M);  H = -K(J) - L(M)/Z
                                if med == "e":
                                    F["Ee"][n, m, 0] += w * (-Z * Lt)
                                    F["Ee"][n, m, 1] += w * Kt
                                    F["He"][n, m, 0] += w * (-Kt)
                                    F["He"][n, m, 1] += w * (-Lt / Z)
                                    if sg:
                                        F["Srot"][n, m, 0] += w * sg * np.dot(gxn, -Z * Lv)
                                        F["Srot"][n, m, 1] += w * sg * np.dot(gxn, Kv)
                                else:
                                    F["Ei"][n, m, 0] += w * (-Z * Lt)
                                    F["Ei"][n, m, 1] += w * Kt
                                    F["Hi"][n, m, 0] += w * (-Kt)
                                    F["Hi"][n, m, 1] += w * (-Lt / Z)
                                    if sg:
                                        F["Ssig"][n, m, 0] += w * sg * np.dot(g, -Z * Lv)
                                        F["Ssig"][n, m, 1] += w * sg * np.dot(g, Kv)
        # local (same-triangle) terms of the one-sided limits and of eq14:
        # Gram <X_n, X_m>, <X_n, n x X_m>, sum w sigma (X_n x n).(n x X_m), sum w sigma X_n.(n x X_m)
        Gram = np.zeros((ne, ne))
        Gnx = np.zeros((ne, ne))
        Grot = np.zeros((ne, ne))
        Gsnx = np.zeros((ne, ne))
        for T in range(self.nt):
            nT = self.nrm[T]
            for i in range(3):
                gi, _ = self.half(T, i, self.qp[T])
                for j in range(3):
                    fj, _ = self.half(T, j, self.qp[T])
                    nf = np.cross(nT[None, :], fj)
                    gxn = np.cross(gi, nT[None, :])
                    n, m = self.tedge[T, i], self.tedge[T, j]
                    w, sg = self.qw[T], self.sigma[T]
                    Gram[n, m] += np.sum(w * np.sum(gi * fj, axis=1))
                    Gnx[n, m] += np.sum(w * np.sum(gi * nf, axis=1))
                    Grot[n, m] += np.sum(w * sg * np.sum(gxn * nf, axis=1))
                    Gsnx[n, m] += np.sum(w * sg * np.sum(gi * nf, axis=1))
        # rows as functions of the per-edge currents (J_e, J_i, M), M_e = M, M_i = -M
        #  E  : <X, E_e^+ - E_i^->                          (residues cancel)
        #  H  : <X, H_e^+ - H_i^->  + sum w sigma (X x n).E_e^+
        #  R14: <X, J_e + J_i> - sum w sigma X.E_i^-
        # E_e^+ = PV + 1/2 n x M, E_i^- = PV - 1/2 n x M_i = PV + 1/2 n x M,
        # H_e^+ - H_i^- = PV_e - PV_i - 1/2 n x (J_e + J_i)
        row = {}
        row["E"] = (F["Ee"][:, :, 0], -F["Ei"][:, :, 0], F["Ee"][:, :, 1] + F["Ei"][:, :, 1])
        row["H"] = (F["He"][:, :, 0] + F["Srot"][:, :, 0] - 0.5 * Gnx,
                    -F["Hi"][:, :, 0] - 0.5 * Gnx,
                    F["He"][:, :, 1] + F["Hi"][:, :, 1] + F["Srot"][:, :, 1] + 0.5 * Grot)
        row["R"] = (Gram, Gram - F["Ssig"][:, :, 0], F["Ssig"][:, :, 1] - 0.5 * Gsnx)
        # unknown and row slots
        NL, NR, idx, isR = self.NL, self.NR, self.idx, self.isR
        A = np.zeros((N, N), complex)
        rows_of = lambda n: ((idx[n], NL + idx[n], None) if not isR[n] else
                             (2 * NL + idx[n], 2 * NL + NR + idx[n], 2 * NL + 2 * NR + idx[n]))
        for n in range(ne):
            rE, rH, r14 = rows_of(n)
            for key, rr in (("E", rE), ("H", rH), ("R", r14)):
                if rr is None:
                    continue
                cJe, cJi, cM = row[key]
                for m in range(ne):
                    if not isR[m]:
                        # J_e = J, J_i = -J
                        A[rr, idx[m]] += cJe[n, m] - cJi[n, m]
                        A[rr, NL + idx[m]] += cM[n, m]
                    else:
                        A[rr, 2 * NL + idx[m]] += cJe[n, m]
                        A[rr, 2 * NL + NR + idx[m]] += cJi[n, m]
                        A[rr, 2 * NL + 2 * NR + idx[m]] += cM[n, m]
        return A


def _octahedron(scale=0.3, jitter=0.03, seed=5):
    rng = synth.SplitMix64(seed)
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float) * scale
    V += np.array([[rng.uniform_range(-jitter, jitter) for _ in range(3)] for _ in range(6)])
    T = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], np.int32)
    c = V.mean(axis=0)
    for i, (a, b, cc) in enumerate(T):
        if np.dot(np.cross(V[b] - V[a], V[cc] - V[a]), V[a] - c) < 0:
            T[i] = (a, cc, b)
    return V, T


def _tetrahedron(scale=0.25):
    V = np.array([[0, 0, 0], [1.0, 0.1, 0], [0.2, 0.9, 0.05], [0.3, 0.3, 0.8]]) * scale
    T = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], np.int32)
    return V, T


def _meshes():
    out = {}
    out["tetra"] = synth.merge_bodies([_tetrahedron()])
    out["octa"] = synth.merge_bodies([_octahedron()])
    v, t = synth.box_mesh(0.0, 0.3, -0.1, 0.1, -0.05, 0.05, 0.3)    # one cell per axis: 12 triangles
    out["box"] = synth.merge_bodies([(v, t)])
    return out


def _random_sigma(nt, seed, ntri=2):
    """Positive conductivity (varying from point to point) on ntri seeded
    triangles, zero elsewhere, so that L and R edges both occur."""
    rng = synth.SplitMix64(seed)
    s = np.zeros((nt, NQ))
    chosen = set()
    while len(chosen) < min(ntri, nt):
        chosen.add(int(rng.uniform() * nt))
    for T in sorted(chosen):
        s[T] = [0.2 + 1.5 * rng.uniform() for _ in range(NQ)]
    return s.ravel()


@pytest.mark.parametrize("name,kappa_s", [("tetra", 1.37), ("octa", 1.37), ("octa", 0.6), ("box", 1.37)])
def test_dense_matches_brute_force(name, kappa_s):
    """P12: the oracle's dense matrix (all eight tested operator types, the
    residues and the Gram block) equals the independent brute-force assembly
    to 1e-11 of its largest entry; kappa_s = 0.6 leaves some pairs to the
    plain rule."""
    mesh = _meshes()[name]
    omega, eps_in = synth.OMEGA, synth.EPS_IN
    o = oracle.Oracle(mesh, omega, eps_in, kappa_s=kappa_s)
    sig = _random_sigma(o.nt, 17 + len(name))
    o.set_sigma_points(sig)
    assert 0 < o.NR < o.ne, "the case must mix L and R edges"
    A = o.dense()
    bf = Brute(mesh, omega, eps_in, kappa_s=kappa_s, sigma=sig)
    assert (bf.NL, bf.NR) == (o.NL, o.NR)
    assert np.array_equal(bf.isR.astype(np.int32), o.isR) and np.array_equal(bf.idx, o.eidx)
    if kappa_s < 1:
        flags = [bf.singular(T, Tp) for T in range(bf.nt) for Tp in range(bf.nt)]
        assert any(flags) and not all(flags)
    B = bf.dense()
    scale = np.max(np.abs(B))
    err = np.max(np.abs(A - B)) / scale
    print(name, kappa_s, "N", o.N, "max |A - A_bf| / max |A_bf|", err)
    assert err < 1e-11
    # every block type is populated (the comparison is not vacuous)
    NL, NR = o.NL, o.NR
    r14 = slice(2 * NL + 2 * NR, None)
    assert np.max(np.abs(B[r14, :])) > 1e-3 * scale


def test_static_parts_brute_force_vs_closed_forms():
    """The brute-force static integrals used above against the oracle's closed
    forms at points off the plane, near an edge and in the plane."""
    P3 = [np.array([0.0, 0, 0]), np.array([1.0, 0.1, 0]), np.array([0.2, 0.9, 0.0])]
    for r in ([0.2, 0.3, 0.15], [0.45, 0.05, 0.01], [0.37, 0.31, 0.0], [1.2, 0.9, 0.0], [0.5, -0.3, -0.2]):
        r = np.array(r)
        I0, I1, Ig = static_parts(r, P3)
        J0, J1, Jg = oracle.static_integrals(r, *P3)
        assert abs(I0 - J0) < 1e-10 * abs(J0)
        assert np.linalg.norm(I1 - J1) < 1e-10 * np.linalg.norm(J1)
        assert np.linalg.norm(Ig - Jg) < 1e-9 * np.linalg.norm(Jg)


def test_rhs_matches_definition():
    """Right-hand side rows <X_n, E_inc>, <X_n, H_inc> and the eq14 row
    sum w sigma X_n.E_inc, from the dipole field at the quadrature points."""
    mesh = _meshes()["octa"]
    o = oracle.Oracle(mesh, synth.OMEGA, synth.EPS_IN)
    sig = _random_sigma(o.nt, 29)
    o.set_sigma_points(sig)
    bf = Brute(mesh, synth.OMEGA, synth.EPS_IN, sigma=sig)
    dip = synth.Dipole(np.array([0.02, -0.01, 0.03]), np.array([0.3, -0.5 + 0.2j, 0.8]), 0)
    b = o.rhs_dipole(dip)
    ref = np.zeros(o.N, complex)
    for T in range(bf.nt):
        for q in range(NQ):
            r = bf.qp[T, q]
            E, H = oracle.dipole_field(bf.k["i"], bf.Z["i"], dip.pos, dip.moment, r)
            for i in range(3):
                g, _ = bf.half(T, i, r[None, :])
                g = g[0]
                n = bf.tedge[T, i]
                w, sg = bf.qw[T, q], bf.sigma[T, q]
                if not bf.isR[n]:
                    ref[bf.idx[n]] += w * np.dot(g, E)
                    ref[bf.NL + bf.idx[n]] += w * np.dot(g, H)
                else:
                    base = 2 * bf.NL
                    ref[base + bf.idx[n]] += w * np.dot(g, E)
                    ref[base + bf.NR + bf.idx[n]] += w * np.dot(g, H)
                    ref[base + 2 * bf.NR + bf.idx[n]] += w * sg * np.dot(g, E)
    assert np.linalg.norm(b - ref) < 1e-12 * np.linalg.norm(ref)
