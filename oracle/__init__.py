"""Oracle for the surface-conductivity-modified PMCHW system (plain FP64).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU-baseline leg
of bench.py may import this package.  It shares no code with the GPU library.

Two operators are defined here, both from the paper's discretisation
(Appendix A, eq19):

* ``dense()`` -- the Galerkin matrix A of the five-current system with
  singularity-subtracted panel quadrature, solved by LU.
* ``PFFT`` -- the precorrected-FFT approximation of the same operator (grid
  projection, lattice convolution with G sampled on the grid, interpolation,
  and exact-minus-grid corrections on near triangle pairs), applied step by
  step; its convolution uses numpy's FFT as a library primitive.

Readings of the paper that these follow are listed in the design notes:
testing of eq13 rotated by n x (so sigma = 0 reduces to PMCHW), pointwise
one-sided fields for the sigma-weighted tests, absorber edges = edges whose
support has sigma > 0 at a quadrature point, 7-point rule everywhere.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np
import scipy.optimize as opt
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scabs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NQ = 7


def build(force: bool = True) -> str:
    """Compile the oracle's C part with gcc (OpenMP, FP64, no -ffast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        zp = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
        L.or_create.restype = P
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_create.argtypes = [C.c_int, dp, C.c_int, ip, ip, C.c_double, C.c_double, C.c_double, C.c_double, C.c_char_p]
        L.or_free.argtypes = [P]
        L.or_error.restype = C.c_char_p
        L.or_error.argtypes = [P]
        L.or_counts.argtypes = [P, ip]
        L.or_get_points.argtypes = [P, dp, dp, dp]
        L.or_get_edges.argtypes = [P, ip, ip, dp, ip, ip]
        L.or_sigma_clear.argtypes = [P]
        L.or_sigma_add_monomial.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double]
        L.or_sigma_add_pwl.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, dp]
        L.or_sigma_pwl_jacobian.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, dp]
        L.or_sigma_set.argtypes = [P, dp]
        L.or_sigma_get.argtypes = [P, dp]
        L.or_layout.restype = C.c_int
        L.or_layout.argtypes = [P, C.c_int]
        L.or_get_layout.argtypes = [P, ip, ip]
        L.or_point_basis.argtypes = [P, dp, dp]
        L.or_static_integrals.argtypes = [dp, dp, dp, dp, dp, dp, dp]
        L.or_dense.restype = C.c_int
        L.or_dense.argtypes = [P, zp]
        L.or_dense_rows.argtypes = [P, C.c_int, ip, zp]
        L.or_local_coo.restype = C.c_long
        L.or_local_coo.argtypes = [P, ip, ip, zp, C.c_long]
        L.or_dipole_field.argtypes = [C.c_double, C.c_double, dp, zp, dp, zp, zp]
        L.or_rhs_dipole.argtypes = [P, dp, zp, C.c_int, zp]
        L.or_incident_at_points.argtypes = [P, dp, zp, C.c_int, zp, zp]
        L.or_point_fields.argtypes = [P, zp, zp, zp]
        L.or_fields_at.argtypes = [P, zp, C.c_int, dp, C.c_int, zp, zp]
        L.or_fields_at_exact.argtypes = [P, zp, C.c_int, dp, C.c_int, zp, zp]
        L.or_source_field.argtypes = [C.c_double, C.c_double, dp, dp, C.c_double, zp, dp, zp, zp]
        L.or_rhs_source.argtypes = [P, dp, dp, C.c_double, zp, C.c_int, zp]
        L.or_stencil.argtypes = [C.c_double, dp, ip, dp, dp]
        L.or_grid_setup.argtypes = [P, C.c_double]
        L.or_grid_weights.argtypes = [P, ip, dp, dp]
        L.or_near_pairs.restype = C.c_long
        L.or_near_pairs.argtypes = [P, C.c_double, ip, C.c_long]
        L.or_singular_radius.restype = C.c_double
        L.or_singular_radius.argtypes = [P]
        L.or_pair_coo.restype = C.c_long
        L.or_pair_coo.argtypes = [P, ip, C.c_long, C.c_int, ip, ip, zp, C.c_long]
        L.or_grid_project.restype = C.c_int
        L.or_grid_project.argtypes = [P, zp, C.c_int, ip, ip, zp]
        L.or_grid_interp_rows.restype = C.c_int
        L.or_grid_interp_rows.argtypes = [P, C.c_int, ip, ip, zp, zp]
        L.or_grid_interp_rows_t.restype = C.c_int
        L.or_grid_interp_rows_t.argtypes = [P, C.c_int, ip, ip, zp, zp]
        L.or_grid_project_t.restype = C.c_int
        L.or_grid_project_t.argtypes = [P, C.c_int, ip, ip, zp, zp]
        L.or_grid_point_fields.restype = C.c_int
        L.or_grid_point_fields.argtypes = [P, C.c_int, ip, ip, zp, zp]
        L.or_point_near_corr.restype = C.c_int
        L.or_point_near_corr.argtypes = [P, zp, ip, C.c_long, zp, zp]
        _lib = L
    return _lib


def static_integrals(r, p0, p1, p2):
    """I0 = int 1/R, I1 = int (r'-r)/R, Ig = int grad_r(1/R) (principal value)."""
    I0 = np.zeros(1)
    I1 = np.zeros(3)
    Ig = np.zeros(3)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    lib().or_static_integrals(f(r), f(p0), f(p1), f(p2), I0, I1, Ig)
    return I0[0], I1, Ig


def dipole_field(k, Z, r0, p, r):
    E = np.zeros(3, complex)
    H = np.zeros(3, complex)
    lib().or_dipole_field(k, Z, np.ascontiguousarray(r0, float), np.ascontiguousarray(p, complex),
                          np.ascontiguousarray(r, float), E, H)
    return E, H


def source_field(k, Z, src, r):
    """Fields of a source (attributes pos, moment, and for a beam direction
    and b > 0) at one point: the dipole, or the dipole at the complex position
    pos - j b direction (Sec. II Gaussian beam), scaled by exp(-k b)."""
    b = float(getattr(src, "b", 0.0))
    bd = b * np.asarray(getattr(src, "direction", (1.0, 0.0, 0.0)), float)
    E = np.zeros(3, complex)
    H = np.zeros(3, complex)
    lib().or_source_field(k, Z, np.ascontiguousarray(src.pos, float), np.ascontiguousarray(bd), b,
                          np.ascontiguousarray(src.moment, complex), np.ascontiguousarray(r, float), E, H)
    return E, H


class Oracle:
    """Dense-Galerkin oracle bound to one mesh, media and sigma profile."""

    def __init__(self, mesh, omega: float, eps_in: float, eps_out: float = 1.0, kappa_s: float = 1.37):
        L = lib()
        err = C.create_string_buffer(256)
        v = np.ascontiguousarray(mesh.verts, dtype=np.float64)
        t = np.ascontiguousarray(mesh.tris, dtype=np.int32)
        b = np.ascontiguousarray(mesh.body, dtype=np.int32)
        self._c = L.or_create(v.shape[0], v.ravel(), t.shape[0], t.ravel(), b, omega, eps_in, eps_out, kappa_s, err)
        if not self._c:
            raise ValueError(err.value.decode())
        self.mesh = mesh
        self.omega, self.eps_in, self.eps_out = omega, eps_in, eps_out
        self.k_e, self.k_i = omega * math.sqrt(eps_out), omega * math.sqrt(eps_in)
        self.Z_e, self.Z_i = 1 / math.sqrt(eps_out), 1 / math.sqrt(eps_in)
        cnt = np.zeros(7, np.int32)
        L.or_counts(self._c, cnt)
        self.nv, self.nt, self.ne, self.nbody = map(int, cnt[:4])
        self.np_ = self.nt * NQ
        self.qp = np.zeros((self.np_, 3))
        self.qw = np.zeros(self.np_)
        self.nrm = np.zeros((self.nt, 3))
        L.or_get_points(self._c, self.qp.ravel(), self.qw, self.nrm.ravel())
        self.ev = np.zeros((self.ne, 2), np.int32)
        self.et = np.zeros((self.ne, 2), np.int32)
        self.elen = np.zeros(self.ne)
        self.tedge = np.zeros((self.nt, 3), np.int32)
        self.tsign = np.zeros((self.nt, 3), np.int32)
        L.or_get_edges(self._c, self.ev.ravel(), self.et.ravel(), self.elen, self.tedge.ravel(), self.tsign.ravel())
        self.N = None
        self.set_sigma([])

    def __del__(self):
        if getattr(self, "_c", None):
            lib().or_free(self._c)
            self._c = None

    # -- sigma and layout ------------------------------------------------
    def set_sigma(self, ends: Sequence, force_all_R: bool = False):
        L = lib()
        L.or_sigma_clear(self._c)
        for e in ends:
            if e.ctrl is not None:
                L.or_sigma_add_pwl(self._c, e.axis, e.x0, e.length, e.direction, len(e.ctrl),
                                   np.ascontiguousarray(e.ctrl, dtype=np.float64))
            else:
                L.or_sigma_add_monomial(self._c, e.axis, e.x0, e.length, e.direction, e.degree, e.sigma0)
        return self._layout(force_all_R)

    def set_sigma_points(self, sigma: np.ndarray, force_all_R: bool = False):
        lib().or_sigma_set(self._c, np.ascontiguousarray(sigma, dtype=np.float64))
        return self._layout(force_all_R)

    def _layout(self, force_all_R):
        L = lib()
        self.N = L.or_layout(self._c, 1 if force_all_R else 0)
        cnt = np.zeros(7, np.int32)
        L.or_counts(self._c, cnt)
        self.NL, self.NR = int(cnt[5]), int(cnt[6])
        self.isR = np.zeros(self.ne, np.int32)
        self.eidx = np.zeros(self.ne, np.int32)
        L.or_get_layout(self._c, self.isR, self.eidx)
        self.sigma = np.zeros(self.np_)
        L.or_sigma_get(self._c, self.sigma)
        return self.N

    def pwl_jacobian(self, end) -> np.ndarray:
        J = np.zeros(self.np_ * len(end.ctrl))
        lib().or_sigma_pwl_jacobian(self._c, end.axis, end.x0, end.length, end.direction, len(end.ctrl), J)
        return J.reshape(self.np_, len(end.ctrl))

    # -- unknown helpers ---------------------------------------------------
    def edge_currents(self, x):
        """(J_e, J_i, M) per edge from the unknown vector (eq10-eq12)."""
        NL, NR = self.NL, self.NR
        Je = np.zeros(self.ne, complex)
        Ji = np.zeros(self.ne, complex)
        M = np.zeros(self.ne, complex)
        l = self.isR == 0
        r = ~l
        il, ir = self.eidx[l], self.eidx[r]
        Je[l] = x[il]
        Ji[l] = -x[il]
        M[l] = x[NL + il]
        Je[r] = x[2 * NL + ir]
        Ji[r] = x[2 * NL + NR + ir]
        M[r] = x[2 * NL + 2 * NR + ir]
        return Je, Ji, M

    # -- operators ---------------------------------------------------------
    def dense(self) -> np.ndarray:
        A = np.zeros((self.N, self.N), complex)
        rc = lib().or_dense(self._c, A.ravel())
        if rc:
            raise RuntimeError(lib().or_error(self._c).decode())
        return A

    def dense_rows(self, rows) -> np.ndarray:
        """Rows of the dense Galerkin matrix (eq19) without assembling the rest:
        the pairs whose test triangle carries one of the rows' edges."""
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.zeros((len(rows), self.N), complex)
        rc = lib().or_dense_rows(self._c, len(rows), rows, out.ravel())
        if rc < 0:
            raise RuntimeError(lib().or_error(self._c).decode())
        return out

    def local_coo(self):
        cap = 64 * self.ne + 64
        ri = np.zeros(cap, np.int32)
        ci = np.zeros(cap, np.int32)
        val = np.zeros(cap, complex)
        n = lib().or_local_coo(self._c, ri, ci, val, cap)
        assert n <= cap
        return sp.coo_matrix((val[:n], (ri[:n], ci[:n])), shape=(self.N, self.N)).tocsr()

    def rhs_dipole(self, dip) -> np.ndarray:
        b = np.zeros(self.N, complex)
        lib().or_rhs_dipole(self._c, np.ascontiguousarray(dip.pos, float), np.ascontiguousarray(dip.moment, complex),
                            int(dip.body), b)
        return b

    def incident_at_points(self, dip):
        E = np.zeros((self.np_, 3), complex)
        H = np.zeros((self.np_, 3), complex)
        lib().or_incident_at_points(self._c, np.ascontiguousarray(dip.pos, float),
                                    np.ascontiguousarray(dip.moment, complex), int(dip.body), E.ravel(), H.ravel())
        return E, H

    def point_fields(self, x):
        """One-sided fields E_e^+ and E_i^- (without E_inc) at all quadrature points."""
        Ee = np.zeros((self.np_, 3), complex)
        Ei = np.zeros((self.np_, 3), complex)
        lib().or_point_fields(self._c, np.ascontiguousarray(x, complex), Ee.ravel(), Ei.ravel())
        return Ee, Ei

    def fields_at(self, x, pts, region: int):
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        E = np.zeros((pts.shape[0], 3), complex)
        H = np.zeros((pts.shape[0], 3), complex)
        lib().or_fields_at(self._c, np.ascontiguousarray(x, complex), pts.shape[0], pts.ravel(), region,
                           E.ravel(), H.ravel())
        return E, H

    def fields_at_exact(self, x, pts, region: int):
        """Scattered fields at points, accurate near the surface (static part
        analytic for triangles within 5 radii of the point)."""
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        E = np.zeros((pts.shape[0], 3), complex)
        H = np.zeros((pts.shape[0], 3), complex)
        lib().or_fields_at_exact(self._c, np.ascontiguousarray(x, complex), pts.shape[0], pts.ravel(), region,
                                 E.ravel(), H.ravel())
        return E, H

    def rhs_source(self, src) -> np.ndarray:
        b = float(getattr(src, "b", 0.0))
        bd = b * np.asarray(getattr(src, "direction", (1.0, 0.0, 0.0)), float)
        out = np.zeros(self.N, complex)
        lib().or_rhs_source(self._c, np.ascontiguousarray(src.pos, float), np.ascontiguousarray(bd), b,
                            np.ascontiguousarray(src.moment, complex), int(src.body), out)
        return out

    def source_fields_at(self, src, pts, region: int):
        """Incident fields of a source at points of a region (zero outside its body)."""
        pts = np.asarray(pts, float).reshape(-1, 3)
        E = np.zeros((pts.shape[0], 3), complex)
        H = np.zeros((pts.shape[0], 3), complex)
        if region == src.body:
            for i, r in enumerate(pts):
                E[i], H[i] = source_field(self.k_i, self.Z_i, src, r)
        return E, H

    def total_fields_at(self, x, src, pts, region: int):
        E, H = self.fields_at_exact(x, pts, region)
        if src is not None:
            Ei, Hi = self.source_fields_at(src, pts, region)
            E, H = E + Ei, H + Hi
        return E, H

    def sigma_profile(self, ends, r) -> float:
        """Conductivity of profile ends (Sec. IV, eq60; hat interpolant) at a point."""
        acc = 0.0
        for e in ends:
            s = e.direction * (r[e.axis] - e.x0) / e.length
            if s < 0:
                continue
            s = min(s, 1.0)
            if getattr(e, "ctrl", None) is None:
                acc += e.sigma0 * (1.0 if e.degree == 0 else s ** e.degree)
            else:
                acc += float(np.interp(s, np.linspace(0.0, 1.0, len(e.ctrl)), e.ctrl))
        return acc

    def magnetic_current_at(self, x, r, body: int):
        """M = E x n at a surface point of `body` (its triangle found by
        barycentric coordinates), from the RWG expansion."""
        v = np.asarray(self.mesh.verts, float)
        t = np.asarray(self.mesh.tris)
        b = np.asarray(self.mesh.body)
        tri = v[t]                                      # (nt, 3, 3)
        n = self.nrm
        h = np.einsum("ta,ta->t", r[None, :] - tri[:, 0], n)
        cand = np.nonzero((np.abs(h) < 1e-7) & (b == body))[0]
        best, bestv = -1, -1e300
        for T in cand:
            P = tri[T]
            area2 = np.dot(np.cross(P[1] - P[0], P[2] - P[0]), n[T])
            lam = [np.dot(np.cross(P[(k + 1) % 3] - r, P[(k + 2) % 3] - r), n[T]) / area2 for k in range(3)]
            if min(lam) > bestv:
                best, bestv = T, min(lam)
        if best < 0 or bestv < -1e-7:
            raise ValueError("point not on the surface of the body")
        _, _, M = self.edge_currents(x)
        P = tri[best]
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        Mv = np.zeros(3, complex)
        for k in range(3):
            e = self.tedge[best, k]
            Mv += self.tsign[best, k] * self.elen[e] / (2 * area) * (r - P[k]) * M[e]
        return Mv

    def poynting_decay(self, x, src, body: int, xpos: float, guide, box, nq: int, ends):
        """Decay rate from Poynting's theorem on the plane x = xpos (Sec. III,
        eq_alpha_power): [int_L' sigma |E_tan|^2 + Re int_L (E x H*).n] /
        [2 Re int_A (E x H*).x]; Gauss-Legendre rules (nq x nq per rectangle of
        A, 2 nq per segment), |E_tan| = |M| on the guide surface."""
        gx, gw = np.polynomial.legendre.leggauss(nq)
        lx, lw = np.polynomial.legendre.leggauss(2 * nq)
        ys = [box[0], guide[0], guide[1], box[1]]
        zs = [box[2], guide[2], guide[3], box[3]]
        fluxA = 0.0
        for iy in range(3):
            for iz in range(3):
                hy, hz = 0.5 * (ys[iy + 1] - ys[iy]), 0.5 * (zs[iz + 1] - zs[iz])
                cy, cz = 0.5 * (ys[iy + 1] + ys[iy]), 0.5 * (zs[iz + 1] + zs[iz])
                Y, Zc = np.meshgrid(cy + hy * gx, cz + hz * gx, indexing="ij")
                W = hy * hz * np.outer(gw, gw)
                pts = np.stack([np.full(Y.size, xpos), Y.ravel(), Zc.ravel()], axis=1)
                region = body if (iy == 1 and iz == 1) else -1
                E, H = self.total_fields_at(x, src, pts, region)
                S = np.cross(E, np.conj(H))
                fluxA += float(np.sum(W.ravel() * S[:, 0].real))
        fluxL = 0.0
        for sd in range(4):
            yside = sd < 2
            lo, hi = (box[2], box[3]) if yside else (box[0], box[1])
            tt = 0.5 * (lo + hi) + 0.5 * (hi - lo) * lx
            if yside:
                pts = np.stack([np.full_like(tt, xpos), np.full_like(tt, box[sd]), tt], axis=1)
            else:
                pts = np.stack([np.full_like(tt, xpos), tt, np.full_like(tt, box[sd])], axis=1)
            nvec = np.zeros(3)
            nvec[1 if yside else 2] = -1.0 if sd % 2 == 0 else 1.0
            E, H = self.total_fields_at(x, src, pts, -1)
            S = np.cross(E, np.conj(H))
            fluxL += float(np.sum(0.5 * (hi - lo) * lw * (S.real @ nvec)))
        perim = 0.0
        for sd in range(4):
            yside = sd < 2
            lo, hi = (guide[2], guide[3]) if yside else (guide[0], guide[1])
            for a in range(2 * nq):
                tpar = 0.5 * (lo + hi) + 0.5 * (hi - lo) * lx[a]
                r = np.array([xpos, guide[sd], tpar]) if yside else np.array([xpos, tpar, guide[sd]])
                Mv = self.magnetic_current_at(x, r, body)
                perim += 0.5 * (hi - lo) * lw[a] * self.sigma_profile(ends, r) * float(np.sum(np.abs(Mv) ** 2))
        return (perim + fluxL) / (2 * fluxA), perim, fluxL, fluxA

    def point_basis(self):
        fv = np.zeros((self.np_, 3, 3))
        fd = np.zeros((self.np_, 3))
        lib().or_point_basis(self._c, fv.ravel(), fd.ravel())
        return fv, fd

    # -- post-processing (powers) ------------------------------------------
    def surface_currents_at_points(self, x):
        Je, Ji, M = self.edge_currents(x)
        fv, _ = self.point_basis()
        tri = np.repeat(np.arange(self.nt), NQ)
        e = self.tedge[tri]                      # (np, 3)
        Jq = np.einsum("pja,pj->pa", fv, Je[e])
        Jiq = np.einsum("pja,pj->pa", fv, Ji[e])
        Mq = np.einsum("pja,pj->pa", fv, M[e])
        return Jq, Jiq, Mq

    def radiated_power(self, x) -> float:
        """P_rad = 1/2 Re oint (E x H*).n = -1/2 Re oint J_e*.(n x M_e) (eq6, eq7)."""
        Jq, _, Mq = self.surface_currents_at_points(x)
        n = np.repeat(self.nrm, NQ, axis=0)
        return float(-0.5 * np.real(np.sum(self.qw * np.einsum("pa,pa->p", np.conj(Jq), np.cross(n, Mq)))))

    def absorbed_power(self, x, dip=None) -> float:
        """P_abs = 1/2 int sigma |E_tan|^2 with the interior-limit field + E_inc."""
        Ee, Ei = self.point_fields(x)
        Et = Ei.copy()
        if dip is not None:
            Einc, _ = self.incident_at_points(dip)
            Et += Einc
        n = np.repeat(self.nrm, NQ, axis=0)
        Et = Et - n * np.einsum("pa,pa->p", n, Et)[:, None]
        return float(0.5 * np.sum(self.qw * self.sigma * np.sum(np.abs(Et) ** 2, axis=1)))

    def dipole_power(self, x, dip) -> float:
        """Power delivered by the dipole: P_0 - 1/2 Re[p* . E_scat(r0)]."""
        k, Z = self.k_i, self.Z_i
        P0 = Z * k * k * np.real(np.vdot(dip.moment, dip.moment)) / (12 * math.pi)
        E, _ = self.fields_at(x, dip.pos[None, :], int(dip.body))
        return float(P0 - 0.5 * np.real(np.vdot(dip.moment, E[0])))

    # -- sigma gradient (adjoint method) --------------------------------------
    def edge_rows(self):
        """(E, H, eq14) row of every edge; eq14 row -1 on sigma-free edges."""
        NL, NR = self.NL, self.NR
        r = self.isR != 0
        rE = np.where(r, 2 * NL + self.eidx, self.eidx)
        rH = np.where(r, 2 * NL + NR + self.eidx, NL + self.eidx)
        r14 = np.where(r, 2 * NL + 2 * NR + self.eidx, -1)
        return rE, rH, r14

    def sigma_gradient_points(self, lam, Ee, Ei, Einc=None) -> np.ndarray:
        """d f / d sigma_q = 2 Re[lam^T (db/dsigma_q - dA/dsigma_q x)] at every
        quadrature point, for A^T lam = g.  sigma enters A only through the
        absorber-edge tests at the points (eq13 rotated by n x and eq14, Appendix
        A): row H_n carries w sigma (f_n x n).E_e^+(q) and row eq14_n carries
        -w sigma f_n.E_i^-(q); b's eq14 row carries w sigma f_n.E_inc(q).  So the
        derivative at q is w_q [t14.(E_inc + E_i^-) - (tH x n).E_e^+] with
        tH = sum lam_H f, t14 = sum lam_14 f over the absorber edges at q."""
        fv, _ = self.point_basis()
        tri = np.repeat(np.arange(self.nt), NQ)
        e = self.tedge[tri]
        isr = (self.isR[e] != 0)
        _, rH, r14 = self.edge_rows()
        lh = np.where(isr, lam[rH[e]], 0)
        l14 = np.where(isr, lam[np.maximum(r14[e], 0)], 0)
        tH = np.einsum("pj,pja->pa", lh, fv)
        t14 = np.einsum("pj,pja->pa", l14, fv)
        n = np.repeat(self.nrm, NQ, axis=0)
        Et = Ei if Einc is None else Ei + Einc
        val = self.qw * (np.einsum("pa,pa->p", t14, Et) - np.einsum("pa,pa->p", np.cross(tH, n), Ee))
        return 2.0 * np.real(val)

    def field_matrix(self, pts, region: int) -> np.ndarray:
        """Q with E(pts) = Q x (scattered field of `region`), rows (point, comp)."""
        pts = np.asarray(pts, float).reshape(-1, 3)
        Q = np.zeros((3 * pts.shape[0], self.N), complex)
        e = np.zeros(self.N, complex)
        for n in range(self.N):
            e[n] = 1.0
            E, _ = self.fields_at(e, pts, region)
            Q[:, n] = E.ravel()
            e[n] = 0.0
        return Q

    # -- pFFT ----------------------------------------------------------------
    def pfft(self, h: float, r_near: float) -> "PFFT":
        return PFFT(self, h, r_near)

    def singular_radius(self) -> float:
        return float(lib().or_singular_radius(self._c))

    def near_pairs(self, r_near: float) -> np.ndarray:
        cap = 256 * self.nt
        while True:
            pairs = np.zeros(2 * cap, np.int32)
            n = lib().or_near_pairs(self._c, r_near, pairs, cap)
            if n <= cap:
                return pairs[: 2 * n].reshape(-1, 2)
            cap = n

    def pair_coo(self, pairs: np.ndarray, mode: int):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32)
        cap = 100 * pairs.shape[0] + 64
        ri = np.zeros(cap, np.int32)
        ci = np.zeros(cap, np.int32)
        val = np.zeros(cap, complex)
        n = lib().or_pair_coo(self._c, pairs.ravel(), pairs.shape[0], mode, ri, ci, val, cap)
        assert n <= cap, (n, cap)
        return sp.coo_matrix((val[:n], (ri[:n], ci[:n])), shape=(self.N, self.N)).tocsr()


def _grid_kernel_hat(k: float, h: float, n: Sequence[int]) -> np.ndarray:
    """FFT of the circulant embedding (size 2n per axis) of H(d) = G(h|d|), H(0) = 0."""
    axes = []
    for m in n:
        i = np.arange(2 * m)
        d = np.where(i < m, i, i - 2 * m).astype(np.float64)
        d[m] = np.inf   # offset +-m is never needed
        axes.append(d)
    dx, dy, dz = np.meshgrid(*axes, indexing="ij")
    R = h * np.sqrt(dx * dx + dy * dy + dz * dz)
    with np.errstate(invalid="ignore", divide="ignore"):
        Hk = np.exp(-1j * k * R) / (4 * math.pi * R)
    Hk[~np.isfinite(R)] = 0
    Hk[0, 0, 0] = 0
    return np.fft.fftn(Hk)


class PFFT:
    """Precorrected-FFT operator A~ = grid(P, H, I) + (A_exact - A_grid)|near + local."""

    def __init__(self, o: Oracle, h: float, r_near: float):
        self.o = o
        self.h = h
        self.r_near = r_near
        srad = o.singular_radius()
        if not r_near > srad:
            raise ValueError("r_near %.6g must exceed the singular-pair radius %.6g" % (r_near, srad))
        L = lib()
        L.or_grid_setup(o._c, h)
        npn = o.np_
        self.anchor = np.zeros((npn, 3), np.int32)
        w = np.zeros(npn * 27)
        gd = np.zeros(npn * 81)
        L.or_grid_weights(o._c, self.anchor.ravel(), w, gd)
        tri_body = o.mesh.body
        pb = np.repeat(tri_body, NQ)
        self.grids = []   # (which, origin, dims, k)
        for which in [-1] + list(range(o.nbody)):
            sel = np.ones(npn, bool) if which < 0 else (pb == which)
            lo = self.anchor[sel].min(axis=0) - 1
            hi = self.anchor[sel].max(axis=0) + 1
            dims = (hi - lo + 1).astype(np.int32)
            k = o.k_e if which < 0 else o.k_i
            self.grids.append((which, lo.astype(np.int32), dims, k, _grid_kernel_hat(k, h, dims)))
        self.pairs = o.near_pairs(r_near)
        self.C_near = o.pair_coo(self.pairs, 0) + o.local_coo()

    def grid_apply(self, x: np.ndarray) -> np.ndarray:
        """grid part only: interpolate(H * project(x)) tested into rows"""
        o = self.o
        L = lib()
        x = np.ascontiguousarray(x, complex)
        y = np.zeros(o.N, complex)
        for which, lo, dims, k, Hhat in self.grids:
            G = int(np.prod(dims))
            Q = np.zeros(8 * G, complex)
            rc = L.or_grid_project(o._c, x, which, lo, dims, Q)
            assert rc == 0
            Q = Q.reshape(8, *dims)
            Phi = np.empty_like(Q)
            n0, n1, n2 = dims
            for f in range(8):
                Qp = np.zeros((2 * n0, 2 * n1, 2 * n2), complex)
                Qp[:n0, :n1, :n2] = Q[f]
                Phi[f] = np.fft.ifftn(np.fft.fftn(Qp) * Hhat)[:n0, :n1, :n2]
            rc = L.or_grid_interp_rows(o._c, which, lo, dims, np.ascontiguousarray(Phi.ravel()), y)
            assert rc == 0
        return y

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.grid_apply(x) + self.C_near @ x

    def _conv(self, Hhat, dims, Q):
        n0, n1, n2 = dims
        Phi = np.empty_like(Q)
        for f in range(8):
            Qp = np.zeros((2 * n0, 2 * n1, 2 * n2), complex)
            Qp[:n0, :n1, :n2] = Q[f]
            Phi[f] = np.fft.ifftn(np.fft.fftn(Qp) * Hhat)[:n0, :n1, :n2]
        return Phi

    def grid_apply_t(self, z: np.ndarray) -> np.ndarray:
        """transpose of grid_apply: test-side sources (value and gradient
        weights), the same symmetric lattice convolution, then the transposed
        projection back to unknowns"""
        o = self.o
        L = lib()
        z = np.ascontiguousarray(z, complex)
        y = np.zeros(o.N, complex)
        for which, lo, dims, k, Hhat in self.grids:
            G = int(np.prod(dims))
            S = np.zeros(8 * G, complex)
            assert L.or_grid_interp_rows_t(o._c, which, lo, dims, z, S) == 0
            Phi = self._conv(Hhat, dims, S.reshape(8, *dims))
            assert L.or_grid_project_t(o._c, which, lo, dims, np.ascontiguousarray(Phi.ravel()), y) == 0
        return y

    def rmatvec(self, z: np.ndarray) -> np.ndarray:
        """A~^T z"""
        return self.grid_apply_t(z) + self.C_near.T @ z

    def solve_t(self, g: np.ndarray, tol: float = 1e-12, restart: int = 200, maxiter: int = 50) -> np.ndarray:
        """A~^T lam = g by GMRES, preconditioned by the transposed sparse LU of
        the exact near-field part; true residual checked."""
        N = self.o.N
        near = self.o.pair_coo(self.pairs, 1) + self.o.local_coo()
        lu = spla.splu(near.T.tocsc())
        M = spla.LinearOperator((N, N), matvec=lu.solve, dtype=complex)
        op = spla.LinearOperator((N, N), matvec=self.rmatvec, dtype=complex)
        lam, info = spla.gmres(op, g, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter, M=M)
        res = np.linalg.norm(self.rmatvec(lam) - g) / np.linalg.norm(g)
        if info != 0 or res > 100 * tol:
            raise RuntimeError("oracle adjoint GMRES did not converge (info=%d, residual %.2e)" % (info, res))
        return lam

    def point_fields(self, x: np.ndarray):
        """One-sided pointwise fields of this operator at every quadrature point:
        grid interpolation, plus exact-minus-grid of the near triangle pairs,
        plus the residue 1/2 n x M (exterior: E_e^+, interior: E_i^-)."""
        o = self.o
        L = lib()
        x = np.ascontiguousarray(x, complex)
        Ee = np.zeros((o.np_, 3), complex)
        Ei = np.zeros((o.np_, 3), complex)
        for which, lo, dims, k, Hhat in self.grids:
            G = int(np.prod(dims))
            Q = np.zeros(8 * G, complex)
            assert L.or_grid_project(o._c, x, which, lo, dims, Q) == 0
            Phi = self._conv(Hhat, dims, Q.reshape(8, *dims))
            tgt = Ee if which < 0 else Ei
            assert L.or_grid_point_fields(o._c, which, lo, dims, np.ascontiguousarray(Phi.ravel()), tgt.ravel()) == 0
        pairs = np.ascontiguousarray(self.pairs, dtype=np.int32)
        assert L.or_point_near_corr(o._c, x, pairs.ravel(), pairs.shape[0], Ee.ravel(), Ei.ravel()) == 0
        _, _, Mq = o.surface_currents_at_points(x)
        n = np.repeat(o.nrm, NQ, axis=0)
        res = 0.5 * np.cross(n, Mq)
        return Ee + res, Ei + res

    def solve(self, b: np.ndarray, tol: float = 1e-12, restart: int = 200, maxiter: int = 50) -> np.ndarray:
        """GMRES on A~ preconditioned by a sparse LU of its exact near-field
        part (the preconditioner changes the iteration path, not the answer);
        the true residual is checked at the end."""
        N = self.o.N
        near = self.o.pair_coo(self.pairs, 1) + self.o.local_coo()
        lu = spla.splu(near.tocsc())
        M = spla.LinearOperator((N, N), matvec=lu.solve, dtype=complex)
        op = spla.LinearOperator((N, N), matvec=self.matvec, dtype=complex)
        x, info = spla.gmres(op, b, rtol=tol, atol=0.0, restart=restart, maxiter=maxiter, M=M)
        res = np.linalg.norm(self.matvec(x) - b) / np.linalg.norm(b)
        if info != 0 or res > 100 * tol:
            raise RuntimeError("oracle GMRES did not converge (info=%d, residual %.2e)" % (info, res))
        return x


def lu_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    lu, piv = sla.lu_factor(A)
    return sla.lu_solve((lu, piv), b)


def gmres_dense(A: np.ndarray, b: np.ndarray, tol: float = 1e-10, max_steps: Optional[int] = None) -> np.ndarray:
    """Full (unrestarted) GMRES on the dense matrix (the solver the paper
    names for eq19): Arnoldi with classical Gram-Schmidt applied twice,
    Givens rotations on the Hessenberg matrix, stop when the updated residual
    norm is at most tol ||b||, then solve the triangular system."""
    n = A.shape[0]
    m = n if max_steps is None else min(n, max_steps)
    beta = np.linalg.norm(b)
    V = np.zeros((n, m + 1), complex)
    R = np.zeros((m + 1, m), complex)
    cs = np.zeros(m, complex)
    sn = np.zeros(m, complex)
    g = np.zeros(m + 1, complex)
    g[0] = beta
    V[:, 0] = b / beta
    j = 0
    for j in range(m):
        w = A @ V[:, j]
        h = V[:, : j + 1].conj().T @ w
        w = w - V[:, : j + 1] @ h
        h2 = V[:, : j + 1].conj().T @ w
        w = w - V[:, : j + 1] @ h2
        col = np.zeros(j + 2, complex)
        col[: j + 1] = h + h2
        col[j + 1] = np.linalg.norm(w)
        for i in range(j):
            a, c = col[i], col[i + 1]
            col[i] = cs[i] * a + sn[i] * c
            col[i + 1] = -np.conj(sn[i]) * a + cs[i] * c
        den = math.hypot(abs(col[j]), abs(col[j + 1]))
        if den == 0:
            cs[j], sn[j] = 1.0, 0.0
        elif col[j] == 0:
            cs[j], sn[j] = 0.0, np.conj(col[j + 1]) / abs(col[j + 1])
        else:
            cs[j] = abs(col[j]) / den
            sn[j] = (col[j] / abs(col[j])) * np.conj(col[j + 1]) / den
        hn = col[j + 1]
        col[j] = cs[j] * col[j] + sn[j] * col[j + 1]
        col[j + 1] = 0
        R[: j + 2, j] = col
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        if abs(g[j + 1]) <= tol * beta or hn == 0:
            break
        V[:, j + 1] = w / hn
    k = j + 1
    y = sla.solve_triangular(R[:k, :k], g[:k])
    return V[:, :k] @ y


def monitor_weights(xs: np.ndarray, beta: float) -> np.ndarray:
    """Least-squares fit of samples E(x_k) to a e^{-j beta x} + b e^{+j beta x}:
    returns w with b = w . E (the reflected amplitude)."""
    P = np.stack([np.exp(-1j * beta * xs), np.exp(1j * beta * xs)], axis=1)
    return np.linalg.pinv(P)[1]


# ---------------------------------------------------------------------------
# field post-processing on samples (Sec. I, Table I; Sec. III)
# ---------------------------------------------------------------------------
def swr(E):
    """Standing-wave ratio max|E| / min|E| and the transmission-line
    reflection coefficient (SWR - 1) / (SWR + 1)."""
    a = np.abs(np.asarray(E))
    s = float(a.max() / a.min())
    return s, (s - 1) / (s + 1)


def standing_wave_fit(xs, E, beta_lo: float, beta_hi: float):
    """Least-squares E = a e^{-j beta x} + c e^{+j beta x}; beta fixed or the
    residual's minimiser in [beta_lo, beta_hi] (dense scan, then bounded
    scalar minimisation).  Returns (beta, |c/a|, relative residual)."""
    xs = np.asarray(xs, float)
    E = np.asarray(E, complex)

    def fit(beta):
        P = np.stack([np.exp(-1j * beta * xs), np.exp(1j * beta * xs)], axis=1)
        coef, *_ = np.linalg.lstsq(P, E, rcond=None)
        return coef, float(np.linalg.norm(E - P @ coef) / np.linalg.norm(E))

    if beta_hi > beta_lo:
        grid = np.linspace(beta_lo, beta_hi, 2001)
        res = [fit(b)[1] for b in grid]
        i = int(np.argmin(res))
        lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
        beta = float(opt.minimize_scalar(lambda b: fit(b)[1], bounds=(lo, hi), method="bounded",
                                         options={"xatol": 1e-12}).x)
    else:
        beta = float(beta_lo)
    coef, r = fit(beta)
    return beta, float(abs(coef[1]) / abs(coef[0])), r


def decay_fit(xs, E):
    """alpha, beta of E ~ exp(-(alpha + j beta) x): straight-line fits of
    ln|E| and of the unwrapped phase."""
    xs = np.asarray(xs, float)
    E = np.asarray(E, complex)
    sa, _ = np.polyfit(xs, np.log(np.abs(E)), 1)
    sp, _ = np.polyfit(xs, np.unwrap(np.angle(E)), 1)
    return float(-sa), float(-sp)
