"""Python binding of libscabs (argument marshalling only).

Every computation runs in the HIP library; PyTorch provides device memory and
the stream.  The library must be built first (``__graft_entry__.build()`` or
``python paper_1004_5076_amd/build.py``); importing works without it, but
every call that needs it raises ``RuntimeError`` -- there is no CPU fallback.

Method names mirror the C ABI in include/scabs.h (``scabs_<name>``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscabs.so")

SCABS_OK = 0
SCABS_E_ARG, SCABS_E_MESH, SCABS_E_STATE, SCABS_E_HIP, SCABS_E_OOM, SCABS_E_NOCONV, SCABS_E_NAN = -1, -2, -3, -4, -5, -6, -7
SCABS_FP64, SCABS_FP32, SCABS_MIXED = 0, 1, 2
SCABS_PRODUCT_PFFT, SCABS_PRODUCT_TOEPLITZ = 0, 1
EXPORTED = ["scabs_create", "scabs_set_graphs", "scabs_set_mesh", "scabs_set_media", "scabs_sigma_clear", "scabs_sigma_add_monomial",
            "scabs_sigma_add_pwl", "scabs_set_sigma_points", "scabs_build", "scabs_info", "scabs_layout", "scabs_rhs_dipole", "scabs_matvec",
            "scabs_solve", "scabs_matvec_transpose", "scabs_solve_transpose", "scabs_precond_apply", "scabs_incident_dipole_points",
            "scabs_point_fields", "scabs_eval_field", "scabs_eval_field_noalloc", "scabs_dipole_field", "scabs_gradient", "scabs_eval_field_transpose", "scabs_sigma_params",
            "scabs_sigma_gradient", "scabs_profile_begin", "scabs_profile_end", "scabs_profile_mask", "scabs_profile_bytes",
            "scabs_last_error", "scabs_destroy", "scabs_eval_field_exact", "scabs_rhs_source",
            "scabs_incident_source_points", "scabs_source_field", "scabs_swr", "scabs_standing_wave_fit",
            "scabs_decay_fit", "scabs_poynting_decay", "scabs_solve_batched", "scabs_autotune", "scabs_set_tune"]
STAGES = ["unpack64", "project64", "fft64", "interp64", "near64", "unpack32", "project32", "fft32", "interp32",
          "near32", "precond", "ortho", "precond_t", "xline32", "gather32", "pcgather32", "toeapply32", "toeapply64",
          "toeproduct32", "toeproduct64", "toeapplyt32", "toeapplyt64"]


class ScabsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"scabs error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("h", C.c_double), ("r_near", C.c_double), ("kappa_s", C.c_double), ("device", C.c_int),
                ("stream", C.c_void_p), ("precond", C.c_int), ("pc_cell", C.c_double), ("pc_overlap", C.c_double),
                ("product", C.c_int)]


class Info(C.Structure):
    _fields_ = [("N", C.c_int64), ("NL", C.c_int64), ("NR", C.c_int64), ("n_edges", C.c_int64),
                ("n_tris", C.c_int64), ("n_points", C.c_int64), ("n_bodies", C.c_int64),
                ("n_near_pairs", C.c_int64), ("nnz_near", C.c_int64), ("grid_phys", C.c_int64 * 3),
                ("grid_fft", C.c_int64 * 3), ("nnz_near_r", C.c_int64), ("n_clusters", C.c_int64),
                ("precond_entries", C.c_int64), ("device_bytes", C.c_int64), ("precond_ext_entries", C.c_int64),
                ("product", C.c_int64), ("rings", C.c_int64), ("circulant_length", C.c_int64),
                ("ring_edges", C.c_int64), ("ring_triangles", C.c_int64), ("nnz_nonperiodic", C.c_int64),
                ("toeplitz_table_bytes", C.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["grid_phys"] = list(self.grid_phys)
        d["grid_fft"] = list(self.grid_fft)
        return d


class Source(C.Structure):
    """scabs_source: a point dipole (b = 0) or the complex-source-point beam
    along +dir with waist at pos and Rayleigh distance b."""
    _fields_ = [("pos", C.c_double * 3), ("dir", C.c_double * 3), ("b", C.c_double), ("moment", C.c_double * 6),
                ("body", C.c_int32), ("pad", C.c_int32)]

    @staticmethod
    def make(pos, moment, body: int = 0, direction=(1.0, 0.0, 0.0), b: float = 0.0) -> "Source":
        s = Source()
        m = np.asarray(moment, dtype=np.complex128)
        for a in range(3):
            s.pos[a] = float(pos[a])
            s.dir[a] = float(direction[a])
            s.moment[2 * a] = float(m[a].real)
            s.moment[2 * a + 1] = float(m[a].imag)
        s.b = float(b)
        s.body = int(body)
        return s


class TuneRecord(C.Structure):
    _fields_ = [("nrhs", C.c_int32), ("apply_form", C.c_int32), ("groups", C.c_int32), ("lines", C.c_int32),
                ("us", C.c_double), ("chosen", C.c_int32), ("overlap", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("outer_iters", C.c_int), ("inner_iters", C.c_int), ("matvecs64", C.c_int),
                ("matvecs32", C.c_int), ("rel_residual", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load() -> C.CDLL:
    """Load libscabs.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.scabs_create.argtypes = [C.POINTER(P), C.POINTER(Opts)]
    L.scabs_set_mesh.argtypes = [P, dp, C.c_int64, C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int32)]
    L.scabs_set_media.argtypes = [P, C.c_double, C.c_double, C.c_double]
    L.scabs_sigma_clear.argtypes = [P]
    L.scabs_sigma_add_monomial.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double]
    L.scabs_sigma_add_pwl.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, dp]
    L.scabs_build.argtypes = [P]
    L.scabs_info.argtypes = [P, C.POINTER(Info)]
    L.scabs_layout.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.scabs_rhs_dipole.argtypes = [P, dp, dp, C.c_int, P]
    L.scabs_matvec.argtypes = [P, P, P, C.c_int, C.c_int]
    L.scabs_solve.argtypes = [P, P, P, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(SolveInfo)]
    L.scabs_matvec_transpose.argtypes = [P, P, P, C.c_int, C.c_int]
    L.scabs_solve_transpose.argtypes = [P, P, P, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int,
                                        C.POINTER(SolveInfo)]
    L.scabs_precond_apply.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int]
    L.scabs_incident_dipole_points.argtypes = [P, dp, dp, C.c_int, P]
    L.scabs_point_fields.argtypes = [P, P, P, P]
    L.scabs_eval_field.argtypes = [P, P, dp, C.c_int, C.c_int, P, P]
    L.scabs_eval_field_noalloc.argtypes = [P, P, dp, C.c_int, C.c_int, P, P]
    L.scabs_dipole_field.argtypes = [P, dp, dp, C.c_int, dp, C.c_int, C.c_int, P, P]
    L.scabs_gradient.argtypes = [P, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int, P, dp, C.POINTER(SolveInfo)]
    L.scabs_set_sigma_points.argtypes = [P, dp, C.c_int64]
    L.scabs_eval_field_transpose.argtypes = [P, dp, C.c_int, C.c_int, P, P]
    L.scabs_sigma_params.argtypes = [P, C.POINTER(C.c_int64)]
    L.scabs_sigma_gradient.argtypes = [P, P, P, P, P, dp]
    L.scabs_profile_begin.argtypes = [P]
    L.scabs_profile_end.argtypes = [P, dp, C.POINTER(C.c_int64)]
    L.scabs_profile_bytes.argtypes = [P, dp]
    L.scabs_profile_mask.argtypes = [P, C.c_uint32]
    L.scabs_last_error.restype = C.c_char_p
    L.scabs_eval_field_exact.argtypes = [P, P, dp, C.c_int, C.c_int, P, P]
    L.scabs_rhs_source.argtypes = [P, C.POINTER(Source), P]
    L.scabs_incident_source_points.argtypes = [P, C.POINTER(Source), P]
    L.scabs_source_field.argtypes = [P, C.POINTER(Source), dp, C.c_int, C.c_int, P, P]
    L.scabs_swr.argtypes = [dp, C.c_int, dp]
    L.scabs_standing_wave_fit.argtypes = [dp, dp, C.c_int, C.c_double, C.c_double, dp]
    L.scabs_decay_fit.argtypes = [dp, dp, C.c_int, dp]
    L.scabs_poynting_decay.argtypes = [P, P, C.POINTER(Source), C.c_int, C.c_double, dp, dp, C.c_int, dp]
    L.scabs_solve_batched.argtypes = [C.POINTER(P), C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(C.c_int),
                                      C.c_double, C.c_int, C.c_int, C.c_int, C.POINTER(C.POINTER(SolveInfo))]
    L.scabs_autotune.argtypes = [P, C.c_int, C.POINTER(TuneRecord), C.c_int, C.POINTER(C.c_int)]
    L.scabs_set_tune.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
    L.scabs_set_graphs.argtypes = [P, C.c_int]
    L.scabs_last_error.argtypes = [P]
    L.scabs_destroy.argtypes = [P]
    _lib = L
    return L


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


class Context:
    """One library context: a mesh, media, conductivity profile and grid."""

    def __init__(self, h: float, r_near: float, kappa_s: float = 1.37, device: int = 0, stream=None,
                 precond: int = 1, pc_cell: float = -1.0, pc_overlap: float = -1.0, product: int = 0):
        import torch
        L = load()
        self._L = L
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        o = Opts(h, r_near, kappa_s, device, C.c_void_p(stream.cuda_stream), precond, pc_cell, pc_overlap, product)
        self._c = C.c_void_p()
        self._check(L.scabs_create(C.byref(self._c), C.byref(o)))
        self.N = None

    def _check(self, rc: int):
        if rc != SCABS_OK:
            msg = self._L.scabs_last_error(self._c).decode() if getattr(self, "_c", None) else ""
            raise ScabsError(rc, msg)

    def close(self):
        if getattr(self, "_c", None) and self._c.value:
            self._L.scabs_destroy(self._c)
            self._c = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setters (host data, copied) ------------------------------------------
    def set_mesh(self, verts, tris, body=None):
        v, vp = _f64(verts)
        t, tp = _i32(tris)
        b, bp = _i32(np.zeros(t.shape[0]) if body is None else body)
        self._check(self._L.scabs_set_mesh(self._c, vp, v.shape[0], tp, t.shape[0], bp))

    def set_media(self, omega: float, eps_out: float, eps_in: float):
        self._check(self._L.scabs_set_media(self._c, omega, eps_out, eps_in))

    def sigma_clear(self):
        self._check(self._L.scabs_sigma_clear(self._c))

    def sigma_add_monomial(self, axis, x0, length, direction, degree, sigma0):
        self._check(self._L.scabs_sigma_add_monomial(self._c, axis, x0, length, direction, degree, sigma0))

    def sigma_add_pwl(self, axis, x0, length, direction, ctrl):
        c, cp = _f64(ctrl)
        self._check(self._L.scabs_sigma_add_pwl(self._c, axis, x0, length, direction, c.shape[0], cp))

    def set_sigma_points(self, sigma_q):
        """Raw conductivity per quadrature point (7 per triangle, rule order)."""
        a, ap = _f64(sigma_q)
        self._check(self._L.scabs_set_sigma_points(self._c, ap, a.shape[0]))

    def set_sigma(self, ends: Iterable):
        self.sigma_clear()
        for e in ends:
            if getattr(e, "ctrl", None) is not None:
                self.sigma_add_pwl(e.axis, e.x0, e.length, e.direction, e.ctrl)
            else:
                self.sigma_add_monomial(e.axis, e.x0, e.length, e.direction, e.degree, e.sigma0)

    def build(self):
        self._check(self._L.scabs_build(self._c))
        self.N = self.info()["N"]

    # -- queries ----------------------------------------------------------------
    def info(self) -> dict:
        i = Info()
        self._check(self._L.scabs_info(self._c, C.byref(i)))
        return i.as_dict()

    def layout(self):
        ne = self.info()["n_edges"]
        isr = np.zeros(ne, np.int32)
        idx = np.zeros(ne, np.int32)
        self._check(self._L.scabs_layout(self._c, isr.ctypes.data_as(C.POINTER(C.c_int32)),
                                         idx.ctypes.data_as(C.POINTER(C.c_int32))))
        return isr, idx

    # -- device operations --------------------------------------------------------
    def _dev(self, t, nrhs_ok=True):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
            raise TypeError("expected a contiguous complex128 CUDA tensor")
        if t.shape[-1] != self.N:
            raise ValueError(f"last dimension must be N={self.N}")
        # a lazily conjugated view shares the unconjugated storage: materialise it
        return t.resolve_conj() if t.is_conj() else t

    def rhs_dipole(self, pos, moment, body: int = 0):
        import torch
        b = torch.empty(self.N, dtype=torch.complex128, device=self.device)
        p, pp = _f64(pos)
        m = np.asarray(moment, dtype=np.complex128)
        mm, mp = _f64(np.stack([m.real, m.imag], axis=1).ravel())
        self._check(self._L.scabs_rhs_dipole(self._c, pp, mp, int(body), C.c_void_p(b.data_ptr())))
        return b

    def matvec(self, x, prec: int = SCABS_FP64, transpose: bool = False):
        import torch
        x = self._dev(x)
        y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        fn = self._L.scabs_matvec_transpose if transpose else self._L.scabs_matvec
        self._check(fn(self._c, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs, prec))
        return y

    def precond_apply(self, x, prec: int = SCABS_FP64, transpose: bool = False):
        """y = M x or M^T x with the Schwarz preconditioner (one or a stack of vectors)."""
        import torch
        x = self._dev(x)
        y = torch.empty_like(x)
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        self._check(self._L.scabs_precond_apply(self._c, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs,
                                                prec, int(bool(transpose))))
        return y

    def incident_dipole_points(self, pos, moment, body: int = 0):
        import torch
        npt = self.info()["n_points"]
        E = torch.empty((npt, 3), dtype=torch.complex128, device=self.device)
        p, pp = _f64(pos)
        m = np.asarray(moment, dtype=np.complex128)
        mm, mp = _f64(np.stack([m.real, m.imag], axis=1).ravel())
        self._check(self._L.scabs_incident_dipole_points(self._c, pp, mp, int(body), C.c_void_p(E.data_ptr())))
        return E

    def point_fields(self, x):
        import torch
        x = self._dev(x)
        npt = self.info()["n_points"]
        Ee = torch.empty((npt, 3), dtype=torch.complex128, device=self.device)
        Ei = torch.empty_like(Ee)
        self._check(self._L.scabs_point_fields(self._c, C.c_void_p(x.data_ptr()), C.c_void_p(Ee.data_ptr()),
                                               C.c_void_p(Ei.data_ptr())))
        return Ee, Ei

    def eval_field(self, x, pts, region: int):
        import torch
        x = self._dev(x)
        p, pp = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        E = torch.empty((p.shape[0], 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E)
        self._check(self._L.scabs_eval_field(self._c, C.c_void_p(x.data_ptr()), pp, p.shape[0], int(region),
                                             C.c_void_p(E.data_ptr()), C.c_void_p(H.data_ptr())))
        return E, H

    def eval_field_exact(self, x, pts, region: int):
        """Scattered fields at points of a region, accurate near the surface."""
        import torch
        x = self._dev(x)
        p, pp = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        E = torch.empty((p.shape[0], 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E)
        self._check(self._L.scabs_eval_field_exact(self._c, C.c_void_p(x.data_ptr()), pp, p.shape[0], int(region),
                                                   C.c_void_p(E.data_ptr()), C.c_void_p(H.data_ptr())))
        return E, H

    def rhs_source(self, src: Source):
        import torch
        b = torch.empty(self.N, dtype=torch.complex128, device=self.device)
        self._check(self._L.scabs_rhs_source(self._c, C.byref(src), C.c_void_p(b.data_ptr())))
        return b

    def incident_source_points(self, src: Source):
        import torch
        npt = self.info()["n_points"]
        E = torch.empty((npt, 3), dtype=torch.complex128, device=self.device)
        self._check(self._L.scabs_incident_source_points(self._c, C.byref(src), C.c_void_p(E.data_ptr())))
        return E

    def source_field(self, src: Source, pts, region: int):
        import torch
        p, pp = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        E = torch.empty((p.shape[0], 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E)
        self._check(self._L.scabs_source_field(self._c, C.byref(src), pp, p.shape[0], int(region),
                                               C.c_void_p(E.data_ptr()), C.c_void_p(H.data_ptr())))
        return E, H

    def autotune(self, reps: int = 3):
        """Time the block-Toeplitz product's launch choices and keep the
        fastest per class (fewer than 8 / 8 vectors); returns the records."""
        recs = (TuneRecord * 64)()
        n = C.c_int(0)
        self._check(self._L.scabs_autotune(self._c, int(reps), recs, 64, C.byref(n)))
        return [recs[i].as_dict() for i in range(min(n.value, 64))]

    def set_graphs(self, on: bool):
        """scabs_set_graphs: replay each Arnoldi step's launches from a HIP graph."""
        self._check(self._L.scabs_set_graphs(self._c, int(bool(on))))

    def set_tune(self, nrhs_class: int, form: int, groups: int, lines: int, overlap: int = 0):
        self._check(self._L.scabs_set_tune(self._c, int(nrhs_class), int(form), int(groups), int(lines),
                                           int(overlap)))

    def poynting_decay(self, x, src: Optional[Source], body: int, xpos: float, guide, box, nq: int = 8):
        """Decay rate from Poynting's theorem on the plane x = xpos; returns
        (alpha, perimeter integral, boundary flux, flux through the box)."""
        x = self._dev(x)
        g, gp = _f64(np.asarray(guide, dtype=np.float64))
        bx, bp = _f64(np.asarray(box, dtype=np.float64))
        out = np.zeros(4)
        self._check(self._L.scabs_poynting_decay(self._c, C.c_void_p(x.data_ptr()),
                                                 C.byref(src) if src is not None else None, int(body), float(xpos),
                                                 gp, bp, int(nq), out.ctypes.data_as(C.POINTER(C.c_double))))
        return tuple(float(v) for v in out)

    def dipole_field(self, pos, moment, body: int, pts, region: int):
        """Closed-form fields of the dipole at points of a region (zero outside
        the dipole's body)."""
        import torch
        p, pp = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        pa, posp = _f64(np.asarray(pos, dtype=np.float64))
        m = np.asarray(moment, dtype=np.complex128)
        ma, mp = _f64(np.stack([m.real, m.imag], axis=1).ravel())
        E = torch.empty((p.shape[0], 3), dtype=torch.complex128, device=self.device)
        H = torch.empty_like(E)
        self._check(self._L.scabs_dipole_field(self._c, posp, mp, int(body), pp, p.shape[0], int(region),
                                               C.c_void_p(E.data_ptr()), C.c_void_p(H.data_ptr())))
        return E, H

    def gradient(self, x, g, einc=None, tol: float = 1e-10, max_iter: int = 4000, restart: int = 200,
                 mode: int = SCABS_FP64):
        """One call: adjoint solve A^T lam = g, then the sigma gradient.
        Returns (d f/d sigma per point [device], d f/d parameters [numpy], solve info)."""
        import torch
        x = self._dev(x)
        g = self._dev(g)
        npt = self.info()["n_points"]
        dfds = torch.empty(npt, dtype=torch.float64, device=self.device)
        dfdp = np.zeros(max(self.sigma_params(), 1))
        if einc is not None:
            einc = einc.resolve_conj().contiguous()
        ep = C.c_void_p(einc.data_ptr()) if einc is not None else C.c_void_p()
        si = SolveInfo()
        self._check(self._L.scabs_gradient(self._c, C.c_void_p(x.data_ptr()), C.c_void_p(g.data_ptr()), ep, tol,
                                           max_iter, restart, mode, C.c_void_p(dfds.data_ptr()),
                                           dfdp.ctypes.data_as(C.POINTER(C.c_double)), C.byref(si)))
        return dfds, dfdp[: self.sigma_params()], si.as_dict()

    def eval_field_noalloc(self, x, pts, region: int, E=None, H=None):
        """scabs_eval_field through the entry point that allocates nothing
        (outputs E, H may be passed in, shape (npts, 3) complex128)."""
        import torch
        x = self._dev(x)
        p, pp = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        if E is None:
            E = torch.empty((p.shape[0], 3), dtype=torch.complex128, device=self.device)
        if H is None:
            H = torch.empty_like(E)
        self._check(self._L.scabs_eval_field_noalloc(self._c, C.c_void_p(x.data_ptr()), pp, p.shape[0], int(region),
                                                     C.c_void_p(E.data_ptr()), C.c_void_p(H.data_ptr())))
        return E, H

    def eval_field_transpose(self, pts, region: int, wE):
        import torch
        p, pp = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        wE = wE.to(device=self.device, dtype=torch.complex128).resolve_conj().contiguous()
        if tuple(wE.shape) != (p.shape[0], 3):
            raise ValueError("wE must have shape (npts, 3)")
        y = torch.empty(self.N, dtype=torch.complex128, device=self.device)
        self._check(self._L.scabs_eval_field_transpose(self._c, pp, p.shape[0], int(region),
                                                       C.c_void_p(wE.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def sigma_params(self) -> int:
        n = C.c_int64()
        self._check(self._L.scabs_sigma_params(self._c, C.byref(n)))
        return n.value

    def sigma_gradient(self, x, lam, einc=None):
        """(d f/d sigma per quadrature point [device], d f/d profile parameters [numpy])."""
        import torch
        x = self._dev(x)
        lam = self._dev(lam)
        npt = self.info()["n_points"]
        dfds = torch.empty(npt, dtype=torch.float64, device=self.device)
        dfdp = np.zeros(max(self.sigma_params(), 1))
        if einc is not None:
            einc = einc.resolve_conj().contiguous()
        ep = C.c_void_p(einc.data_ptr()) if einc is not None else C.c_void_p()
        self._check(self._L.scabs_sigma_gradient(self._c, C.c_void_p(x.data_ptr()), C.c_void_p(lam.data_ptr()), ep,
                                                 C.c_void_p(dfds.data_ptr()),
                                                 dfdp.ctypes.data_as(C.POINTER(C.c_double))))
        return dfds, dfdp[: self.sigma_params()]

    def profile_begin(self):
        self._check(self._L.scabs_profile_begin(self._c))

    def profile_mask(self, stages=None):
        """Record only the named stages in later sessions (None: all stages)."""
        mask = 0 if not stages else sum(1 << STAGES.index(k) for k in stages)
        self._check(self._L.scabs_profile_mask(self._c, mask))

    def profile_end(self) -> dict:
        ms = (C.c_double * len(STAGES))()
        cnt = (C.c_int64 * len(STAGES))()
        self._check(self._L.scabs_profile_end(self._c, ms, cnt))
        nbytes = (C.c_double * len(STAGES))()
        self._check(self._L.scabs_profile_bytes(self._c, nbytes))
        return {name: {"ms": ms[k], "count": cnt[k], "bytes": nbytes[k]} for k, name in enumerate(STAGES)}

    def solve(self, b, x0=None, tol: float = 1e-6, max_iter: int = 2000, restart: int = 60,
              mode: int = SCABS_MIXED, raise_on_noconv: bool = False, transpose: bool = False):
        import torch
        b = self._dev(b)
        x = torch.zeros_like(b) if x0 is None else self._dev(x0).clone()
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        infos = (SolveInfo * nrhs)()
        fn = self._L.scabs_solve_transpose if transpose else self._L.scabs_solve
        rc = fn(self._c, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs, tol, max_iter, restart, mode,
                infos)
        if rc != SCABS_OK and (rc != SCABS_E_NOCONV or raise_on_noconv):
            self._check(rc)
        out = [infos[k].as_dict() for k in range(nrhs)]
        return x, (out[0] if b.dim() == 1 else out)


def solve_batched(ctxs: Sequence["Context"], bs, tol: float = 1e-6, max_iter: int = 2000, restart: int = 60,
                  mode: int = SCABS_MIXED, raise_on_noconv: bool = False):
    """scabs_solve_batched: context i solves the systems bs[i] (one vector or
    a stack); the contexts run concurrently.  Returns ([x_i], [infos_i])."""
    import torch
    n = len(ctxs)
    if n != len(bs) or n == 0:
        raise ValueError("one right-hand side block per context")
    bs = [c._dev(b) for c, b in zip(ctxs, bs)]
    xs = [torch.zeros_like(b) for b in bs]
    nr = [1 if b.dim() == 1 else b.shape[0] for b in bs]
    infos = [(SolveInfo * k)() for k in nr]
    L = load()
    cp = (C.c_void_p * n)(*[c._c for c in ctxs])
    bp = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    ip = (C.POINTER(SolveInfo) * n)(*[C.cast(i, C.POINTER(SolveInfo)) for i in infos])
    rc = L.scabs_solve_batched(cp, n, bp, xp, (C.c_int * n)(*nr), tol, max_iter, restart, mode, ip)
    if rc != SCABS_OK and (rc != SCABS_E_NOCONV or raise_on_noconv):
        for c in ctxs:
            msg = L.scabs_last_error(c._c).decode()
            if msg:
                raise ScabsError(rc, msg)
        raise ScabsError(rc, "scabs_solve_batched")
    out = [[inf[k].as_dict() for k in range(m)] for inf, m in zip(infos, nr)]
    return xs, out


def context_for(workload, device: int = 0, kappa_s: float = 1.37, h: Optional[float] = None,
                r_near: Optional[float] = None, **opts) -> Context:
    """Build a context from a synth.Workload-like object."""
    ctx = Context(workload.h if h is None else h, workload.r_near if r_near is None else r_near, kappa_s, device,
                  **opts)
    m = workload.mesh
    ctx.set_mesh(m.verts, m.tris, m.body)
    ctx.set_media(workload.omega, workload.eps_out, workload.eps_in)
    ctx.set_sigma(workload.sigma)
    ctx.build()
    return ctx


# ---------------------------------------------------------------------------
# differentiation: torch.autograd wrappers over the adjoint entry points
# ---------------------------------------------------------------------------
def _autograd_functions():
    import torch

    class SigmaSolve(torch.autograd.Function):
        """x = A(p)^-1 b(p) for the profile parameters p of one context (the
        context is rebuilt with p).  Backward: A^T lam = g by the transposed
        solve, then d/dp = 2 Re[lam^T (db/dp - dA/dp x)] from the library.
        PyTorch's gradient of a real loss for complex x is 2 conj(d loss/dx),
        so g = conj(x.grad) / 2."""

        @staticmethod
        def forward(fctx, params, ctx, set_params, dipole, tol, restart, mode):
            set_params(ctx, params.detach().cpu().numpy())
            ctx.build()
            d = dipole
            b = ctx.rhs_dipole(d.pos, d.moment, d.body)
            x, info = ctx.solve(b, tol=tol, restart=restart, mode=mode, max_iter=20000, raise_on_noconv=True)
            einc = ctx.incident_dipole_points(d.pos, d.moment, d.body)
            fctx.ctx, fctx.tol, fctx.restart, fctx.mode = ctx, tol, restart, mode
            fctx.save_for_backward(x, einc)
            return x

        @staticmethod
        def backward(fctx, gx):
            x, einc = fctx.saved_tensors
            ctx = fctx.ctx
            g = (torch.conj(gx) * 0.5).resolve_conj().contiguous()
            lam, _ = ctx.solve(g, tol=fctx.tol, restart=fctx.restart, mode=fctx.mode, max_iter=20000,
                               raise_on_noconv=True, transpose=True)
            _, dp = ctx.sigma_gradient(x, lam, einc)
            return torch.from_numpy(dp), None, None, None, None, None, None

    class FieldAt(torch.autograd.Function):
        """E at off-surface points (scattered part) as a function of x."""

        @staticmethod
        def forward(fctx, x, ctx, pts, region):
            E, _ = ctx.eval_field(x.detach(), pts, region)
            fctx.ctx, fctx.pts, fctx.region = ctx, pts, region
            return E

        @staticmethod
        def backward(fctx, gE):
            # vector-Jacobian product of a complex-linear map: Q^H gE = conj(Q^T conj(gE))
            y = fctx.ctx.eval_field_transpose(fctx.pts, fctx.region, torch.conj(gE).resolve_conj())
            return torch.conj(y).resolve_conj(), None, None, None

    return SigmaSolve, FieldAt


def sigma_solve(params, ctx: Context, set_params, dipole, tol: float = 1e-10, restart: int = 200,
                mode: int = SCABS_FP64):
    """Differentiable solve: x(params) with d/dparams by the adjoint method.
    set_params(ctx, values) must apply the profile parameters to ctx."""
    SigmaSolve, _ = _autograd_functions()
    return SigmaSolve.apply(params, ctx, set_params, dipole, tol, restart, mode)


def field_at(x, ctx: Context, pts, region: int):
    """Differentiable scattered field E at off-surface points."""
    _, FieldAt = _autograd_functions()
    return FieldAt.apply(x, ctx, pts, region)


def reflected_amplitude(E_y, xs, beta: float):
    """b of the least-squares fit E_y(x_k) = a e^{-j beta x} + b e^{+j beta x}
    at monitor positions xs (torch, differentiable in E_y): b = w . E_y with w
    the second row of the pseudo-inverse of the 2-column fit matrix."""
    import torch
    xs = np.asarray(xs, float)
    P = np.stack([np.exp(-1j * beta * xs), np.exp(1j * beta * xs)], axis=1)
    w = torch.as_tensor(np.linalg.pinv(P)[1], dtype=torch.complex128, device=E_y.device)
    return (w * E_y).sum()


def _cplx(E):
    e = np.ascontiguousarray(np.asarray(E, dtype=np.complex128))
    return e, e.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))


def swr(E):
    """(standing-wave ratio, reflection coefficient) of field samples."""
    e, ep = _cplx(E)
    out = np.zeros(2)
    rc = load().scabs_swr(ep, e.shape[0], out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != SCABS_OK:
        raise ScabsError(rc, "scabs_swr")
    return float(out[0]), float(out[1])


def standing_wave_fit(xs, E, beta_lo: float, beta_hi: float):
    """(beta, |r|, relative residual, |a|, |c|, arg r) of E = a e^{-j beta x} + c e^{j beta x}."""
    x = np.ascontiguousarray(np.asarray(xs, dtype=np.float64))
    e, ep = _cplx(E)
    out = np.zeros(6)
    rc = load().scabs_standing_wave_fit(x.ctypes.data_as(C.POINTER(C.c_double)), ep, e.shape[0], float(beta_lo),
                                        float(beta_hi), out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != SCABS_OK:
        raise ScabsError(rc, "scabs_standing_wave_fit")
    return tuple(float(v) for v in out)


def decay_fit(xs, E):
    """(alpha, beta, relative residual, c0) of ln|E| = c0 - alpha x, phase = p0 - beta x."""
    x = np.ascontiguousarray(np.asarray(xs, dtype=np.float64))
    e, ep = _cplx(E)
    out = np.zeros(4)
    rc = load().scabs_decay_fit(x.ctypes.data_as(C.POINTER(C.c_double)), ep, e.shape[0],
                                out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != SCABS_OK:
        raise ScabsError(rc, "scabs_decay_fit")
    return tuple(float(v) for v in out)
