"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only builds the
inputs the method consumes -- closed triangulated surfaces, absorber profile
descriptions, dipole sources and random vectors -- from explicit seeds.

Units follow the paper's convention: lengths in wavelengths inside the
waveguide medium (lambda_i = 1), eps0 = mu0 = 1, so the interior wavenumber is
2*pi and the free-space wavenumber is 2*pi / sqrt(eps_in).

Geometry recipe (rectangular dielectric guides, Sec. I Fig. "waveguide",
Sec. III/IV): each guide is an axis-aligned box meshed with a structured grid
of quads split along one diagonal, so the surface mesh repeats along x (the
periodic unit of the fast-solver appendix).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood 2014); uniform doubles from
    the top 53 bits."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()

    def normal(self) -> float:
        # Box-Muller on two uniforms (first one shifted away from 0)
        u1 = 1.0 - self.uniform()
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


# ----------------------------------------------------------------------------
# surfaces
# ----------------------------------------------------------------------------

@dataclass
class Mesh:
    verts: np.ndarray          # (nv, 3) float64
    tris: np.ndarray           # (nt, 3) int32, outward (counter-clockwise seen from outside)
    body: np.ndarray           # (nt,) int32

    @property
    def nv(self) -> int:
        return self.verts.shape[0]

    @property
    def nt(self) -> int:
        return self.tris.shape[0]


def _divisions(extent: float, edge: float) -> int:
    return max(1, int(math.ceil(extent / edge - 1e-9)))


def box_mesh(x0: float, x1: float, y0: float, y1: float, z0: float, z1: float,
             edge: float) -> Tuple[np.ndarray, np.ndarray]:
    """Closed, outward-oriented structured triangulation of a box surface.

    Each axis gets ceil(extent/edge) equal divisions; every quad is split along
    the diagonal joining its (i, j) and (i+1, j+1) corners."""
    nx, ny, nz = _divisions(x1 - x0, edge), _divisions(y1 - y0, edge), _divisions(z1 - z0, edge)
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    zs = np.linspace(z0, z1, nz + 1)
    index = {}
    verts: List[Tuple[float, float, float]] = []

    def vid(i, j, k):
        key = (i, j, k)
        v = index.get(key)
        if v is None:
            v = len(verts)
            index[key] = v
            verts.append((xs[i], ys[j], zs[k]))
        return v

    tris: List[Tuple[int, int, int]] = []

    def quad(a, b, c, d, outward):
        # a-b-c-d around the quad; split along a-c
        pa, pb, pc = (np.array(verts[a]), np.array(verts[b]), np.array(verts[c]))
        nrm = np.cross(pb - pa, pc - pa)
        if np.dot(nrm, outward) < 0:
            tris.append((a, c, b))
            tris.append((a, d, c))
        else:
            tris.append((a, b, c))
            tris.append((a, c, d))

    # faces normal to x
    for i, sgn in ((0, -1.0), (nx, 1.0)):
        for j in range(ny):
            for k in range(nz):
                quad(vid(i, j, k), vid(i, j + 1, k), vid(i, j + 1, k + 1), vid(i, j, k + 1),
                     np.array([sgn, 0, 0]))
    # faces normal to y
    for j, sgn in ((0, -1.0), (ny, 1.0)):
        for i in range(nx):
            for k in range(nz):
                quad(vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j, k + 1), vid(i, j, k + 1),
                     np.array([0, sgn, 0]))
    # faces normal to z
    for k, sgn in ((0, -1.0), (nz, 1.0)):
        for i in range(nx):
            for j in range(ny):
                quad(vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i, j + 1, k),
                     np.array([0, 0, sgn]))
    return np.asarray(verts, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def merge_bodies(parts: Sequence[Tuple[np.ndarray, np.ndarray]]) -> Mesh:
    vs, ts, bs = [], [], []
    off = 0
    for b, (v, t) in enumerate(parts):
        vs.append(v)
        ts.append(t + off)
        bs.append(np.full(t.shape[0], b, dtype=np.int32))
        off += v.shape[0]
    return Mesh(np.concatenate(vs), np.concatenate(ts).astype(np.int32), np.concatenate(bs))


def icosphere(radius: float, level: int, center=(0.0, 0.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """Subdivided icosahedron projected onto a sphere, outward oriented."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, dtype=np.float64) / np.linalg.norm(x) for x in v]
    faces = list(f)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.asarray(verts) * radius + np.asarray(center, dtype=np.float64)
    T = np.asarray(faces, dtype=np.int32)
    # orient outward
    c = np.asarray(center, dtype=np.float64)
    for i, (a, b, cc) in enumerate(T):
        n = np.cross(V[b] - V[a], V[cc] - V[a])
        if np.dot(n, V[a] - c) < 0:
            T[i] = (a, cc, b)
    return V, T


# ----------------------------------------------------------------------------
# absorber profile descriptions (evaluated by the method, not here)
# ----------------------------------------------------------------------------

@dataclass
class SigmaEnd:
    """One absorber: sigma = sigma0 * u(s), s = dir*(x_axis - x0)/L clamped to
    [0, 1] (Sec. IV, the monomial u(s) = s^d with u = 0 for s < 0), or a
    piecewise-linear u given by control values at s_k = k/(n-1)."""
    axis: int
    x0: float
    length: float
    direction: int = +1
    degree: int = 2
    sigma0: float = 1.0
    ctrl: Optional[np.ndarray] = None   # piecewise-linear control values (then sigma0/degree unused)


# ----------------------------------------------------------------------------
# sources and vectors
# ----------------------------------------------------------------------------

@dataclass
class Dipole:
    pos: np.ndarray        # (3,)
    moment: np.ndarray     # (3,) complex current moment I*l
    body: int = 0


@dataclass
class Beam:
    """Gaussian-beam source (Sec. II): a dipole of moment `moment` at the
    complex position pos - j b direction; waist at pos, Rayleigh distance b."""
    pos: np.ndarray
    moment: np.ndarray
    body: int = 0
    direction: tuple = (1.0, 0.0, 0.0)
    b: float = 1.0


def seeded_dipole(seed: int, base=(0.5, 0.0, 0.0), jitter=(0.05, 0.02, 0.02), body: int = 0) -> Dipole:
    rng = SplitMix64(seed)
    pos = np.array([base[i] + rng.uniform_range(-jitter[i], jitter[i]) for i in range(3)])
    z = rng.uniform_range(-1.0, 1.0)
    ph = rng.uniform_range(0.0, 2.0 * math.pi)
    s = math.sqrt(max(0.0, 1.0 - z * z))
    mom = np.array([s * math.cos(ph), s * math.sin(ph), z], dtype=np.complex128)
    return Dipole(pos, mom, body)


def random_complex(seed: int, n: int) -> np.ndarray:
    rng = SplitMix64(seed)
    out = np.empty(n, dtype=np.complex128)
    for i in range(n):
        out[i] = complex(rng.uniform_range(-1, 1), rng.uniform_range(-1, 1))
    return out


def random_uniform(seed: int, n: int, lo: float, hi: float) -> np.ndarray:
    rng = SplitMix64(seed)
    return np.array([rng.uniform_range(lo, hi) for _ in range(n)])


# ----------------------------------------------------------------------------
# workloads (shapes of the paper's guides, in lambda_i units)
# ----------------------------------------------------------------------------

EPS_IN = 12.25          # silicon-like guide (the paper uses 11.9; configs use 12.25)
EPS_OUT = 1.0
OMEGA = 2.0 * math.pi / math.sqrt(EPS_IN)   # free-space wavenumber k0 when lambda_i = 1


@dataclass
class Workload:
    name: str
    mesh: Mesh
    sigma: List[SigmaEnd]
    dipoles: List[Dipole]
    h: float                      # projection-grid spacing
    r_near: float                 # near-list radius (centroid distance)
    omega: float = OMEGA
    eps_in: float = EPS_IN
    eps_out: float = EPS_OUT
    notes: dict = field(default_factory=dict)


def guide(length: float, edge: float, width: float = 0.4, thick: float = 0.2,
          yc: float = 0.0, zc: float = 0.0, x0: float = 0.0):
    return box_mesh(x0, x0 + length, yc - width / 2, yc + width / 2, zc - thick / 2, zc + thick / 2, edge)


def workload_small(seed: int = 0, edge: float = 0.15, length: float = 4.0, absorber: float = 2.0,
                   degree: int = 2, sigma0: float = 1.0, h: float = 0.05, r_near: float = 0.3137) -> Workload:
    """The CPU-small case: straight 0.4 x 0.2 guide, length 4, quadratic
    absorber on the last 2 (sigma0 = 1 in units of 1/Z0), one seeded dipole
    0.5 from the input end."""
    v, t = guide(length, edge)
    mesh = merge_bodies([(v, t)])
    sig = [SigmaEnd(axis=0, x0=length - absorber, length=absorber, direction=+1, degree=degree, sigma0=sigma0)]
    dip = seeded_dipole(1000 * 0 + seed)
    return Workload("guide4_edge%.3g" % edge, mesh, sig, [dip], h=h, r_near=r_near)


def workload_transition(L: float, degree: int, edge: float = 0.1, guide_len: float = 20.0,
                        h: float = 0.05, r_near: float = 0.3137, seed: int = 0) -> Workload:
    """Transition-reflection family: guide of fixed length plus an appended
    absorber of length L with sigma0 = 2/L (fixed round-trip loss)."""
    v, t = guide(guide_len + L, edge)
    mesh = merge_bodies([(v, t)])
    sig = [SigmaEnd(axis=0, x0=guide_len, length=L, direction=+1, degree=degree, sigma0=2.0 / L)]
    dip = seeded_dipole(1000 * 1 + seed)
    return Workload("transition_L%g_d%d" % (L, degree), mesh, sig, [dip], h=h, r_near=r_near)


def workload_gradient(guide_len: float = 20.0, absorber: float = 4.0, edge: float = 0.1, n_ctrl: int = 256,
                      n_monitor: int = 16, h: float = 0.05, r_near: float = 0.3137, seed: int = 0,
                      beta_frac: float = 0.9) -> Workload:
    """Differentiation form: guide of length guide_len with an appended
    absorber whose conductivity is piecewise linear with n_ctrl control values
    drawn U[0, 2] from the seed; n_monitor field samples on the guide axis over
    [2, guide_len - 2] (clamped to the guide); fitted propagation constant
    frozen at beta_frac * k_i (notes: 'monitor_x', 'beta')."""
    v, t = guide(guide_len + absorber, edge)
    mesh = merge_bodies([(v, t)])
    rng = SplitMix64(7000 + seed)
    ctrl = np.array([rng.uniform_range(0.0, 2.0) for _ in range(n_ctrl)])
    sig = [SigmaEnd(axis=0, x0=guide_len, length=absorber, direction=+1, ctrl=ctrl)]
    dip = seeded_dipole(1000 * 4 + seed)
    a, b = min(2.0, 0.25 * guide_len), max(guide_len - 2.0, 0.75 * guide_len)
    xs = np.linspace(a, b, n_monitor)
    k_i = OMEGA * math.sqrt(EPS_IN)
    return Workload("gradient_W%g_L%g_edge%.3g" % (guide_len, absorber, edge), mesh, sig, [dip], h=h, r_near=r_near,
                    notes={"monitor_x": xs, "beta": beta_frac * k_i})


def workload_two_channel(edge: float = 0.072, length: float = 30.0, absorber: float = 4.0,
                         nx_target: int = 512, r_near: Optional[float] = None, seed: int = 0) -> Workload:
    """Two parallel 0.4 x 0.2 channels (gap 0.3, centres y = +-0.35), quartic
    absorbers of length 4 at both ends, one seeded dipole in channel 0."""
    parts = [guide(length, edge, yc=-0.35), guide(length, edge, yc=+0.35)]
    mesh = merge_bodies(parts)
    sig = [SigmaEnd(axis=0, x0=length - absorber, length=absorber, direction=+1, degree=4, sigma0=1.0),
           SigmaEnd(axis=0, x0=absorber, length=absorber, direction=-1, degree=4, sigma0=1.0)]
    # grid spacing chosen so that the physical x-extent (plus one stencil node
    # each side) fits nx_target nodes
    h = length / (nx_target - 4)
    if r_near is None:
        r_near = 3.61 * h
    dip = seeded_dipole(1000 * 2 + seed, base=(4.5, -0.35, 0.0), jitter=(0.5, 0.02, 0.02), body=0)
    return Workload("two_channel_%gx_edge%g" % (length, edge), mesh, sig, [dip], h=h, r_near=r_near)
