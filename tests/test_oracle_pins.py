"""Pins of the oracle against things other than itself: textbook rules, closed
forms, brute-force quadrature, physical identities and structural facts the
paper states.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import synth




# ---------------------------------------------------------------------------
# quadrature and singular integrals
# ---------------------------------------------------------------------------

def _tri_rule():
    import ctypes as C
    b = np.zeros((7, 3))
    w = np.zeros(7)
    oracle.lib().or_rule7.argtypes = [np.ctypeslib.ndpointer(np.float64), np.ctypeslib.ndpointer(np.float64)]
    oracle.lib().or_rule7(b, w)
    return b, w


def test_rule7_exact_to_degree_5():
    # int over the unit right triangle of x^a y^b = a! b! / (a+b+2)!
    b, w = _tri_rule()
    x, y = b[:, 1], b[:, 2]
    for a in range(6):
        for c in range(6 - a):
            exact = math.factorial(a) * math.factorial(c) / math.factorial(a + c + 2)
            got = 0.5 * np.sum(w * x ** a * y ** c)
            assert abs(got - exact) < 1e-15, (a, c)
    # degree 6 is not integrated exactly (the rule is degree 5)
    got = 0.5 * np.sum(w * x ** 6)
    assert abs(got - math.factorial(6) / math.factorial(8)) > 1e-6


def _duffy_integral(fun, r, p0, p1, p2, ng=400):
    """Brute force: split the triangle at the projection of r and integrate
    each sub-triangle in Duffy coordinates with tensor Gauss-Legendre
    (fun takes an (m, 3) array of source points)."""
    n = np.cross(p1 - p0, p2 - p0)
    n /= np.linalg.norm(n)
    P = r - np.dot(r - p0, n) * n
    g, gw = np.polynomial.legendre.leggauss(ng)
    g = 0.5 * (g + 1)
    gw = 0.5 * gw
    U, Vv = np.meshgrid(g, g, indexing="ij")
    W = np.outer(gw, gw)
    tot = 0
    for (B, Cc) in ((p0, p1), (p1, p2), (p2, p0)):
        cr = np.cross(B - P, Cc - P)
        jac = np.linalg.norm(cr) * np.sign(np.dot(cr, n))
        q = P + U[..., None] * (B - P) + (U * Vv)[..., None] * (Cc - B)
        vals = fun(q.reshape(-1, 3))
        wts = (W * U * jac).reshape(-1)
        tot = tot + np.tensordot(wts, vals, axes=(0, 0))
    return tot


@pytest.mark.parametrize("pt", [
    (0.2, 0.3, 0.15),      # above the interior
    (0.9, 0.8, -0.05),     # below, outside the projection
    (0.45, 0.05, 0.01),    # close to an edge
    (1.5, -0.4, 0.3),      # far
])
def test_static_integrals_brute_force(pt):
    p0, p1, p2 = np.array([0.0, 0, 0]), np.array([1.0, 0.1, 0]), np.array([0.2, 0.9, 0.0])
    r = np.array(pt, float)
    I0, I1, Ig = oracle.static_integrals(r, p0, p1, p2)
    R = lambda q: np.linalg.norm(r - q, axis=1)
    b0 = _duffy_integral(lambda q: 1 / R(q), r, p0, p1, p2)
    b1 = _duffy_integral(lambda q: (q - r) / R(q)[:, None], r, p0, p1, p2)
    bg = _duffy_integral(lambda q: -(r - q) / R(q)[:, None] ** 3, r, p0, p1, p2, ng=800)
    assert abs(I0 - b0) < 1e-9 * abs(b0)
    assert np.linalg.norm(I1 - b1) < 1e-9 * np.linalg.norm(b1)
    assert np.linalg.norm(Ig - bg) < 1e-6 * np.linalg.norm(bg)


def test_static_integrals_in_plane():
    # point inside the triangle: I0 by brute force (Duffy removes 1/R), the
    # in-plane gradient equals the gradient of I0 (finite differences), the
    # principal-value normal component is zero
    p0, p1, p2 = np.array([0.0, 0, 0]), np.array([1.0, 0.1, 0]), np.array([0.2, 0.9, 0.0])
    r = np.array([0.37, 0.31, 0.0])
    I0, I1, Ig = oracle.static_integrals(r, p0, p1, p2)
    R = lambda q: np.linalg.norm(r - q, axis=1)
    b0 = _duffy_integral(lambda q: 1 / R(q), r, p0, p1, p2)
    b1 = _duffy_integral(lambda q: (q - r) / R(q)[:, None], r, p0, p1, p2)
    assert abs(I0 - b0) < 1e-10 * abs(b0)
    assert np.linalg.norm(I1 - b1) < 1e-10 * np.linalg.norm(b1)
    eps = 1e-6
    for a in range(2):
        d = np.zeros(3)
        d[a] = eps
        fd = (oracle.static_integrals(r + d, p0, p1, p2)[0] - oracle.static_integrals(r - d, p0, p1, p2)[0]) / (2 * eps)
        assert abs(Ig[a] - fd) < 1e-6 * max(1, abs(fd))
    assert Ig[2] == 0.0
    # just above the plane the normal component tends to -2 pi (solid angle of a half space)
    _, _, Ig_up = oracle.static_integrals(r + np.array([0, 0, 1e-9]), p0, p1, p2)
    assert abs(Ig_up[2] + 2 * math.pi) < 1e-6


def test_dipole_fields_satisfy_maxwell():
    # curl E = -j k Z H and curl H = (j k / Z) E  (e^{jwt}, eps0 = mu0 = 1)
    k, Z = 2 * math.pi, 1 / 3.5
    r0 = np.array([0.1, -0.2, 0.05])
    p = np.array([0.3 + 0.1j, -0.7, 0.5j])
    r = np.array([0.6, 0.25, -0.3])
    eps = 1e-5

    def curl(fun):
        J = np.zeros((3, 3), complex)
        for a in range(3):
            d = np.zeros(3)
            d[a] = eps
            J[:, a] = (fun(r + d) - fun(r - d)) / (2 * eps)
        return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])

    E, H = oracle.dipole_field(k, Z, r0, p, r)
    cE = curl(lambda q: oracle.dipole_field(k, Z, r0, p, q)[0])
    cH = curl(lambda q: oracle.dipole_field(k, Z, r0, p, q)[1])
    assert np.linalg.norm(cE + 1j * k * Z * H) < 1e-7 * np.linalg.norm(cE)
    assert np.linalg.norm(cH - 1j * k / Z * E) < 1e-7 * np.linalg.norm(cH)


# ---------------------------------------------------------------------------
# mesh, RWG
# ---------------------------------------------------------------------------

def test_rwg_edges_and_normal_continuity():
    w = synth.workload_small()
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    assert o.ne == 3 * o.nt // 2
    # edges sorted by (v_min, v_max), T+ the lower triangle index
    key = o.ev[:, 0].astype(np.int64) * o.nv + o.ev[:, 1]
    assert np.all(np.diff(key) > 0) and np.all(o.ev[:, 0] < o.ev[:, 1])
    assert np.all(o.et[:, 0] < o.et[:, 1])
    # total divergence of each RWG integrates to zero; flux through the shared edge is 1
    fv, fd = o.point_basis()
    for e in range(0, o.ne, 37):
        tot = 0
        for s in range(2):
            T = o.et[e, s]
            j = list(o.tedge[T]).index(e)
            tot += np.sum(o.qw[T * 7:(T + 1) * 7] * fd[T * 7:(T + 1) * 7, j])
        assert abs(tot) < 1e-14
    e = 5
    va, vb = w.mesh.verts[o.ev[e, 0]], w.mesh.verts[o.ev[e, 1]]
    mid = 0.5 * (va + vb)
    for s in range(2):
        T = o.et[e, s]
        j = list(o.tedge[T]).index(e)
        vfree = w.mesh.verts[w.mesh.tris[T, j]]
        f = o.tsign[T, j] * o.elen[e] / (2 * 0.5 * np.linalg.norm(np.cross(*(w.mesh.verts[w.mesh.tris[T, 1:]] - w.mesh.verts[w.mesh.tris[T, 0]])))) * (mid - vfree)
        m = np.cross(vb - va, o.nrm[T])
        m = m / np.linalg.norm(m)
        sgn = 1 if np.dot(mid - vfree, m) > 0 else -1
        flux = np.dot(f, m) * sgn
        assert abs(abs(flux) - 1) < 1e-12


def test_mesh_validation_rejects_open_and_inverted():
    v, t = synth.box_mesh(0, 1, 0, 0.4, 0, 0.2, 0.2)
    with pytest.raises(ValueError):
        oracle.Oracle(synth.Mesh(v, t[:-1].copy(), np.zeros(t.shape[0] - 1, np.int32)), 1.0, 12.25)
    with pytest.raises(ValueError):
        oracle.Oracle(synth.Mesh(v, t[:, ::-1].copy(), np.zeros(t.shape[0], np.int32)), 1.0, 12.25)


# ---------------------------------------------------------------------------
# closed forms: dielectric sphere with a centred dipole (TM1), with and
# without a uniform surface conductivity
# ---------------------------------------------------------------------------

def tm1_sphere(a, ki, Zi, ke, Ze, p, sigma):
    """Closed-form l = 1 TM solution: H_phi = sin(theta) F(r), with
    F_i = -(j k_i^2 p / 4 pi) h1(k_i r) + A j1(k_i r), F_e = B h1(k_e r);
    E_theta continuous and H_phi^i - H_phi^e = sigma E_theta at r = a."""
    h1 = lambda x: np.exp(-1j * x) * (1j / x ** 2 - 1 / x)
    j1 = lambda x: math.sin(x) / x ** 2 - math.cos(x) / x
    dpsih = lambda x: np.exp(-1j * x) * (1 / x + 1j - 1j / x ** 2)
    dpsij = lambda x: math.cos(x) / x - math.sin(x) / x ** 2 + math.sin(x)
    S = -1j * ki ** 2 * p / (4 * math.pi)
    xi, xe = ki * a, ke * a
    M = np.array([[-(Zi / ki) * dpsij(xi), (Ze / ke) * dpsih(xe)],
                  [j1(xi), -h1(xe) - sigma * (1j * Ze / ke) * dpsih(xe) / a]], complex)
    rhs = np.array([(Zi / ki) * S * dpsih(xi), -S * h1(xi)], complex)
    A, B = np.linalg.solve(M, rhs)
    Ez0 = -(2j * Zi * A / 3)                     # scattered interior field at the centre
    Hy = lambda r: B * h1(ke * r)                 # exterior H_phi on the x axis
    return Ez0, Hy


@pytest.mark.parametrize("sigma", [0.0, 0.7])
def test_sphere_dipole_closed_form(sigma):
    a = 0.25
    v, t = synth.icosphere(a, 2)
    mesh = synth.merge_bodies([(v, t)])
    o = oracle.Oracle(mesh, synth.OMEGA, synth.EPS_IN)
    if sigma == 0:
        o.set_sigma([])
    else:
        o.set_sigma_points(np.full(o.np_, sigma))
        assert o.NR == o.ne
    dip = synth.Dipole(np.zeros(3), np.array([0, 0, 1.0 + 0j]), 0)
    x = oracle.lu_solve(o.dense(), o.rhs_dipole(dip))
    Ez0, Hy = tm1_sphere(a, o.k_i, o.Z_i, o.k_e, o.Z_e, 1.0, sigma)
    E0, _ = o.fields_at(x, np.zeros((1, 3)), 0)
    _, H2 = o.fields_at(x, np.array([[2 * a, 0, 0]]), -1)
    # 320-triangle sphere: discretisation error of a few percent at the centre
    assert abs(E0[0, 2] - Ez0) < 0.04 * abs(Ez0)
    assert abs(H2[0, 1] - Hy(2 * a)) < 0.006 * abs(Hy(2 * a))
    # the conductivity changes the answer far beyond that tolerance
    if sigma > 0:
        Ez0_0, Hy_0 = tm1_sphere(a, o.k_i, o.Z_i, o.k_e, o.Z_e, 1.0, 0.0)
        assert abs(Ez0_0 - Ez0) > 0.2 * abs(Ez0)


# ---------------------------------------------------------------------------
# identities of the discrete system
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    w = synth.workload_small()
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    return w, o


def test_sigma_zero_reduction(small):
    """All edges treated as absorber edges with sigma = 0 gives the PMCHW
    currents, with J_i = -J_e (eq10) and G(J_e + J_i) = 0."""
    w, o = small
    dip = w.dipoles[0]
    o.set_sigma([])
    x2 = oracle.lu_solve(o.dense(), o.rhs_dipole(dip))
    Je2, _, M2 = o.edge_currents(x2)
    o.set_sigma([], force_all_R=True)
    assert o.N == 3 * o.ne
    x5 = oracle.lu_solve(o.dense(), o.rhs_dipole(dip))
    Je5, Ji5, M5 = o.edge_currents(x5)
    s = np.linalg.norm(Je2)
    assert np.linalg.norm(Je5 - Je2) < 1e-9 * s
    assert np.linalg.norm(Ji5 + Je2) < 1e-9 * s
    assert np.linalg.norm(M5 - M2) < 1e-9 * np.linalg.norm(M2)
    o.set_sigma(w.sigma)


def test_reciprocity_symmetry(small):
    """With D = diag(I, -I) the sigma-free PMCHW matrix D A is complex
    symmetric; entries between far-apart edges (plain quadrature on both
    sides) are symmetric to rounding, near entries to quadrature accuracy."""
    w, o = small
    o.set_sigma([])
    A = o.dense()
    N = o.N
    D = np.ones(N)
    D[o.NL:] = -1
    DA = D[:, None] * A
    asym = DA - DA.T
    assert np.linalg.norm(asym) < 2e-2 * np.linalg.norm(DA)
    mid = 0.5 * (w.mesh.verts[o.ev[:, 0]] + w.mesh.verts[o.ev[:, 1]])
    far = np.linalg.norm(mid[:, None, :] - mid[None, :, :], axis=2) > 1.0
    farmask = np.tile(far, (2, 2))
    assert np.max(np.abs(asym[farmask])) < 1e-13 * np.max(np.abs(DA))
    o.set_sigma(w.sigma)


def test_power_balance(small):
    """P_dip = P_rad (sigma = 0) and P_dip = P_rad + P_abs (sigma > 0), to
    discretisation accuracy on this coarse mesh; P_abs > 0."""
    w, o = small
    dip = w.dipoles[0]
    bal = []
    for sig in ([], w.sigma):
        o.set_sigma(sig)
        x = oracle.lu_solve(o.dense(), o.rhs_dipole(dip))
        pd, pr = o.dipole_power(x, dip), o.radiated_power(x)
        pa = o.absorbed_power(x, dip) if sig else 0.0
        bal.append((pr + pa) / pd)
        if sig:
            assert pa > 0
    assert abs(bal[0] - 1) < 0.1 and abs(bal[1] - 1) < 0.1
    assert abs(bal[1] - bal[0]) < 2e-3


def test_block_toeplitz_rings(small):
    """On the x-periodic mesh the sigma-free interaction between two rings of
    side-face edges depends only on their ring offset (fast-solver appendix)."""
    w, o = small
    o.set_sigma([])
    A = o.dense()
    V = w.mesh.verts
    mid = 0.5 * (V[o.ev[:, 0]] + V[o.ev[:, 1]])
    dx = 4.0 / 27
    ring = np.floor(mid[:, 0] / dx + 0.25).astype(int)
    side = (mid[:, 0] > 1.5 * dx) & (mid[:, 0] < 4.0 - 1.5 * dx)

    def ring_edges(i):
        idx = np.where(side & (ring == i))[0]
        return idx[np.lexsort((mid[idx, 2], mid[idx, 1], mid[idx, 0] - i * dx))]

    for d in (0, 1, 3):
        ref_r, ref_c = ring_edges(5), ring_edges(5 + d)
        blk0 = A[np.ix_(o.eidx[ref_r], o.eidx[ref_c])]
        for i in (9, 14):
            rr, cc = ring_edges(i), ring_edges(i + d)
            assert np.allclose(mid[rr] - mid[ref_r], [(i - 5) * dx, 0, 0], atol=1e-9)
            blk = A[np.ix_(o.eidx[rr], o.eidx[cc])]
            assert np.max(np.abs(blk - blk0)) < 1e-10 * np.max(np.abs(blk0))
    o.set_sigma(w.sigma)


# ---------------------------------------------------------------------------
# the pFFT operator's definition
# ---------------------------------------------------------------------------

def test_stencil_interpolates_quadratics():
    h = 0.07
    lib = oracle.lib()
    rng = np.random.default_rng(3)
    for _ in range(5):
        r = rng.uniform(-1, 1, 3)
        anc = np.zeros(3, np.int32)
        w = np.zeros(27)
        gw = np.zeros(81)
        lib.or_stencil(h, r, anc, w, gw)
        nodes = np.array([[(anc[0] + i) * h, (anc[1] + j) * h, (anc[2] + k) * h]
                          for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
        f = lambda p: 1.3 + p[..., 0] - 2 * p[..., 1] * p[..., 2] + 0.7 * p[..., 0] ** 2 + p[..., 1] * p[..., 0]
        grad = np.array([1 + 1.4 * r[0] + r[1], -2 * r[2] + r[0], -2 * r[1]])
        assert abs(np.dot(w, f(nodes)) - f(r)) < 1e-13
        assert np.linalg.norm(gw.reshape(27, 3).T @ f(nodes) - grad) < 1e-11


def test_pfft_all_near_is_exact(small):
    """With every triangle pair in the near list, the precorrected operator
    is the dense Galerkin matrix (the grid part cancels exactly)."""
    w, o = small
    o.set_sigma(w.sigma)
    A = o.dense()
    P = o.pfft(0.05, 100.0)
    x = synth.random_complex(11, o.N)
    y = P.matvec(x)
    assert np.linalg.norm(y - A @ x) < 1e-12 * np.linalg.norm(A @ x)


def test_pfft_approximates_galerkin(small):
    """A~ x approximates A x; the error falls with a finer grid."""
    w, o = small
    o.set_sigma(w.sigma)
    A = o.dense()
    x = synth.random_complex(12, o.N)
    ya = A @ x
    e1 = np.linalg.norm(o.pfft(0.05, 0.3137).matvec(x) - ya) / np.linalg.norm(ya)
    e2 = np.linalg.norm(o.pfft(0.0375, 0.3137).matvec(x) - ya) / np.linalg.norm(ya)
    assert e1 < 1e-3 and e2 < 0.6 * e1


def test_pfft_rejects_small_near_radius(small):
    w, o = small
    with pytest.raises(ValueError):
        o.pfft(0.05, 0.5 * o.singular_radius())


# ---------------------------------------------------------------------------
# the absorber profile (Sec. IV, eq60) and the dense GMRES solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("degree", [0, 1, 2, 4])
def test_sigma_monomial_profile(degree):
    """sigma = sigma0 s^d with s = dir (x - x0)/L: zero before the absorber,
    sigma0 beyond its end, and inside exactly the monomial of degree d
    (a least-squares polynomial fit in s recovers sigma0 at degree d and
    nothing else); both directions."""
    w = synth.workload_small(edge=0.2, length=3.0)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    x = o.qp[:, 0]
    for direction, x0 in ((+1, 1.7), (-1, 1.3)):
        sig0, L = 0.83, 0.9
        o.set_sigma([synth.SigmaEnd(axis=0, x0=x0, length=L, direction=direction, degree=degree, sigma0=sig0)])
        s = direction * (x - x0) / L
        before, inside, after = s < 0, (s > 0) & (s < 1), s > 1
        assert np.all(o.sigma[before] == 0)
        assert np.allclose(o.sigma[after], sig0, rtol=0, atol=1e-15)
        coef = np.polynomial.polynomial.polyfit(s[inside], o.sigma[inside], 5)
        want = np.zeros(6)
        want[degree] = sig0
        assert np.allclose(coef, want, atol=1e-9), coef
        assert inside.sum() > 20


def test_sigma_piecewise_linear_profile():
    """Piecewise-linear profile: the hat-function interpolant of the control
    values at s_k = k/(n-1), i.e. numpy's linear interpolation; held at the
    last control value beyond the end, zero before the start; two absorbers
    add."""
    w = synth.workload_small(edge=0.2, length=3.0)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    x = o.qp[:, 0]
    ctrl = synth.random_uniform(31, 9, 0.0, 2.0)
    ctrl2 = synth.random_uniform(32, 5, 0.0, 1.0)
    e1 = synth.SigmaEnd(axis=0, x0=2.0, length=0.8, direction=+1, ctrl=ctrl)
    e2 = synth.SigmaEnd(axis=0, x0=1.2, length=1.0, direction=-1, ctrl=ctrl2)
    o.set_sigma([e1, e2])
    s1 = (x - 2.0) / 0.8
    s2 = -(x - 1.2) / 1.0
    ref = np.where(s1 >= 0, np.interp(np.clip(s1, 0, 1), np.linspace(0, 1, 9), ctrl), 0.0)
    ref += np.where(s2 >= 0, np.interp(np.clip(s2, 0, 1), np.linspace(0, 1, 5), ctrl2), 0.0)
    assert np.allclose(o.sigma, ref, rtol=0, atol=1e-14)
    # its Jacobian with respect to the control values is the hat basis
    J = o.pwl_jacobian(e1)
    for k in range(9):
        e = np.zeros(9)
        e[k] = 1.0
        hat = np.where(s1 >= 0, np.interp(np.clip(s1, 0, 1), np.linspace(0, 1, 9), e), 0.0)
        assert np.allclose(J[:, k], hat, rtol=0, atol=1e-14)


def test_gmres_dense_matches_lu():
    """Unrestarted GMRES on the dense matrix (configuration 0's solver)
    reaches the LU solution: residual 1e-11, solution to 1e-7."""
    w = synth.workload_small(length=2.0, absorber=1.0)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    A = o.dense()
    b = o.rhs_dipole(w.dipoles[0])
    x_lu = oracle.lu_solve(A, b)
    x_g = oracle.gmres_dense(A, b, tol=1e-11)
    assert np.linalg.norm(A @ x_g - b) < 2e-11 * np.linalg.norm(b)
    assert np.linalg.norm(x_g - x_lu) < 1e-7 * np.linalg.norm(x_lu)


def test_dense_rows_equal_dense_matrix_rows():
    """or_dense_rows (the pairs of the selected rows' test triangles only)
    against the full dense assembly on the 4-long guide: E, H and eq14 rows
    of sigma-free and absorber edges, in a scrambled order."""
    w = synth.workload_small()
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    A = o.dense()
    rE, rH, r14 = o.edge_rows()
    ls = np.nonzero(o.isR == 0)[0][[3, 100]]
    rs = np.nonzero(o.isR != 0)[0][[5, 200]]
    rows = np.array([rH[ls[1]], rE[ls[0]], r14[rs[0]], rE[rs[1]], rH[rs[0]], r14[rs[1]]])
    R = o.dense_rows(rows)
    err = np.max(np.abs(R - A[rows])) / np.max(np.abs(A[rows]))
    assert err < 1e-13, err
