"""GPU parity of the transposed operator, the pointwise one-sided fields, the
off-surface field evaluation and the adjoint sigma gradient with the oracle,
through the C ABI.  Same tolerances as the forward parity tests: FP64 1e-10
relative (same discrete operator, summation order differs), FP32 2e-5; the
gradient, a product of two solves, 1e-6 relative to its largest entry."""
import copy

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _set_ctrl(end):
    def set_params(ctx, values):
        e = copy.copy(end)
        e.ctrl = np.asarray(values, float)
        ctx.set_sigma([e])
    return set_params


@pytest.fixture(scope="module")
def grad_case():
    import torch
    import paper_1004_5076_amd as pk
    assert torch.cuda.is_available()
    w = synth.workload_gradient(guide_len=0.8, absorber=1.2, edge=0.15, n_ctrl=8, n_monitor=6)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    P = o.pfft(w.h, w.r_near)
    ctx = pk.context_for(w)
    print("gradient case N", ctx.N, flush=True)
    return w, o, P, ctx


def _vec(seed, n):
    return synth.random_complex(seed, n)


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 2e-5)])
def test_transpose_matches_oracle(grad_case, prec, tol):
    import torch
    w, o, P, ctx = grad_case
    assert ctx.N == o.N
    z = _vec(31, o.N)
    y = ctx.matvec(torch.from_numpy(z).cuda(), prec=prec, transpose=True).cpu().numpy()
    ref = P.rmatvec(z)
    print("transpose prec", prec, "rel", _rel(y, ref), flush=True)
    assert _rel(y, ref) < tol


def test_transpose_bilinear_identity_gpu(grad_case):
    import torch
    w, o, P, ctx = grad_case
    x = torch.from_numpy(_vec(41, ctx.N)).cuda()
    y = torch.from_numpy(_vec(42, ctx.N)).cuda()
    a = (y * ctx.matvec(x)).sum().item()
    b = (x * ctx.matvec(y, transpose=True)).sum().item()
    assert abs(a - b) <= 1e-12 * abs(a)


def test_transpose_solve(grad_case):
    import torch
    import paper_1004_5076_amd as pk
    w, o, P, ctx = grad_case
    g = torch.from_numpy(_vec(51, ctx.N)).cuda()
    for mode in (pk.SCABS_FP64, pk.SCABS_MIXED):
        lam, info = ctx.solve(g, tol=1e-10, restart=120, mode=mode, max_iter=5000, transpose=True)
        print("transpose solve", mode, info, flush=True)
        assert info["status"] == 0
        r = np.linalg.norm(P.rmatvec(lam.cpu().numpy()) - g.cpu().numpy()) / np.linalg.norm(g.cpu().numpy())
        assert r < 1e-9


def test_point_fields_match_oracle(grad_case):
    import torch
    w, o, P, ctx = grad_case
    x = _vec(61, o.N)
    Ee, Ei = ctx.point_fields(torch.from_numpy(x).cuda())
    Re, Ri = P.point_fields(x)
    # exact on triangles carrying an absorber edge (the points the gradient reads)
    tri = np.repeat(np.arange(o.nt), oracle.NQ)
    sel = (o.isR[o.tedge[tri]] != 0).any(axis=1)
    for g, r in ((Ee.cpu().numpy(), Re), (Ei.cpu().numpy(), Ri)):
        err = np.max(np.abs(g[sel] - r[sel])) / np.max(np.abs(r[sel]))
        print("point fields rel", err, flush=True)
        assert err < 1e-10


def test_eval_field_matches_oracle(grad_case):
    import torch
    w, o, P, ctx = grad_case
    x = _vec(71, o.N)
    xs = w.notes["monitor_x"]
    pts = np.stack([xs, 0.02 * np.ones_like(xs), -0.01 * np.ones_like(xs)], 1)
    for region in (-1, 0):
        E, H = ctx.eval_field(torch.from_numpy(x).cuda(), pts, region)
        Er, Hr = o.fields_at(x, pts, region)
        assert _rel(E.cpu().numpy(), Er) < 1e-11 and _rel(H.cpu().numpy(), Hr) < 1e-11
        wE = _vec(72, 3 * len(xs)).reshape(-1, 3)
        q = ctx.eval_field_transpose(pts, region, torch.from_numpy(wE).cuda()).cpu().numpy()
        Q = o.field_matrix(pts, region)
        assert _rel(q, Q.T @ wE.ravel()) < 1e-11


def test_sigma_gradient_matches_oracle(grad_case):
    """Full adjoint gradient of the reflected amplitude |b|^2 at the monitor
    points: GPU (FP64 solves, transposed solve, gradient kernel, chain rule)
    against the oracle's pFFT-operator gradient on the same inputs."""
    import torch
    import paper_1004_5076_amd as pk
    w, o, P, ctx = grad_case
    d = w.dipoles[0]
    xs, beta = w.notes["monitor_x"], w.notes["beta"]
    pts = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], 1)
    wts = oracle.monitor_weights(xs, beta)
    # oracle
    b = o.rhs_dipole(d)
    x_or = P.solve(b, tol=1e-13)
    Einc_m = np.array([oracle.dipole_field(o.k_i, o.Z_i, d.pos, d.moment, p)[0] for p in pts])
    q = wts @ o.field_matrix(pts, 0).reshape(len(xs), 3, o.N)[:, 1, :]
    bh = wts @ Einc_m[:, 1] + q @ x_or
    g = np.conj(bh) * q
    lam_or = P.solve_t(g, tol=1e-13)
    Ee, Ei = P.point_fields(x_or)
    Einc, _ = o.incident_at_points(d)
    dfs_or = o.sigma_gradient_points(lam_or, Ee, Ei, Einc)
    grad_or = o.pwl_jacobian(w.sigma[0]).T @ dfs_or
    # GPU
    bg = ctx.rhs_dipole(d.pos, d.moment, d.body)
    x, info = ctx.solve(bg, tol=1e-12, restart=200, mode=pk.SCABS_FP64, max_iter=5000)
    assert info["status"] == 0
    wE = np.zeros((len(xs), 3), complex)
    wE[:, 1] = wts
    qg = ctx.eval_field_transpose(pts, 0, torch.from_numpy(wE).cuda())
    E, _ = ctx.eval_field(x, pts, 0)
    bh_g = (torch.from_numpy(wts).cuda() * (torch.from_numpy(Einc_m[:, 1]).cuda() + E[:, 1])).sum()
    gg = torch.conj(bh_g) * qg
    lam, info = ctx.solve(gg.contiguous(), tol=1e-12, restart=200, mode=pk.SCABS_FP64, max_iter=5000, transpose=True)
    assert info["status"] == 0
    einc = ctx.incident_dipole_points(d.pos, d.moment, d.body)
    dfs, grad = ctx.sigma_gradient(x, lam, einc)
    print("grad gpu", grad, "oracle", grad_or, flush=True)
    # the library's dipole field at the monitor points is the closed form the
    # oracle evaluates (zero outside the dipole's body)
    Ed, _ = ctx.dipole_field(d.pos, d.moment, d.body, pts, 0)
    assert _rel(Ed.cpu().numpy(), Einc_m) < 1e-13
    E0, _ = ctx.dipole_field(d.pos, d.moment, d.body, pts, -1)
    assert E0.abs().max().item() == 0
    # one call: adjoint solve and gradient together
    dfs1, grad1, info1 = ctx.gradient(x, gg.contiguous(), einc, tol=1e-12, restart=200, max_iter=5000)
    assert info1["status"] == 0
    assert np.max(np.abs(grad1 - grad)) <= 1e-8 * np.max(np.abs(grad))
    assert abs(bh_g.item() - bh) < 1e-9 * abs(bh)
    assert np.max(np.abs(grad - grad_or)) <= 1e-6 * np.max(np.abs(grad_or))
    scale = np.max(np.abs(dfs_or))
    assert np.max(np.abs(dfs.cpu().numpy() - dfs_or)) <= 1e-6 * scale


def test_autograd_matches_central_differences(grad_case):
    """torch.autograd through the differentiable solve and field evaluation
    against central differences of the same GPU objective (each a rebuild and
    a re-solve)."""
    import torch
    import paper_1004_5076_amd as pk
    w, o, P, _ = grad_case
    ctx = pk.context_for(w)
    end = w.sigma[0]
    d = w.dipoles[0]
    xs, beta = w.notes["monitor_x"], w.notes["beta"]
    pts = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], 1)
    Einc_y = torch.from_numpy(np.array([oracle.dipole_field(o.k_i, o.Z_i, d.pos, d.moment, p)[0][1]
                                        for p in pts])).cuda()
    set_params = _set_ctrl(end)

    def objective(params):
        x = pk.sigma_solve(params, ctx, set_params, d, tol=1e-12, restart=200, mode=pk.SCABS_FP64)
        E = pk.field_at(x, ctx, pts, 0)
        return pk.reflected_amplitude(Einc_y + E[:, 1], xs, beta).abs() ** 2

    p0 = torch.tensor(end.ctrl, dtype=torch.float64, requires_grad=True)
    f = objective(p0)
    f.backward()
    grad = p0.grad.numpy()
    scale = np.max(np.abs(grad))
    dl = 1e-5
    for k in (0, 5):
        pp, pm = end.ctrl.copy(), end.ctrl.copy()
        pp[k] += dl
        pm[k] -= dl
        with torch.no_grad():
            fd = (objective(torch.tensor(pp)).item() - objective(torch.tensor(pm)).item()) / (2 * dl)
        print("autograd k", k, grad[k], "fd", fd, flush=True)
        assert abs(fd - grad[k]) <= 2e-6 * scale
