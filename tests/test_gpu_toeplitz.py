"""The block-Toeplitz product (fast-solver appendix) against the oracle's dense
Galerkin matrix (Appendix A, eq19), through the C ABI.  On a mesh that repeats
along x the product is the discrete Galerkin operator itself (no lattice), so
FP64 products match A x to rounding (1e-11 relative, every row block on its
own), FP32 products to single precision (2e-6), and solves match the LU
solution of A to the solve tolerance."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _blocks(o):
    NL, NR = o.NL, o.NR
    return [(0, NL), (NL, 2 * NL), (2 * NL, 2 * NL + NR), (2 * NL + NR, 2 * NL + 2 * NR), (2 * NL + 2 * NR, o.N)]


def _section():
    w = synth.workload_two_channel(length=1.0, absorber=0.5, edge=0.072)
    w.sigma = [synth.SigmaEnd(axis=0, x0=0.5, length=0.5, direction=+1, degree=4, sigma0=1.0)]
    w.dipoles = [synth.seeded_dipole(2000, base=(0.25, -0.35, 0.0), jitter=(0.05, 0.02, 0.02), body=0)]
    w.h = 30.0 / 508
    w.r_near = 3.61 * w.h
    return w


def _rotated():
    """The 4-long guide with the vertex lists of every 5th triangle between
    x = 1 and x = 2 rotated (same orientation): those triangles' quadrature
    points and local edges no longer follow the ring template's numbering,
    so ring detection must leave them out and their pairs become stored
    entries; the product stays exact."""
    w = synth.workload_small()
    t = w.mesh.tris.copy()
    cx = w.mesh.verts[t].mean(axis=1)[:, 0]
    sel = np.nonzero((cx > 1.0) & (cx < 2.0))[0][::5]
    t[sel] = t[sel][:, [1, 2, 0]]
    w.mesh.tris = t
    return w


CASES = {
    "guide4": synth.workload_small,    # one guide, quadratic absorber on [2, 4], 27 rings
    "section": _section,               # two channels, quartic absorber, 14 rings
    "rotated": _rotated,               # guide4 with part of the triangles renumbered
    # 30 rings: circulant length 64, a multiple of 8, so the per-frequency
    # kernels take their XCD-ordered grids
    "guide44": lambda: synth.workload_small(length=4.4),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    import paper_1004_5076_amd as pk
    w = CASES[request.param]()
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    A = o.dense()
    ctx = pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ)
    info = ctx.info()
    print(request.param, "info", info, flush=True)
    return request.param, w, o, A, ctx


def test_layout_and_rings(case):
    name, w, o, A, ctx = case
    info = ctx.info()
    assert info["product"] == 1 and info["N"] == o.N
    assert info["rings"] >= 3 and info["circulant_length"] >= 2 * info["rings"] - 1
    if name == "guide44":
        assert info["circulant_length"] % 8 == 0


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-6)])
def test_product_matches_dense_galerkin(case, prec, tol):
    import torch
    name, w, o, A, ctx = case
    for seed in (81, 82):
        x = synth.random_complex(seed, o.N)
        ref = A @ x
        y = ctx.matvec(torch.from_numpy(x).cuda(), prec=prec).cpu().numpy()
        for a, b in _blocks(o):
            e = _rel(y[a:b], ref[a:b])
            print(name, "prec", prec, "rows", a, b, "rel err", e, flush=True)
            assert e < tol, (a, b)


def test_unit_columns(case):
    """Single columns (periodic and non-periodic edges, J and M, L and R):
    a misplaced unknown or a wrong template sign shows up here."""
    import torch
    name, w, o, A, ctx = case
    rng = synth.SplitMix64(83)
    cols = sorted({int(rng.uniform() * o.N) for _ in range(12)} | {0, o.NL, o.N - 1})
    for col in cols:
        x = np.zeros(o.N, complex)
        x[col] = 1.0
        y = ctx.matvec(torch.from_numpy(x).cuda(), prec=0).cpu().numpy()
        assert _rel(y, A[:, col]) < 1e-11, col


def test_batched_equals_single(case):
    """Batches of 5 vectors (the same arithmetic per vector as single ones)
    give each vector its single product; batches of 8 in FP32 run the
    per-frequency products on the matrix cores and match the dense matrix to
    single precision."""
    import torch
    name, w, o, A, ctx = case
    X = np.stack([synth.random_complex(90 + k, o.N) for k in range(8)])
    for prec in (0, 1):
        Y = ctx.matvec(torch.from_numpy(X[:5].copy()).cuda(), prec=prec).cpu().numpy()
        for k in range(5):
            y1 = ctx.matvec(torch.from_numpy(X[k].copy()).cuda(), prec=prec).cpu().numpy()
            assert _rel(Y[k], y1) < 1e-13
    for prec, tol in ((0, 1e-11), (1, 2e-6)):
        Y = ctx.matvec(torch.from_numpy(X).cuda(), prec=prec).cpu().numpy()
        for k in range(8):
            ref = A @ X[k]
            for a, b in _blocks(o):
                assert _rel(Y[k][a:b], ref[a:b]) < tol, (prec, k, a, b)


@pytest.mark.parametrize("mode", [0, 2])
def test_solve_matches_dense_lu(case, mode):
    """Solves with the exact product reach the LU solution of the dense
    Galerkin system (the 1e-6 target), in FP64 and in mixed precision."""
    import torch
    import paper_1004_5076_amd as pk
    name, w, o, A, ctx = case
    b = o.rhs_dipole(w.dipoles[0])
    x_lu = oracle.lu_solve(A, b)
    x, info = ctx.solve(torch.from_numpy(b).cuda(), tol=1e-11, max_iter=4000, restart=200, mode=mode)
    print(name, "mode", mode, info, flush=True)
    assert info["status"] == 0
    err = _rel(x.cpu().numpy(), x_lu)
    print(name, "mode", mode, "solution vs dense LU", err, flush=True)
    assert err < 1e-8


def test_every_launch_choice_is_exact(case):
    """The tunable launch choices (apply form, column groups of the sparse
    rows, transform lines per work-group, the sparse parts on the second
    stream) change only the order of sums: every one keeps the products
    exact, forward and transposed, and the overlap changes no bit."""
    import torch
    name, w, o, A, ctx = case
    X = np.stack([synth.random_complex(200 + k, o.N) for k in range(8)])
    R1 = A @ X[0]
    R8 = X @ A.T
    T1 = A.T @ X[0]
    T8 = X @ A
    Xd = torch.from_numpy(X).cuda()
    for cls in (0, 1):
        for form in ((0,) if cls == 0 else (0, 1)):
            for groups in (1, 3, 16):
                for lines in (1, 2, 0):
                    outs = []
                    for overlap in (0, 1):
                        ctx.set_tune(cls, form, groups, lines, overlap)
                        key = (cls, form, groups, lines, overlap)
                        if cls == 0:
                            y = ctx.matvec(Xd[0].clone(), prec=0)
                            yt = ctx.matvec(Xd[0].clone(), prec=0, transpose=True)
                            assert _rel(y.cpu().numpy(), R1) < 1e-11, key
                            assert _rel(yt.cpu().numpy(), T1) < 1e-11, key
                        else:
                            y = ctx.matvec(Xd, prec=1)
                            yt = ctx.matvec(Xd, prec=1, transpose=True)
                            assert _rel(y.cpu().numpy(), R8) < 2e-6, key
                            assert _rel(yt.cpu().numpy(), T8) < 2e-6, key
                        outs.append((y, yt))
                    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]), key
    ctx.set_tune(0, 0, 8, 0)
    ctx.set_tune(1, 0, 8, 0)
    import paper_1004_5076_amd as pk
    with pytest.raises(pk.ScabsError):
        ctx.set_tune(1, 2, 8, 0)
    with pytest.raises(pk.ScabsError):
        ctx.set_tune(0, 0, 17, 0)
    with pytest.raises(pk.ScabsError):
        ctx.set_tune(0, 0, 8, 0, 2)


def test_autotune_keeps_fastest(case):
    import torch
    name, w, o, A, ctx = case
    recs = ctx.autotune(reps=2)
    print(name, "autotune", recs, flush=True)
    for nrhs in (1, 8):
        rs = [r for r in recs if r["nrhs"] == nrhs]
        assert len(rs) >= 3
        chosen = [r for r in rs if r["chosen"]]
        assert len(chosen) == 1 and chosen[0]["us"] == min(r["us"] for r in rs)
    x = synth.random_complex(210, o.N)
    y = ctx.matvec(torch.from_numpy(x).cuda(), prec=0).cpu().numpy()
    assert _rel(y, A @ x) < 1e-11


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-6)])
def test_transposed_product_matches_dense(case, prec, tol):
    """A^T z with the transposed block-Toeplitz product (circulant at -f,
    transposed sigma tests, local terms and stored entries) against the
    oracle's dense matrix, per column block."""
    import torch
    name, w, o, A, ctx = case
    for seed in (85, 86):
        z = synth.random_complex(seed, o.N)
        ref = A.T @ z
        y = ctx.matvec(torch.from_numpy(z).cuda(), prec=prec, transpose=True).cpu().numpy()
        for a, b in _blocks(o):
            e = _rel(y[a:b], ref[a:b])
            print(name, "transposed prec", prec, "cols", a, b, "rel err", e, flush=True)
            assert e < tol, (a, b)


def test_transposed_solve_matches_dense_lu(case):
    import torch
    import paper_1004_5076_amd as pk
    name, w, o, A, ctx = case
    g = synth.random_complex(87, o.N)
    lam, info = ctx.solve(torch.from_numpy(g).cuda(), tol=1e-11, max_iter=4000, restart=200, mode=pk.SCABS_MIXED,
                          transpose=True)
    assert info["status"] == 0, info
    ref = oracle.lu_solve(A.T.copy(), g)
    assert _rel(lam.cpu().numpy(), ref) < 1e-8


def test_transposed_bilinear_identity(case):
    """y^T (A x) = x^T (A^T y) with both block-Toeplitz products, FP64."""
    import torch
    name, w, o, A, ctx = case
    x = torch.from_numpy(synth.random_complex(88, o.N)).cuda()
    y = torch.from_numpy(synth.random_complex(89, o.N)).cuda()
    a = (y * ctx.matvec(x)).sum().item()
    b = (x * ctx.matvec(y, transpose=True)).sum().item()
    assert abs(a - b) <= 1e-12 * abs(a)


def test_rebuilds_keep_products_exact(case):
    """Rebuilding a context releases all its device memory; the per-vector
    buffers the products grow afterwards must be fresh ones.  Single, 8-vector
    and transposed products in both precisions after each of three rebuilds
    equal those after the first build bit for bit."""
    import torch
    name, w, o, A, ctx = case
    x = torch.from_numpy(synth.random_complex(95, o.N)).cuda()
    X = torch.from_numpy(np.stack([synth.random_complex(96 + i, o.N) for i in range(8)])).cuda()

    def products():
        return [ctx.matvec(x, prec=p) for p in (0, 1)] + [ctx.matvec(X, prec=p) for p in (0, 1)] + \
               [ctx.matvec(x, prec=p, transpose=True) for p in (0, 1)]

    ref = [y.clone() for y in products()]
    for _ in range(3):
        ctx.build()
        for a, b in zip(products(), ref):
            assert torch.equal(a, b)
    assert _rel(ref[0].cpu().numpy(), A @ x.cpu().numpy()) < 1e-11


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-6)])
def test_batched_transposed_products(case, prec, tol):
    """Transposed products of 3 and 8 vectors at once (tables and stored
    entries read once for all of them) equal the single-vector products and
    the dense A^T."""
    import torch
    name, w, o, A, ctx = case
    for nb in (3, 8):
        Z = np.stack([synth.random_complex(1400 + 10 * nb + k, o.N) for k in range(nb)])
        Y = ctx.matvec(torch.from_numpy(Z).cuda(), prec=prec, transpose=True).cpu().numpy()
        for k in range(nb):
            y1 = ctx.matvec(torch.from_numpy(Z[k]).cuda(), prec=prec, transpose=True).cpu().numpy()
            d = np.max(np.abs(Y[k] - y1)) / np.max(np.abs(y1))
            assert d <= (1e-15 if prec == 0 else 1e-6), (nb, k, d)
            assert _rel(Y[k], A.T @ Z[k]) < tol


def test_batched_transposed_solve(case):
    import torch
    import paper_1004_5076_amd as pk
    name, w, o, A, ctx = case
    G = np.stack([synth.random_complex(1500 + k, o.N) for k in range(3)])
    lam, infos = ctx.solve(torch.from_numpy(G).cuda(), tol=1e-10, max_iter=4000, restart=200, mode=pk.SCABS_MIXED,
                           transpose=True)
    assert all(i["status"] == 0 for i in infos)
    for k in range(3):
        assert _rel(lam[k].cpu().numpy(), oracle.lu_solve(A.T.copy(), G[k])) < 1e-8
