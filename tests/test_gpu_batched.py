"""Several operators of uneven N solved together (scabs_solve_batched):
absorbers of different lengths and a second wavelength, with several dipoles
each.  The batched results equal the per-context solves (same kernels, same
order), and the smallest member's solution equals the LU solution of the
oracle's dense Galerkin system (block-Toeplitz product, exact)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _workloads():
    a = synth.workload_small(length=3.0, absorber=1.0)
    b = synth.workload_small(length=4.0, absorber=2.0)
    c = synth.workload_small(length=3.5, absorber=1.5, degree=3)
    c.omega = 1.1 * c.omega        # another wavelength
    return [a, b, c]


@pytest.fixture(scope="module")
def batch():
    import torch
    import paper_1004_5076_amd as pk
    ws = _workloads()
    ctxs = [pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ) for w in ws]
    nr = [2, 1, 3]
    bs = []
    for i, (w, c) in enumerate(zip(ws, ctxs)):
        ds = [synth.seeded_dipole(300 + 10 * i + k, base=(0.5, 0.0, 0.0)) for k in range(nr[i])]
        bs.append(torch.stack([c.rhs_dipole(d.pos, d.moment, 0) for d in ds]).contiguous())
    print("N", [c.N for c in ctxs], flush=True)
    return ws, ctxs, bs


@pytest.mark.parametrize("mode", [0, 2])
def test_batched_equals_per_context(batch, mode):
    import paper_1004_5076_amd as pk
    ws, ctxs, bs = batch
    xs, infos = pk.solve_batched(ctxs, bs, tol=1e-10, max_iter=3000, restart=200, mode=mode)
    for c, b, x, inf in zip(ctxs, bs, xs, infos):
        assert all(i["status"] == 0 for i in inf), inf
        x1, inf1 = c.solve(b, tol=1e-10, max_iter=3000, restart=200, mode=mode)
        err = float((x - x1).abs().max() / x1.abs().max())
        print("N", c.N, "batched vs single", err, [i["inner_iters"] for i in inf], flush=True)
        assert err < 1e-12


def test_batched_member_matches_oracle(batch):
    import paper_1004_5076_amd as pk
    ws, ctxs, bs = batch
    xs, _ = pk.solve_batched(ctxs, bs, tol=1e-11, max_iter=3000, restart=200, mode=pk.SCABS_MIXED)
    w = ws[0]
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    A = o.dense()
    for k in range(bs[0].shape[0]):
        ref = oracle.lu_solve(A, bs[0][k].cpu().numpy())
        got = xs[0][k].cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-8


def test_batched_rejects_a_repeated_context(batch):
    import paper_1004_5076_amd as pk
    ws, ctxs, bs = batch
    with pytest.raises(pk.ScabsError):
        pk.solve_batched([ctxs[0], ctxs[0]], [bs[0], bs[0]])
