"""HIP graphs of the Arnoldi step (scabs_set_graphs): solves whose per-step
preconditioner + product launches are replayed from a captured graph equal
the solves with ordinary launches bit for bit -- FP64 and mixed, forward and
transposed, 1, 3 and 8 right-hand sides, block-Toeplitz and lattice
contexts, the block-Toeplitz sparse parts on the second stream or not, the
Schwarz and the circulant + Schwarz preconditioners -- over
several solves in a row (hundreds of replays, each between the host's
read-backs and the eager Gram-Schmidt launches) and across batch-size
changes (buffers regrown, graphs dropped and captured again), and inside
scabs_solve_batched (one capturing thread per context).  Wall times with and
without graphs are printed for the batched-form contexts."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _rhs(ctx, n, seed):
    import torch
    return torch.from_numpy(np.stack([synth.random_complex(seed + k, ctx.N) for k in range(n)])).cuda()


def _solve(ctx, b, mode, trans, max_iter=3000):
    return ctx.solve(b, tol=1e-8 if mode == 0 else 1e-6, max_iter=max_iter, restart=120, mode=mode, transpose=trans)


def _compare(ctx, cases, max_iter=3000):
    import torch
    for mode, trans, n in cases:
        b = _rhs(ctx, n, 700 + n)
        ctx.set_graphs(False)
        x0, i0 = _solve(ctx, b, mode, trans, max_iter)
        ctx.set_graphs(True)
        for rep in range(2):            # capture on the first step, replays after
            x1, i1 = _solve(ctx, b, mode, trans, max_iter)
            assert torch.equal(x0, x1), (mode, trans, n, rep)
            assert i0 == i1
        print("mode", mode, "transpose", trans, "nrhs", n, "steps", [i["inner_iters"] for i in i0], flush=True)


@pytest.fixture(scope="module")
def toe_ctx():
    import paper_1004_5076_amd as pk
    return pk.context_for(synth.workload_small(), device=0, product=pk.SCABS_PRODUCT_TOEPLITZ)


@pytest.mark.parametrize("mode", [0, 2])
def test_toeplitz_graph_solves_equal_eager(toe_ctx, mode):
    _compare(toe_ctx, [(mode, False, 1), (mode, False, 3), (mode, False, 8), (mode, True, 1), (mode, False, 1)])


def test_graphs_with_second_stream_equal_eager():
    """With the stored entries' sparse parts on the context's second stream
    (overlap 1), the captured graphs take that stream in through the fork and
    join events; the solves still equal the eager ones bit for bit."""
    import paper_1004_5076_amd as pk
    ctx = pk.context_for(synth.workload_small(), device=0, product=pk.SCABS_PRODUCT_TOEPLITZ)
    for cls in (0, 1):
        ctx.set_tune(cls, 0, 8, 0, 1)
    _compare(ctx, [(2, False, 8), (2, False, 1), (2, True, 1), (0, True, 8), (0, False, 3)])
    ctx.close()


def test_lattice_graph_solves_equal_eager():
    import paper_1004_5076_amd as pk
    ctx = pk.context_for(synth.workload_small(), device=0)
    _compare(ctx, [(2, False, 1), (2, False, 8), (2, True, 1), (0, True, 1)])
    ctx.close()


def test_circulant_preconditioner_graph_solves_equal_eager():
    import paper_1004_5076_amd as pk
    w = synth.workload_small()
    ctx = pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ, precond=3)
    # the circulant preconditioner converges slowly with an absorber: a bounded
    # number of steps, compared whatever the outcome
    _compare(ctx, [(2, False, 1), (2, False, 8), (2, True, 1)], max_iter=300)
    ctx.close()


def test_batched_solve_with_graphs_and_timing():
    import torch
    import paper_1004_5076_amd as pk
    import test_gpu_batched_form as bf
    ws = bf._workloads()[::4]        # 8 of the 32 batched-form contexts (each absorber, two wavelengths)
    ctxs = [pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ) for w in ws]
    dips = [synth.seeded_dipole(900 + k, base=(0.5, 0.0, 0.0)) for k in range(8)]
    bs = [torch.stack([c.rhs_dipole(d.pos, d.moment, d.body) for d in dips]).contiguous() for c in ctxs]
    res = {}
    for on in (False, True, True):
        for c in ctxs:
            c.set_graphs(on)
        torch.cuda.synchronize()
        t0 = time.time()
        xs, _ = pk.solve_batched(ctxs, bs, tol=1e-6, max_iter=6000, restart=400, mode=pk.SCABS_MIXED)
        torch.cuda.synchronize()
        t_b = time.time() - t0
        t0 = time.time()
        seq = [c.solve(b, tol=1e-6, max_iter=6000, restart=400, mode=pk.SCABS_MIXED)[0] for c, b in zip(ctxs, bs)]
        torch.cuda.synchronize()
        t_s = time.time() - t0
        print(f"graphs {on}: batched {t_b:.3f} s, one after another {t_s:.3f} s", flush=True)
        for a, b in zip(xs, seq):
            assert torch.equal(a, b)
        if on in res:
            for a, b in zip(xs, res[False]):
                assert torch.equal(a, b)
        res.setdefault(on, xs)
        for a, b in zip(res[on], res[False]):
            assert torch.equal(a, b)
    for c in ctxs:
        c.close()
