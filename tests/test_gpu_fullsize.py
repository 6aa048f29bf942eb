"""Properties of the HIP path at the benchmark size (two 30-long channels,
N = 102 852, the launch configuration bench.py times), where the oracle is
too slow for element-wise parity: FP32 against FP64 products, batched against
single products, the transposed product against the product (bilinear
identity), and batched mixed-precision solves reaching 1e-6 with the FP64
operator."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    import paper_1004_5076_amd as pk
    assert torch.cuda.is_available()
    w = synth.workload_two_channel(edge=0.072)
    ctx = pk.context_for(w)
    print("benchmark size", ctx.info(), flush=True)
    return w, ctx


def _rel(a, b):
    import torch
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def test_fp32_product_close_to_fp64(big):
    import torch
    w, ctx = big
    x = torch.from_numpy(synth.random_complex(11, ctx.N)).cuda()
    y64 = ctx.matvec(x, prec=0)
    y32 = ctx.matvec(x, prec=1)
    err = _rel(y32, y64)
    print("fp32 vs fp64", err, flush=True)
    assert err < 2e-5


def test_batched_products_equal_single(big):
    import torch
    w, ctx = big
    X = torch.from_numpy(np.stack([synth.random_complex(20 + k, ctx.N) for k in range(8)])).cuda()
    for prec in (0, 1):
        Y = ctx.matvec(X, prec=prec)
        for k in (0, 3, 7):
            assert _rel(Y[k], ctx.matvec(X[k].clone(), prec=prec)) < 1e-13


def test_precond_apply_at_benchmark_size(big):
    """The Schwarz operator at full size (clusters up to 8192 ext / 4096 core
    unknowns): transpose identity, FP32 against FP64, batch against single."""
    from test_gpu_parity import _precond_checks
    w, ctx = big
    _precond_checks(ctx, 960, (8,))


def test_transpose_bilinear_identity(big):
    import torch
    w, ctx = big
    x = torch.from_numpy(synth.random_complex(31, ctx.N)).cuda()
    y = torch.from_numpy(synth.random_complex(32, ctx.N)).cuda()
    a = (y * ctx.matvec(x)).sum().item()
    b = (x * ctx.matvec(y, transpose=True)).sum().item()
    print("bilinear", a, b, flush=True)
    assert abs(a - b) <= 1e-11 * abs(a)


def test_batched_mixed_solves_reach_tolerance(big):
    import torch
    import paper_1004_5076_amd as pk
    w, ctx = big
    d0 = w.dipoles[0]
    dips = [d0, synth.seeded_dipole(601, base=(0.5, float(d0.pos[1]), 0.0), body=d0.body)]
    B = torch.stack([ctx.rhs_dipole(d.pos, d.moment, d.body) for d in dips]).contiguous()
    X, infos = ctx.solve(B, tol=1e-6, restart=240, mode=pk.SCABS_MIXED, max_iter=4000)
    print("solves", infos, flush=True)
    for k in range(2):
        assert infos[k]["status"] == 0
        r = _rel(ctx.matvec(X[k].contiguous(), prec=0), B[k])   # ||A x - b|| / ||b||
        assert r <= 1.0001e-6
