"""The block-Toeplitz product at the benchmark size (two 30-long channels,
N = 102 852, autotuned as bench.py sets it up) against the oracle's dense
Galerkin matrix on sampled rows (each assembled from its test triangles'
pairs by or_dense_rows): E, H and eq14 rows of periodic edges in both
channels, of end-cap edges and of absorber edges at both ends.  Checked: the
FP64 and FP32 products of a seeded vector and the FP32 product of a seeded
batch of 8 (the matrix-core form) at those rows, and whole rows from the
transposed product of unit vectors (FP64, and FP32 one at a time and as a
batch of 8).  Scale of a row's error: the sum of the
magnitudes of its terms."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _sample_rows(w, o):
    """rows of edges picked by where their triangles lie"""
    cen = w.mesh.verts[w.mesh.tris].mean(axis=1)
    nrm = o.nrm
    rE, rH, r14 = o.edge_rows()
    picks = []
    xs = cen[:, 0]
    crit = [
        (np.abs(xs - 15.0) < 0.05) & (cen[:, 1] < 0),              # mid-guide, channel 0
        (np.abs(xs - 12.3) < 0.05) & (cen[:, 1] > 0),              # mid-guide, channel 1
        (np.abs(nrm[:, 0]) > 0.9) & (xs < 0.01),                    # end cap at x = 0
        (np.abs(nrm[:, 0]) > 0.9) & (xs > 29.99) & (cen[:, 1] > 0), # end cap at x = 30
        (np.abs(xs - 28.5) < 0.05),                                 # absorber near x = 30
        (np.abs(xs - 1.2) < 0.05) & (cen[:, 1] > 0),                # absorber near x = 0
    ]
    for c in crit:
        T = np.nonzero(c)[0]
        assert len(T) > 0
        e = o.tedge[T[len(T) // 2], 0]
        picks.append(e)
    rows = []
    for e in picks:
        rows += [rE[e], rH[e]]
        if o.isR[e]:
            rows.append(r14[e])
    return np.array(rows), picks


@pytest.fixture(scope="module")
def big():
    import paper_1004_5076_amd as pk
    w = synth.workload_two_channel(edge=0.072)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    ctx = pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ)
    ctx.autotune(3)
    rows, edges = _sample_rows(w, o)
    R = o.dense_rows(rows)
    print("N", ctx.N, "sampled rows", len(rows), "edges", edges, "absorber", [int(o.isR[e]) for e in edges],
          flush=True)
    return w, o, ctx, rows, R


def _check(y_rows, R, x, tol, what):
    ref = R @ x
    scale = np.abs(R) @ np.abs(x)
    err = np.max(np.abs(y_rows - ref) / scale)
    print(what, "max error / row scale", err, flush=True)
    assert err < tol, what


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 1e-6)])
def test_product_at_sampled_rows(big, prec, tol):
    import torch
    w, o, ctx, rows, R = big
    x = synth.random_complex(1201, o.N)
    y = ctx.matvec(torch.from_numpy(x).cuda(), prec=prec).cpu().numpy()
    _check(y[rows], R, x, tol, "prec %d" % prec)


def test_batched_fp32_product_at_sampled_rows(big):
    import torch
    w, o, ctx, rows, R = big
    X = np.stack([synth.random_complex(1300 + k, o.N) for k in range(8)])
    Y = ctx.matvec(torch.from_numpy(X).cuda(), prec=1).cpu().numpy()
    for k in range(8):
        _check(Y[k, rows], R, X[k], 1e-6, "batch vector %d" % k)


def test_fp32_and_batched_transposed_products_give_rows(big):
    """FP32 transposed products of unit vectors, one at a time and as one
    batch of 8 (the batched instances), against the dense rows: error per
    row scaled by the sum of the row's magnitudes."""
    import torch
    w, o, ctx, rows, R = big
    ks = list(range(min(8, len(rows))))
    E = np.zeros((len(ks), o.N), complex)
    for n, k in enumerate(ks):
        E[n, rows[k]] = 1.0
    Ed = torch.from_numpy(E).cuda()
    Y8 = ctx.matvec(Ed, prec=1, transpose=True).cpu().numpy()
    for n, k in enumerate(ks):
        y1 = ctx.matvec(Ed[n].clone(), prec=1, transpose=True).cpu().numpy()
        scale = np.sum(np.abs(R[k]))
        e1 = np.max(np.abs(y1 - R[k])) / scale
        e8 = np.max(np.abs(Y8[n] - R[k])) / scale
        print("row", rows[k], "FP32 transposed: single", e1, "batched", e8, flush=True)
        assert e1 < 1e-6 and e8 < 1e-6


def test_transposed_product_gives_rows(big):
    import torch
    w, o, ctx, rows, R = big
    for k in (0, 3, len(rows) - 1):
        e = np.zeros(o.N, complex)
        e[rows[k]] = 1.0
        r = ctx.matvec(torch.from_numpy(e).cuda(), prec=0, transpose=True).cpu().numpy()
        err = np.max(np.abs(r - R[k])) / np.max(np.abs(R[k]))
        print("row", rows[k], "from the transposed product: max rel", err, flush=True)
        assert err < 1e-12
