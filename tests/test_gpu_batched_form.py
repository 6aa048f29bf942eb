"""Batched form at its stated size: four guides of the benchmark's 0.4 x 0.2
cross-section (eps 12.25 in air, mesh edge 0.08) with an 8-long guide
before quartic absorbers of length 1, 2, 4 and 8 (N = 11 705 to 24 233),
each at 8 wavelengths spread over +-5% around the centre one, 8 seeded
dipoles in the first wavelength of the guide: 32 block-Toeplitz contexts of
uneven N, 256 systems, solved together by scabs_solve_batched in mixed
precision to 1e-6.  Checks: every system converged, its residual with the
exact FP64 operator is at the tolerance, and two members equal their
per-context solves bit for bit; the wall times of the batched and of the
per-context solves are printed."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GUIDE = 8.0
ABSORBERS = (1.0, 2.0, 4.0, 8.0)
EDGE = 0.08
N_EXPECTED = (11705, 13433, 17033, 24233)


def _workloads():
    ws = []
    for L in ABSORBERS:
        v, t = synth.guide(GUIDE + L, EDGE)
        mesh = synth.merge_bodies([(v, t)])
        for k in range(8):
            om = synth.OMEGA * (1.0 + 0.05 * (2.0 * k / 7.0 - 1.0))
            ws.append(synth.Workload("batched_L%g_w%d" % (L, k), mesh,
                                     [synth.SigmaEnd(axis=0, x0=GUIDE, length=L, direction=+1, degree=4,
                                                     sigma0=1.0)], [], h=0.05, r_near=0.3137, omega=om))
    return ws


def test_batched_form_full_size():
    import torch
    import paper_1004_5076_amd as pk
    ws = _workloads()
    t0 = time.time()
    ctxs = []
    for w in ws:
        ctxs.append(pk.context_for(w, device=0, product=pk.SCABS_PRODUCT_TOEPLITZ))
        if len(ctxs) % 8 == 0:
            print("built", len(ctxs), "contexts,", round(time.time() - t0, 1), "s", flush=True)
    assert tuple(ctxs[8 * i].N for i in range(4)) == N_EXPECTED
    dips = [synth.seeded_dipole(900 + k, base=(0.5, 0.0, 0.0)) for k in range(8)]
    bs = [torch.stack([c.rhs_dipole(d.pos, d.moment, d.body) for d in dips]).contiguous() for c in ctxs]
    torch.cuda.synchronize()
    t1 = time.time()
    xs, infos = pk.solve_batched(ctxs, bs, tol=1e-6, max_iter=6000, restart=400, mode=pk.SCABS_MIXED)
    torch.cuda.synchronize()
    t_batch = time.time() - t1
    iters = [[i["inner_iters"] for i in inf] for inf in infos]
    print(f"batched: 32 contexts x 8 systems, {t_batch:.2f} s; inner steps per context (max) "
          f"{[max(v) for v in iters]}", flush=True)
    for c, b, x, inf in zip(ctxs, bs, xs, infos):
        assert all(i["status"] == 0 for i in inf), inf
        r = b - c.matvec(x, prec=pk.SCABS_FP64)
        rel = (torch.linalg.norm(r, dim=1) / torch.linalg.norm(b, dim=1)).max().item()
        assert rel < 1.5e-6, (c.N, rel)
    # per-context solves of two members, and the sequential time of all
    t2 = time.time()
    seq = [c.solve(b, tol=1e-6, max_iter=6000, restart=400, mode=pk.SCABS_MIXED)[0] for c, b in zip(ctxs, bs)]
    torch.cuda.synchronize()
    t_seq = time.time() - t2
    print(f"per-context solves one after another: {t_seq:.2f} s (batched {t_batch:.2f} s)", flush=True)
    for i in (0, 31):
        assert torch.equal(seq[i], xs[i])
    for c in ctxs:
        c.close()
