"""Field tools through the C ABI against the oracle on the same inputs: the
near-surface field evaluation, the Gaussian-beam source (Sec. II), the
standing-wave / reflection pipeline on the guide axis (Sec. I, Table I) and
the Poynting decay rate (Sec. III, eq_alpha_power)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GUIDE = (-0.2, 0.2, -0.1, 0.1)      # cross-section of synth.guide (0.4 x 0.2)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def guide4():
    import torch
    import paper_1004_5076_amd as pk
    w = synth.workload_small()
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    ctx = pk.context_for(w, device=0)
    src = synth.Beam(pos=np.array([0.25, 0.0, 0.0]), moment=np.array([0, 1.0, 0.2j]), body=0,
                     direction=(1.0, 0.0, 0.0), b=0.3)
    x = oracle.lu_solve(o.dense(), o.rhs_source(src))
    xd = torch.from_numpy(x).cuda()
    return w, o, ctx, src, x, xd


def _src(pk, s):
    return pk.Source.make(s.pos, s.moment, s.body, s.direction, s.b)


def test_beam_source_matches_oracle(guide4):
    import paper_1004_5076_amd as pk
    w, o, ctx, src, x, xd = guide4
    s = _src(pk, src)
    b = ctx.rhs_source(s).cpu().numpy()
    assert _rel(b, o.rhs_source(src)) < 1e-12
    pts = np.array([[0.9, 0.05, 0.02], [1.7, -0.1, 0.05], [3.0, 0.0, 0.0]])
    E, H = ctx.source_field(s, pts, 0)
    Eo, Ho = o.source_fields_at(src, pts, 0)
    assert _rel(E.cpu().numpy(), Eo) < 1e-12 and _rel(H.cpu().numpy(), Ho) < 1e-12
    Einc = ctx.incident_source_points(s).cpu().numpy()
    Eq, _ = o.source_fields_at(src, o.qp[:: 97], 0)
    assert _rel(Einc[:: 97], Eq) < 1e-12
    # b = 0 is the dipole of scabs_rhs_dipole, bit for bit
    d = w.dipoles[0]
    b0 = ctx.rhs_source(pk.Source.make(d.pos, d.moment, 0)).cpu().numpy()
    assert np.array_equal(b0, ctx.rhs_dipole(d.pos, d.moment, 0).cpu().numpy())


@pytest.mark.parametrize("region", [-1, 0])
def test_exact_fields_match_oracle(guide4, region):
    """Points from 0.004 to 1 away from the surface, on the region's side."""
    w, o, ctx, src, x, xd = guide4
    sgn = 1.0 if region < 0 else -1.0
    pts = np.array([[0.47, 0.13, 0.1 + sgn * 0.004], [1.61, 0.2 + sgn * 0.01, -0.02],
                    [2.33, -0.05, -0.1 - sgn * 0.05],
                    [3.1, 0.0, 0.0] if region == 0 else [3.1, 1.0, 0.4]])
    E, H = ctx.eval_field_exact(xd, pts, region)
    Eo, Ho = o.fields_at_exact(x, pts, region)
    assert _rel(E.cpu().numpy(), Eo) < 1e-10
    assert _rel(H.cpu().numpy(), Ho) < 1e-10


def test_axis_standing_wave_matches_oracle(guide4):
    """Total interior E_y on the axis over the lossless part: the library's
    SWR and standing-wave fit of the GPU fields equal the oracle's of its
    own fields."""
    import paper_1004_5076_amd as pk
    w, o, ctx, src, x, xd = guide4
    xs = np.linspace(0.8, 1.9, 24)
    pts = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], axis=1)
    E, _ = ctx.eval_field_exact(xd, pts, 0)
    Ei, _ = ctx.source_field(_src(pk, src), pts, 0)
    Ey = (E + Ei).cpu().numpy()[:, 1]
    Eo, _ = o.total_fields_at(x, src, pts, 0)
    assert _rel(Ey, Eo[:, 1]) < 1e-10
    s, r = pk.swr(Ey)
    so, ro = oracle.swr(Eo[:, 1])
    assert abs(s - so) < 1e-9 and abs(r - ro) < 1e-9
    fit = pk.standing_wave_fit(xs, Ey, 0.5 * o.k_i, o.k_i)
    fo = oracle.standing_wave_fit(xs, Eo[:, 1], 0.5 * o.k_i, o.k_i)
    print("axis fit (beta, |r|, residual)", fit[:3], "oracle", fo, flush=True)
    assert abs(fit[0] - fo[0]) < 1e-6 * fo[0] and abs(fit[1] - fo[1]) < 1e-6


def test_poynting_decay_matches_oracle(guide4):
    """eq_alpha_power on the plane x = 2.9 (inside the quadratic absorber)."""
    import paper_1004_5076_amd as pk
    w, o, ctx, src, x, xd = guide4
    box = (-0.6, 0.7, -0.5, 0.45)
    out = ctx.poynting_decay(xd, _src(pk, src), 0, 2.9, GUIDE, box, 6)
    ref = o.poynting_decay(x, src, 0, 2.9, GUIDE, box, 6, w.sigma)
    print("poynting (alpha, perimeter, boundary, flux A)", out, "oracle", ref, flush=True)
    for a, b in zip(out, ref):
        assert abs(a - b) < 1e-9 * max(abs(b), abs(ref[3])), (out, ref)
    assert out[1] > 0 and out[3] > 0
