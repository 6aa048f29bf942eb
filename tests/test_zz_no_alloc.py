"""The entry point that allocates nothing (scabs_eval_field_noalloc) against
scabs_eval_field, through the C ABI: two calls in a row, the second with
fewer points, and the size limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_eval_field_noalloc_matches_eval_field():
    import torch
    import paper_1004_5076_amd as pk
    assert torch.cuda.is_available()
    w = synth.workload_small(length=2.0, absorber=1.0)
    ctx = pk.context_for(w, device=0)
    x = torch.from_numpy(synth.random_complex(51, ctx.N)).cuda()
    rng = synth.SplitMix64(52)
    # off-surface exterior points, well away from the guide
    pts1 = np.array([[rng.uniform_range(-0.5, 2.5), rng.uniform_range(0.8, 1.5), rng.uniform_range(-0.6, 0.6)]
                     for _ in range(300)])
    pts2 = pts1[:37] + np.array([0.1, 0.2, -0.05])
    for pts in (pts1, pts2):
        E_ref, H_ref = ctx.eval_field(x, pts, -1)
        E, H = ctx.eval_field_noalloc(x, pts, -1)
        print("npts", pts.shape[0], "max |E| diff", (E - E_ref).abs().max().item(), flush=True)
        # the same kernel on the same inputs: identical results
        assert torch.equal(E, E_ref) and torch.equal(H, H_ref)
        assert E.abs().max().item() > 0
    # interior region of body 0, a point inside the guide
    pin = np.array([[1.0, 0.0, 0.0], [0.5, 0.05, 0.02]])
    E_ref, H_ref = ctx.eval_field(x, pin, 0)
    E, H = ctx.eval_field_noalloc(x, pin, 0)
    assert torch.equal(E, E_ref) and torch.equal(H, H_ref)
    too_many = np.zeros((4097, 3)) + np.array([0.0, 1.0, 0.0])
    with pytest.raises(pk.ScabsError) as ei:
        ctx.eval_field_noalloc(x, too_many, -1)
    assert ei.value.code == pk.SCABS_E_ARG
    ctx.close()
