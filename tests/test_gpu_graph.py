"""Graph-captured iterations: em_iterate on a created stream captures one EM
iteration into a HIP graph and replays it.  Every replay is checked against
eager execution of the same job on the default stream, with host
synchronisation and eager work between the replays."""
import numpy as np
import pytest

from paper_2302_05804_amd import synth
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name,sr", [("FP32", 1), ("BF16_SPLIT", 1), ("FP32", 2)])
def test_graph_replays_match_eager(prec_name, sr):
    import torch

    from paper_2302_05804_amd import em
    prec = getattr(em, prec_name)
    p = synth.make_problem("c2" if sr == 1 else "c4", H=192, W=160, n=3, seed=31)
    prob = em.Problem.make(3, 192 // sr, 160 // sr, 43, sr=sr, precision=prec)
    x0 = synth.positive_start(p.latent_shape, 20.0, seed=32)
    xe = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    xg = torch.empty_like(xe)
    eager = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), xe, x0=to_dev(x0))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        graphed = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), xg, x0=to_dev(x0),
                             stream=side)
    for k in range(5):
        eager.iterate(1)
        graphed.iterate(1)
        torch.cuda.synchronize()
        assert torch.equal(xe, xg), f"replay {k}"
        _ = (xe * 2).sum().item()          # unrelated eager work between replays
    tre = eager.iterate(3, trace=True)
    trg = graphed.iterate(3, trace=True)
    torch.cuda.synchronize()
    assert np.array_equal(tre, trg)
    assert torch.equal(xe, xg)
    eager.close()
    graphed.close()
