"""kmpar_init captured in a HIP graph: no host synchronisation, memset or
allocation happens inside the call, so the whole Algorithm 2 pipeline
replays from the graph.  Every replay -- with eager library work between
replays -- must match the eager result bit for bit."""
import numpy as np
import pytest
import torch

from paper_1203_6402_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_1203_6402_amd import kmpar
    assert torch.cuda.is_available()
    return kmpar


@pytest.mark.parametrize("mode", ["plain", "refined"])
def test_graph_replays_match_eager(K, mode):
    m = K.MODE_REFINED if mode == "refined" else K.MODE_PLAIN_FP32
    X = torch.from_numpy(synth.heavy_tailed(50000, 42, seed=13)).to("cuda:0")
    Y = torch.from_numpy(synth.gauss_mixture(20000, 15, 30, 10.0, seed=2)).to("cuda:0")
    ctx = K.Context(0, m)
    eager = ctx.init(X, k=80, ell=160.0, rounds=5, seed=3)
    torch.cuda.synchronize()
    cap = K.CapturedInit(ctx, X, 80, 160.0, 5, 3)
    other = K.Context(0, m)
    for rep in range(4):
        cap.centers.zero_()
        cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(cap.centers, eager.centers), rep
        st = cap.stats()
        assert st["phi"] == eager.stats["phi"] and st["round_count"] == eager.stats["round_count"]
        # eager work on another context and input between replays
        other.init(Y, k=30, ell=60.0, rounds=3, seed=rep)
        torch.cuda.synchronize()
