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


def test_batched_graph_replays_match_eager(K):
    # A batch of independent instances in one fixed launch sequence, captured once:
    # every replay must give the eager batch's centers and stats.
    ns, ds, ks = synth.batch_instances(40, seed=6, n_lo=500, n_hi=8000)
    Xs = [torch.from_numpy(X).to("cuda:0") for X in synth.batch_gauss_mixture(ns, ds, ks, seed=6)]
    ells = 2.0 * ks
    ctx = K.Context(0, K.MODE_PLAIN_FP32)
    ec, es, _ = ctx.init_batched(Xs, ks, ells, 4, seed=5)
    cap = K.CapturedBatch(ctx, Xs, ks, ells, 4, 5)
    Y = torch.from_numpy(synth.gauss_mixture(20000, 15, 30, 10.0, seed=2)).to("cuda:0")
    for rep in range(3):
        cap.batch.centers.zero_()
        cap.replay()
        torch.cuda.synchronize()
        cs, st = cap.results()
        for i in range(len(Xs)):
            assert torch.equal(cs[i], ec[i]), (rep, i)
            assert st[i] == es[i], (rep, i)
        # eager work on the same context (its own workspace) between replays
        ctx.init(Y, k=30, ell=60.0, rounds=3, seed=rep)
        torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["plain", "refined"])
def test_lloyd_graph_replays_match_eager(K, mode):
    # kmpar_lloyd (three iterations) captured once: every replay from the same
    # starting centers gives the eager centers, last assignment and costs,
    # with eager library work on another context between replays.
    m = K.MODE_REFINED if mode == "refined" else K.MODE_PLAIN_FP32
    X = torch.from_numpy(synth.heavy_tailed(40000, 42, seed=17)).to("cuda:0")
    Y = torch.from_numpy(synth.gauss_mixture(20000, 15, 30, 10.0, seed=2)).to("cuda:0")
    ctx = K.Context(0, m)
    C0 = X[torch.arange(0, 40000, 400, device="cuda:0")].clone()   # 100 centers
    Ce = C0.clone()
    ae, pe = ctx.lloyd(X, Ce, 3, want_assign=True)
    torch.cuda.synchronize()
    C = C0.clone()
    graph, s = torch.cuda.CUDAGraph(), torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            a, p = ctx.lloyd(X, C, 3, want_assign=True, stream=s)
    other = K.Context(0, m)
    Cy = torch.from_numpy(synth.gauss_mixture(30, 15, 30, 10.0, seed=3)).to("cuda:0")
    for rep in range(4):
        C.copy_(C0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, Ce), rep
        assert torch.equal(a, ae), rep
        assert torch.equal(p, pe), rep
        other.lloyd_step(Y, Cy)
        torch.cuda.synchronize()
