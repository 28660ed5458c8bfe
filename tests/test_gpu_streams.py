"""Independent kmpar_init calls in flight on several streams at once (one
context and workspace per stream): one call's step-8 recluster runs
beside the other's distance passes, and every call gives the result it gives
alone on one stream."""
import pytest
import torch

from paper_1203_6402_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,nstr", [("refined", 2), ("refined", 3), ("plain", 3)])
def test_streams_interleaved_equal_single_stream(mode, nstr):
    from paper_1203_6402_amd import kmpar
    m = kmpar.MODE_REFINED if mode == "refined" else kmpar.MODE_PLAIN_FP32
    X = torch.from_numpy(synth.heavy_tailed(200000, 42, seed=3)).to("cuda:0")
    Y = torch.from_numpy(synth.gauss_mixture(150000, 24, 60, 10.0, seed=4)).to("cuda:0")
    args = {"X": (X, dict(k=100, ell=200.0, rounds=5, seed=1)),
            "Y": (Y, dict(k=60, ell=120.0, rounds=4, seed=2))}
    alone = kmpar.Context(0, m)
    ref = {name: alone.init(D, **kw) for name, (D, kw) in args.items()}
    torch.cuda.synchronize()
    ctxs = [kmpar.Context(0, m) for _ in range(nstr)]
    strs = [torch.cuda.Stream() for _ in range(nstr)]
    cur = torch.cuda.current_stream()
    for s in strs:
        s.wait_stream(cur)
    outs = []
    for i in range(6):
        name = "X" if i % 2 == 0 else "Y"
        D, kw = args[name]
        outs.append((name, ctxs[i % nstr].init(D, stream=strs[i % nstr], check=False, **kw)))
    for s in strs:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    for name, o in outs:
        st = kmpar.parse_stats(o.stats["_raw"], args[name][1]["rounds"])
        assert st["status"] == 0, (name, st["status"])
        assert st["n_centers"] == ref[name].stats["n_centers"]
        assert torch.equal(o.centers[:st["n_centers"]], ref[name].centers), name


@pytest.mark.parametrize("mode", ["refined", "plain"])
def test_lloyd_streams_beside_init(mode):
    # kmpar_lloyd on two streams (one context and workspace each) while a
    # kmpar_init runs on a third: every Lloyd call gives its one-stream
    # centers, costs and assignment.
    from paper_1203_6402_amd import kmpar
    m = kmpar.MODE_REFINED if mode == "refined" else kmpar.MODE_PLAIN_FP32
    X = torch.from_numpy(synth.heavy_tailed(200000, 42, seed=3)).to("cuda:0")
    Y = torch.from_numpy(synth.gauss_mixture(150000, 24, 60, 10.0, seed=4)).to("cuda:0")
    CX = X[torch.arange(0, 200000, 2000, device="cuda:0")].clone()
    CY = Y[torch.arange(0, 150000, 2500, device="cuda:0")].clone()
    alone = kmpar.Context(0, m)
    ref = {}
    for name, D, C0 in (("X", X, CX), ("Y", Y, CY)):
        C = C0.clone()
        a, p = alone.lloyd(D, C, 4, want_assign=True)
        ref[name] = (C, a, p)
    rinit = alone.init(X, k=100, ell=200.0, rounds=5, seed=1)
    torch.cuda.synchronize()
    ctxs = [kmpar.Context(0, m) for _ in range(3)]
    strs = [torch.cuda.Stream() for _ in range(3)]
    Cs = {"X": CX.clone(), "Y": CY.clone()}
    cur = torch.cuda.current_stream()
    for s in strs:
        s.wait_stream(cur)
    oi = ctxs[2].init(X, k=100, ell=200.0, rounds=5, seed=1, stream=strs[2], check=False)
    ax, px = ctxs[0].lloyd(X, Cs["X"], 4, want_assign=True, stream=strs[0])
    ay, py = ctxs[1].lloyd(Y, Cs["Y"], 4, want_assign=True, stream=strs[1])
    for s in strs:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    for name, a, p in (("X", ax, px), ("Y", ay, py)):
        C, ra, rp = ref[name]
        assert torch.equal(Cs[name], C), name
        assert torch.equal(a, ra), name
        assert torch.equal(p, rp), name
    assert torch.equal(oi.centers, rinit.centers)


def test_outputs_prepared_on_the_call_stream():
    # With the current stream kept busy, calls on side streams must not have
    # their outputs zeroed by work queued behind the current stream's: every
    # init's stats record holds its own figures once all streams are done.
    # Four side streams, so that some run on another hardware queue than the
    # current stream (a binding that zeroed the stats on the current stream
    # left n_centers = 0 on one of the four).
    from paper_1203_6402_amd import kmpar
    X = torch.from_numpy(synth.gauss_mixture(50000, 16, 40, 10.0, seed=8)).to("cuda:0")
    ctxs = [kmpar.Context(0, kmpar.MODE_REFINED) for _ in range(4)]
    ref = ctxs[0].init(X, k=40, ell=80.0, rounds=4, seed=6)
    torch.cuda.synchronize()
    a = torch.rand(2048, 2048, device="cuda:0") / 2048.0
    b = torch.empty_like(a)
    sides = [torch.cuda.Stream() for _ in range(4)]
    cur = torch.cuda.current_stream()
    for s in sides:
        s.wait_stream(cur)
    for _ in range(40):          # keeps the current stream busy for several ms
        torch.mm(a, a, out=b)
    rs = [c.init(X, k=40, ell=80.0, rounds=4, seed=6, stream=s, check=False)
          for c, s in zip(ctxs, sides)]
    for s in sides:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    for r in rs:
        st = kmpar.parse_stats(r.stats["_raw"], 4)
        assert st["status"] == 0 and st["n_centers"] == ref.stats["n_centers"]
        assert torch.equal(r.centers[:st["n_centers"]], ref.centers)
