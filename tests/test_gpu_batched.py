"""Batched k-means|| (many independent instances in grouped launches): each
instance is replayed by the FP64 oracle with its own Philox instance index."""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from paper_1203_6402_amd import synth
from tests.gpu_util import compare_init, decoded_fp64, to_bf16_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1203_6402_amd import kmpar
    assert torch.cuda.is_available()
    return kmpar.Context(0, kmpar.MODE_PLAIN_FP32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _replay_all(Xs64, cs, sts, trs, ks, ells, rounds, seed):
    for i, X64 in enumerate(Xs64):
        st = sts[i]
        assert st["status"] == 0, (i, st)
        tr = {key: v.cpu().numpy() for key, v in trs[i].items()}
        r = SimpleNamespace(stats=st, centers=cs[i])
        compare_init(X64, r, tr, int(ks[i]), float(ells[i]), rounds, seed, inst=i, argmins=False)
        assert tr["cand_weight"].sum() == X64.shape[0]


def test_batched_f32_matches_oracle_per_instance(ctx):
    ns, ds, ks = synth.batch_instances(48, seed=3, n_lo=500, n_hi=20000)
    Xs = synth.batch_gauss_mixture(ns, ds, ks, seed=3)
    ells = 2.0 * ks
    cs, sts, trs = ctx.init_batched([_dev(X) for X in Xs], ks, ells, 5, seed=11, trace=True)
    torch.cuda.synchronize()
    _replay_all([X.astype(np.float64) for X in Xs], cs, sts, trs, ks, ells, 5, 11)


def test_batched_c4_draw_sample_matches_oracle(ctx):
    # The batching workload itself: 4,096 instances with n log-uniform in
    # [2,000, 200,000], d in {32, 64, 128}, k = ceil(sqrt(n)/2), ell = 2k,
    # r = 5, GaussMixture data (R = 10), made on the device exactly as the
    # benchmark makes them and run as one batch; 64 instances drawn at random
    # are replayed by the oracle with their own Philox instance index.
    ns, ds, ks = synth.batch_instances(4096, seed=0)
    ells = 2.0 * ks
    Xs = synth.batch_gauss_mixture_torch(ns, ds, ks, seed=0, device="cuda:0")
    cs, sts, trs = ctx.init_batched(Xs, ks, ells, 5, seed=0, trace=True)
    torch.cuda.synchronize()
    assert all(s_["status"] == 0 for s_ in sts)
    pick = np.sort(np.random.default_rng(7).choice(4096, 64, replace=False))
    print(f"C4: replaying instances with n = {int(ns[pick].min())} .. {int(ns[pick].max())}",
          flush=True)
    for i in pick:
        tr = {key: v.cpu().numpy() for key, v in trs[i].items()}
        r = SimpleNamespace(stats=sts[i], centers=cs[i])
        compare_init(Xs[i].cpu().numpy().astype(np.float64), r, tr, int(ks[i]), float(ells[i]), 5, 0,
                     inst=int(i), argmins=False)


def test_batched_bf16_and_ragged_dims(ctx):
    ns = np.array([300, 4097, 999, 1, 2600])
    ds = np.array([128, 42, 7, 5, 256])
    ks = np.array([12, 30, 9, 1, 25])
    Xb = [to_bf16_bits(X) for X in synth.batch_gauss_mixture(ns, ds, np.maximum(ks, 2), seed=5)]
    ells = np.array([24.0, 60.0, 18.0, 3.0, 50.0])
    cs, sts, trs = ctx.init_batched([_dev(X).view(torch.bfloat16) for X in Xb], ks, ells, 4,
                                    seed=2, trace=True)
    torch.cuda.synchronize()
    _replay_all([decoded_fp64(X, "bf16") for X in Xb], cs, sts, trs, ks, ells, 4, 2)


def test_batch_of_one_equals_single_instance(ctx):
    X = synth.heavy_tailed(30011, 42, seed=4)
    Xd = _dev(X)
    single = ctx.init(Xd, k=60, ell=120.0, rounds=5, seed=9, trace=True)
    cs, sts, trs = ctx.init_batched([Xd], [60], [120.0], 5, seed=9, trace=True)
    torch.cuda.synchronize()
    for key in ("cand_point", "cand_weight", "assign", "d2"):
        assert torch.equal(single.trace[key], trs[0][key]), key
    assert sts[0]["round_count"] == single.stats["round_count"]
    assert sts[0]["phi"] == single.stats["phi"]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_row_split_fold_equals_single_instance(ctx, dtype):
    # Rows of 65 to 128 padded elements are folded with each row split over
    # two waves (the first 64 elements, then the rest from the partial sum).
    # For every padded length of that range, a batch of one (Philox instance
    # 0, as a single call uses) equals the single-instance init bit for bit.
    for j, d in enumerate((65, 72, 90, 100, 113, 127)):
        X = _dev(synth.gauss_mixture(4000 + 997 * j, d, 12, 10.0, seed=30 + j))
        if dtype == "bf16":
            X = X.to(torch.bfloat16)
        k = 12 + 3 * j
        single = ctx.init(X, k=k, ell=2.0 * k, rounds=4, seed=17, trace=True)
        cs, sts, trs = ctx.init_batched([X], [k], [2.0 * k], 4, seed=17, trace=True)
        torch.cuda.synchronize()
        for key in ("cand_point", "cand_weight", "assign", "d2"):
            assert torch.equal(single.trace[key], trs[0][key]), (d, key)
        assert torch.equal(single.centers, cs[0]), d
        assert sts[0]["phi"] == single.stats["phi"], d


def _same_batches(a, b):
    (ca, sa, ta), (cb, sb, tb) = a, b
    for i in range(len(ca)):
        assert torch.equal(ca[i], cb[i]), i
        for key in ta[i]:
            assert torch.equal(ta[i][key], tb[i][key]), (i, key)
        x, y = dict(sa[i]), dict(sb[i])
        x.pop("n_rescanned")
        y.pop("n_rescanned")
        assert x == y, i


@pytest.mark.skip(reason="the batched MFMA screen is switched off: its 4,096-instance run "
                         "stopped with an illegal-address fault whose cause was not found; "
                         "batched instances run the direct form in every mode")
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batched_refined_equals_plain(ctx, dtype):
    # REFINED batches screen the instances that qualify (ell >= 32, supported
    # width) on the matrix cores, with their undecided points recomputed by
    # the screen's own waves; every output must equal the direct form's.
    from paper_1203_6402_amd import kmpar
    ns = np.array([4000, 9001, 2500, 700, 12000, 3333, 1800, 6000])
    ds = np.array([32, 64, 128, 42, 170 if dtype == "f32" else 256, 7, 96, 33])
    ks = np.array([30, 45, 25, 12, 50, 20, 18, 40])
    ells = np.array([60.0, 90.0, 50.0, 24.0, 100.0, 40.0, 36.0, 80.0])  # one below 32: direct form
    Xs = synth.batch_gauss_mixture(ns, ds, ks, seed=8)
    if dtype == "bf16":
        Xs = [to_bf16_bits(X) for X in Xs]
        devs = [_dev(X).view(torch.bfloat16) for X in Xs]
    else:
        devs = [_dev(X) for X in Xs]
    refined = kmpar.Context(0, kmpar.MODE_REFINED)
    a = ctx.init_batched(devs, ks, ells, 4, seed=13, trace=True)
    b = refined.init_batched(devs, ks, ells, 4, seed=13, trace=True)
    torch.cuda.synchronize()
    _same_batches(a, b)
    # the screened instances resolve most points on the matrix cores
    for i in range(len(ns)):
        assert b[1][i]["n_rescanned"] <= 0.1 * ns[i] * 4, (i, b[1][i]["n_rescanned"])
    # and the refined run replays against the oracle like the plain one
    X64 = [decoded_fp64(X, dtype) if dtype == "bf16" else X.astype(np.float64) for X in Xs]
    _replay_all(X64[:3], b[0][:3], b[1][:3], b[2][:3], ks[:3], ells[:3], 4, 13)


def test_batched_autotune_keeps_results():
    # The tuner times every candidates-per-step variant of each group's fold
    # on round 1 (re-applying a fold changes nothing): a tuned context, a
    # context that has tuned already and an untuned one give the same batch.
    from paper_1203_6402_amd import kmpar
    ns, ds, ks = synth.batch_instances(24, seed=9, n_lo=500, n_hi=12000, dims=(32, 60, 128, 160))
    Xs = synth.batch_gauss_mixture(ns, ds, ks, seed=9)
    devs = [_dev(X) for X in Xs]
    ells = 2.0 * ks
    fixed = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
    fixed.set_option(kmpar.OPT_BATCH_AUTOTUNE, 0)
    tuned = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
    a = fixed.init_batched(devs, ks, ells, 4, seed=21, trace=True)
    b = tuned.init_batched(devs, ks, ells, 4, seed=21, trace=True)   # tunes on round 1
    c = tuned.init_batched(devs, ks, ells, 4, seed=21, trace=True)   # uses the tuned shapes
    torch.cuda.synchronize()
    _same_batches(a, b)
    _same_batches(a, c)
    assert fixed.batch_tiles() == []
    tiles = tuned.batch_tiles()
    dps = sorted({kmpar_dp(int(d)) for d in ds})
    assert sorted(t[1] for t in tiles) == dps
    for dt, dp, cb in tiles:
        # candidates per step (whole rows up to 128 elements, halves beyond);
        # 200: each row split over two waves (65 to 128 elements)
        if dp > 128:
            assert cb in (4, 8)
        else:
            assert cb in ((1, 2, 4, 200) if dp > 64 else (1, 2, 4))


def kmpar_dp(d):
    # padded row length of the candidate rows (multiples of 4 / 16 / 32)
    if d <= 64:
        return (d + 3) // 4 * 4
    if d <= 128:
        return (d + 15) // 16 * 16
    return (d + 31) // 32 * 32
