"""Quality by the Table 1 protocol on GaussMixture (Section 5.1; n = 10,000,
d = 15, k = 50, R = 10, 11 seeds): the GPU's median seed and final costs
(k-means++, k-means|| with ell = k/2 and 2k, r = 5, then Lloyd until stable)
against the FP64 oracle run with the same seeds, and against the paper's
medians in scale (a different data draw and generator)."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1203_6402_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_gaussmixture.json")


@pytest.fixture(scope="module")
def K():
    from paper_1203_6402_amd import kmpar
    assert torch.cuda.is_available()
    return kmpar


@pytest.mark.parametrize("method,ell,golden_key", [("kmeanspp", 0, "kmeans_pp"),
                                                    ("par", 25, "kmeans_par_ell_half_k"),
                                                    ("par", 100, "kmeans_par_ell_2k")])
def test_table1_protocol_r10(K, method, ell, golden_key):
    n, d, k = 10_000, 15, 50
    X = synth.gauss_mixture(n, d, k, 10.0, seed=0)
    X64 = X.astype(np.float64)
    Xd = torch.from_numpy(X).to("cuda:0")
    ctx = K.Context(0, K.MODE_REFINED)
    gpu_seed, gpu_final, orc_seed, orc_final = [], [], [], []
    for s in range(11):
        if method == "kmeanspp":
            C, _, _, _ = ctx.kmeanspp(Xd, k, seed=s)
            p, _, _, _ = O.kmeanspp(X64, k, s)
            Co = X64[p]
        else:
            C = ctx.init(Xd, k=k, ell=float(ell), rounds=5, seed=s).centers
            Co = O.kmeans_parallel_init(X64, k, ell, 5, s).centers
        C = C.contiguous().clone()
        gpu_seed.append(float(ctx.cost(Xd, C).item()))
        it, _, phi = ctx.lloyd_until_stable(Xd, C, 500)
        gpu_final.append(float(phi[-1].item()))
        orc_seed.append(O.cost(X64, Co))
        _, oit, ophi, _, _ = O.lloyd_until_stable(X64, Co, 500)
        orc_final.append(ophi[-1])
    gs, gf = np.median(gpu_seed), np.median(gpu_final)
    assert gs == pytest.approx(np.median(orc_seed), rel=1e-4)
    assert gf == pytest.approx(np.median(orc_final), rel=1e-3)
    agree = sum(abs(a - b) <= 1e-4 * b for a, b in zip(gpu_final, orc_final))
    assert agree >= 9, (gpu_final, orc_final)
    g = json.load(open(GOLDEN))[golden_key]["R=10"]
    assert 0.5 * g["seed"] <= gs / 1e4 <= 2.0 * g["seed"]
    assert 0.5 * g["final"] <= gf / 1e4 <= 2.0 * g["final"]
    assert gf <= gs
