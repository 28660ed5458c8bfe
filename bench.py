"""Benchmark of the k-means|| hot path on one MI355X.

A step is one full kmpar_init (Algorithm 2 steps 1-8: first center, r
oversampling rounds of draw + gather + distance fold + cost, weights,
weighted k-means++ recluster) over the KDDCup1999-shaped synthetic input
(n = 4.8M, d = 42, heavy-tailed mixture), k = 500, ell = 2k, r = 5, timed on
one stream.

Prints one JSON line.  value = point-center distance evaluations per second
of one step (sum over distance passes of n * m_pass, divided by the device
time of one kmpar_init on one stream), with X already resident in HBM.  The
other workloads run as legs of the same job, each with its own roofline entry
for its dominant kernel: the GaussMixture Lloyd run (n = 10,000), the BF16
precision workload (16M x 128), the FP8 workload with ten Lloyd iterations
(50M x 256) and the 4,096-instance batch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-means|| init pt·ctr evals/s + %roofline; BF16-refined vs FP32 at Δφ≤1e-4"
UNIT = "pt·ctr evals/s"
# MI355X published peaks.
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

NSTREAMS = 3   # concurrent inits of the extra three-stream measurement
LEGS = ("c1", "c1lloyd", "sweep", "c0", "quality", "largec", "c2", "c3", "c4")

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_screen_c1.json")
SCREEN_SRCS = [os.path.join(ROOT, "paper_1203_6402_amd", "csrc", f)
               for f in ("screen_mfma.hip", "geometry.hpp")]


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed_ms(torch, fn, reps):
    """Average device time of `reps` calls of fn on the current stream."""
    e0, e1 = events(torch)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / max(1, reps)


def roofline_entry(kernel, flops_per_launch, us_per_launch, bound, launches, traffic=None,
                   profile=None):
    peak = PEAK_BF16_MFMA_TFLOPS if bound == "mfma" else PEAK_FP32_VECTOR_TFLOPS
    achieved = flops_per_launch / (us_per_launch * 1e-6) / 1e12
    e = {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
         "frac": achieved / peak, "traffic": traffic, "launches": launches,
         "avg_launch_us": us_per_launch, "flops_per_launch": flops_per_launch}
    if profile:
        e["profile"] = profile
    return e


def screen_roofline(kmpar, ctx, d, profile=None, traffic=None):
    """Roofline entry of the REFINED screen from the library's event timing
    of the launches since profiling was enabled (2 d flop per point-center
    pair; its matrix instructions are bf16)."""
    p = ctx.profile_read(kmpar.SLOT_SCREEN)
    us = p["ms"] / p["launches"] * 1e3
    flops = 2.0 * d * p["pairs"] / p["launches"]
    return roofline_entry("k_screen", flops, us, "mfma", p["launches"], traffic, profile)


def screen_traffic():
    """HBM bytes per C1 screen launch from the committed counter summary, or
    None when the summary is missing or the kernel sources (the screen and
    its launch geometry) changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        h = hashlib.sha256()
        for src in SCREEN_SRCS:
            with open(src, "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    if t.get("source_sha256") != h.hexdigest():
        return None
    return t["hbm_bytes_per_launch"]


# ----------------------------------------------------------------------- C1
def c1_leg(kmpar, synth, torch, args, X):
    """The headline: one kmpar_init on one stream (REFINED by default)."""
    n, d, k, rounds, seed = X.shape[0], X.shape[1], args.k, args.rounds, args.seed
    ell = args.ell_mult * k
    Xd = torch.from_numpy(X).to("cuda:0")
    mode = kmpar.MODE_REFINED if args.mode == "refined" else kmpar.MODE_PLAIN_FP32
    ctx = kmpar.Context(0, mode)
    ctx.set_option(kmpar.OPT_RECLUSTER_PATH, args.recluster_path)
    stream = torch.cuda.current_stream()
    log(f"C1: warmup {args.warmup}")
    r = None
    for _ in range(max(1, args.warmup)):
        r = ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=seed)
    torch.cuda.synchronize()
    stats = r.stats
    ncand = stats["n_candidates"]
    evals = float(n) * ncand          # first pass n*1 + sum_t n*m_t
    log(f"C1: timing {args.steps} steps on one stream")
    outs = []
    e0, e1 = events(torch)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        outs.append(ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=seed, check=False))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(1, args.steps)
    for o in outs:          # every timed init finished with status OK and the same centers
        st = kmpar.parse_stats(o.stats["_raw"], rounds)
        kmpar.check_status(st["status"], False, "timed C1 init")
        assert torch.equal(o.centers, r.centers)
    del outs
    log(f"C1: {ms:.3f} ms/step, |C|={ncand}, {evals / (ms / 1e3):.3e} evals/s")
    out = {"ms": ms, "evals": evals, "stats": stats, "r": r, "ctx": ctx, "Xd": Xd}

    # Extra: NSTREAMS contexts on as many streams take the same steps in
    # turn, so one init's step-8 recluster (a few workgroups) and small
    # kernels run beside the others' distance passes.
    ctxs = [ctx] + [kmpar.Context(0, mode) for _ in range(NSTREAMS - 1)]
    streams = [torch.cuda.Stream() for _ in range(NSTREAMS)]
    for c_, s_ in zip(ctxs, streams):
        c_.set_option(kmpar.OPT_RECLUSTER_PATH, args.recluster_path)
        c_.init(Xd, k=k, ell=ell, rounds=rounds, seed=seed, stream=s_, check=False)
    torch.cuda.synchronize()
    outs = []
    e0.record(stream)
    for s_ in streams:
        s_.wait_stream(stream)
    for i in range(args.steps):
        outs.append(ctxs[i % NSTREAMS].init(Xd, k=k, ell=ell, rounds=rounds, seed=seed,
                                            stream=streams[i % NSTREAMS], check=False))
    for s_ in streams:
        stream.wait_stream(s_)
    e1.record(stream)
    torch.cuda.synchronize()
    ms3 = e0.elapsed_time(e1) / max(1, args.steps)
    for o in outs:
        st = kmpar.parse_stats(o.stats["_raw"], rounds)
        kmpar.check_status(st["status"], False, "three-stream C1 init")
        assert torch.equal(o.centers, r.centers), "a concurrent init differs from the one-stream result"
    del outs, ctxs[1:]
    out["three_streams"] = {"streams": NSTREAMS, "ms_per_init": ms3, "evals_per_s": evals / (ms3 / 1e3)}
    log(f"C1: {ms3:.3f} ms per init with {NSTREAMS} inits in flight")

    # The same step replayed from a HIP graph.
    cap = kmpar.CapturedInit(ctx, Xd, k, ell, rounds, seed)
    cap.replay()
    torch.cuda.synchronize()
    out["graph_replay_ms"] = timed_ms(torch, cap.replay, args.steps)
    assert torch.equal(cap.centers, r.centers)
    kmpar.check_status(cap.stats()["status"], False, "graph replay")
    del cap
    log(f"C1: graph replay {out['graph_replay_ms']:.3f} ms/step")

    # Dominant kernel, timed live with HIP events on its own stream over one
    # further step.
    ctx.profile(True)
    rp = ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=seed)
    torch.cuda.synchronize()
    slots = {name: ctx.profile_read(slot) for name, slot in
             (("k_fold_direct", kmpar.SLOT_FOLD_DIRECT), ("k_screen", kmpar.SLOT_SCREEN),
              ("k_rescan", kmpar.SLOT_RESCAN))}
    ctx.profile(False)
    dom = max(slots, key=lambda nm: slots[nm]["ms"])
    p = slots[dom]
    flops = 2.0 * d * p["pairs"] / p["launches"]
    us = p["ms"] / p["launches"] * 1e3
    out["roofline"] = roofline_entry(
        dom, flops, us, "mfma" if dom == "k_screen" else "alu", p["launches"],
        screen_traffic() if dom == "k_screen" else None,
        "profiles/screen_c1_refined_kernel_stats.md" if dom == "k_screen" else
        "profiles/fold_direct_c1_plain_kernel_trace.md")
    out["roofline"]["distance_kernels_ms"] = {nm: q["ms"] for nm, q in slots.items() if q["launches"]}
    out["rescanned_points"] = rp.stats["n_rescanned"]
    log(f"C1: dominant {dom} avg {us:.1f} us, {out['roofline']['achieved']:.1f} TFLOP/s "
        f"({100 * out['roofline']['frac']:.1f}% of {out['roofline']['peak']})")

    # ell = k/2 on the same input, one stream.
    ell_h = 0.5 * k
    rh = ctx.init(Xd, k=k, ell=ell_h, rounds=rounds, seed=seed)
    torch.cuda.synchronize()
    msh = timed_ms(torch, lambda: ctx.init(Xd, k=k, ell=ell_h, rounds=rounds, seed=seed,
                                           check=False), args.steps)
    out["ell_half_k"] = {"ell": ell_h, "ms_per_init": msh, "n_candidates": rh.stats["n_candidates"],
                         "evals_per_s": float(n) * rh.stats["n_candidates"] / (msh / 1e3),
                         "flagged_draws": rh.stats["flagged_draws"],
                         "flagged_picks": rh.stats["flagged_picks"],
                         "flagged_argmins": rh.stats["flagged_argmins"]}
    log(f"C1 ell=k/2: {msh:.3f} ms/init, |C|={rh.stats['n_candidates']}")

    # The baseline the paper measures k-means|| against (Section 4.2):
    # k-means++ on all of X, k passes over the data, on the same GPU.
    kctx = kmpar.Context(0)
    kctx.kmeanspp(Xd, k, seed=seed)
    torch.cuda.synchronize()
    holder = {}
    mspp = timed_ms(torch, lambda: holder.__setitem__("r", kctx.kmeanspp(Xd, k, seed=seed,
                                                                         check=False)), 2)
    out["kmeanspp"] = {"ms": mspp, "passes_over_X": k, "speedup_of_kmeans_par": mspp / ms,
                       "GBps_X_read": float(n) * d * 4 * k / (mspp / 1e3) / 1e9}
    log(f"C1 k-means++ (all of X): {mspp:.1f} ms, {mspp / ms:.1f}x the k-means|| init")
    return out


def c1_lloyd_leg(kmpar, torch, c1, iters=5):
    """Row a9 at full size: Lloyd iterations on the C1 input from the init's
    centers, as lloyd_step calls, as one kmpar_lloyd call and as its graph."""
    ctx, Xd, r = c1["ctx"], c1["Xd"], c1["r"]
    C = r.centers.clone()
    phi0 = float(ctx.cost(Xd, C).item())
    ctx.lloyd_step(Xd, C)
    torch.cuda.synchronize()
    Cstart = C.clone()
    holder = {}

    def steps():
        for _ in range(iters):
            _, holder["phi"] = ctx.lloyd_step(Xd, C)
    out = {"iterations": iters + 1, "phi_init": phi0,
           "ms_per_iter": timed_ms(torch, steps, 1) / iters}
    out["phi_after"] = float(holder["phi"].item())
    Cm = Cstart.clone()
    ms = timed_ms(torch, lambda: holder.__setitem__("m", ctx.lloyd(Xd, Cm, iters)), 1)
    assert torch.equal(Cm, C) and float(holder["m"][1][-1].item()) == out["phi_after"]
    out["one_call_ms_per_iter"] = ms / iters
    Cg = Cstart.clone()
    graph, gs = torch.cuda.CUDAGraph(), torch.cuda.Stream()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            _, phig = ctx.lloyd(Xd, Cg, iters, stream=gs)
    Cg.copy_(Cstart)
    torch.cuda.synchronize()
    out["graph_one_call_ms_per_iter"] = timed_ms(torch, graph.replay, 1) / iters
    assert torch.equal(Cg, C) and float(phig[-1].item()) == out["phi_after"]
    log(f"C1 Lloyd: {out['ms_per_iter']:.3f} ms/iter as steps, {out['one_call_ms_per_iter']:.3f} "
        f"in one call, {out['graph_one_call_ms_per_iter']:.3f} as a graph")
    return out


# ----------------------------------------------------------------------- C0
def sweep_leg(kmpar, torch, X, ms=(1, 2, 4, 8, 16, 32, 64), reps=5):
    """The distance pass where HBM bounds it: kmpar_assign (PLAIN) of the C1
    rows (n = 4.8M, d = 42 FP32) against m = 1 .. 64 centers.  Per m, the
    fold's event-timed duration, its rate in bytes -- n (4 d + 8) per launch:
    the rows read once, the assignment and D^2 written -- against the 8 TB/s
    HBM peak, and its FLOP rate (2 d n m) beside it."""
    ctx = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
    n, d = X.shape
    rows = []
    for m in ms:
        C = X[:: max(1, n // m)][:m].clone()
        ctx.assign(X, C)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.assign(X, C)
        torch.cuda.synchronize()
        p = ctx.profile_read(kmpar.SLOT_FOLD_DIRECT)
        ctx.profile(False)
        us = p["ms"] / p["launches"] * 1e3
        gbs = n * (4 * d + 8) / (us * 1e-6) / 1e9
        rows.append({"m": m, "us_per_launch": us, "GB_per_s": gbs, "frac_hbm": gbs / PEAK_HBM_GBS,
                     "tflops": 2.0 * d * n * m / (us * 1e-6) / 1e12})
        log(f"sweep m={m}: {us:.1f} us, {gbs:.0f} GB/s ({100 * gbs / PEAK_HBM_GBS:.1f}% of HBM)")
    return {"workload": f"kmpar_assign PLAIN, C1 rows n = {n}, d = {d} FP32, m centers",
            "bytes_per_launch": f"n (4 d + 8) = {n * (4 * d + 8)}", "sweep": rows}


def c0_leg(kmpar, synth, torch, seed, iters=20, reps=5):
    """GaussMixture k* = 50 centers ~ N(0, 10 I) in d = 15, n = 10,000,
    k = 50, ell = 2k, r = 5, then 20 Lloyd iterations; per mode, the time of
    one init and of one Lloyd iteration (these calls are launch-bound)."""
    n, d, k = 10_000, 15, 50
    Xh = synth.gauss_mixture(n, d, k, 10.0, seed=seed)
    X = torch.from_numpy(Xh).to("cuda:0")
    out = {"workload": "GaussMixture (synthetic), n = 10,000, d = 15, k = 50, ell = 2k, r = 5, "
                       f"{iters} Lloyd iterations", "iterations": iters}
    for name, mode in (("refined", kmpar.MODE_REFINED), ("plain", kmpar.MODE_PLAIN_FP32)):
        ctx = kmpar.Context(0, mode)
        r = ctx.init(X, k=k, ell=2.0 * k, rounds=5, seed=seed, trace=True)
        torch.cuda.synchronize()
        out[f"{name}_init_ms"] = timed_ms(torch, lambda: ctx.init(X, k=k, ell=2.0 * k, rounds=5,
                                                                  seed=seed, check=False), reps)
        C = r.centers.clone()
        holder = {}

        def lloyd():
            for _ in range(iters):
                _, holder["phi"] = ctx.lloyd_step(X, C)
        out[f"{name}_lloyd_ms_per_iter"] = timed_ms(torch, lloyd, 1) / iters
        out[f"{name}_final_phi"] = float(holder["phi"].item())
        if name == "refined":
            out["_trace"] = (Xh, r, seed)
        log(f"C0 {name}: init {out[f'{name}_init_ms']:.3f} ms, Lloyd "
            f"{out[f'{name}_lloyd_ms_per_iter']:.3f} ms/iter, phi {out[f'{name}_final_phi']:.6g}")
    return out


# ------------------------------------------------------------------ quality
def gauss_runs(kmpar, torch, X, k, method, ell, rounds, seeds, max_iters=500):
    """Per seed: the seed cost (after the initialisation) and the final cost
    and number of Lloyd updates after Lloyd's iteration until stable, on the
    GPU.  method: "kmeanspp" (Algorithm 1 on all of X) or "par" (k-means||,
    independent draws, ell and rounds as given) or "exact" (exactly ell per
    round)."""
    out = []
    ctx = kmpar.Context(0, kmpar.MODE_REFINED)
    if method == "exact":
        ctx.set_option(kmpar.OPT_SAMPLING, kmpar.SAMPLING_EXACT)
    lctx = kmpar.Context(0, kmpar.MODE_REFINED)
    for s in seeds:
        if method == "kmeanspp":
            C, _, _, st = ctx.kmeanspp(X, k, seed=s)
        else:
            C = ctx.init(X, k=k, ell=float(ell), rounds=rounds, seed=s, allow_toofew=True).centers
        C = C.contiguous().clone()
        seed_cost = float(lctx.cost(X, C).item())
        it, _, phi = lctx.lloyd_until_stable(X, C, max_iters)
        out.append({"seed": s, "centers": int(C.shape[0]), "seed_cost": seed_cost,
                    "final_cost": float(phi[-1].item()), "lloyd_updates": it})
    return out


def quality_leg(kmpar, synth, torch, seeds=range(11)):
    """Quality on GaussMixture (n = 10,000, d = 15, k = 50; Section 4.1) by
    the paper's protocols, every run on the GPU: the Table 1 protocol (median
    seed and final cost over 11 runs, R in {1, 10, 100}, k-means++ and
    k-means|| with ell = k/2 and 2k, r = 5), the Figure 5.2 protocol (median
    final cost against the number of rounds, ell in {k/10, k/2, k, 2k}, R =
    10) and the Table 6 protocol (mean Lloyd updates to convergence, k in
    {20, 50, 100}, R = 10, 10 runs)."""
    import numpy as np
    n, d, k = 10_000, 15, 50
    med = lambda runs, key: float(np.median([r[key] for r in runs]))
    t1 = {}
    for R in (1.0, 10.0, 100.0):
        X = torch.from_numpy(synth.gauss_mixture(n, d, k, R, seed=0)).to("cuda:0")
        row = {}
        for name, method, ell in (("kmeans++", "kmeanspp", 0), ("kmeans|| l=k/2 r=5", "par", k // 2),
                                  ("kmeans|| l=2k r=5", "par", 2 * k)):
            runs = gauss_runs(kmpar, torch, X, k, method, ell, 5, seeds)
            row[name] = {"seed_median_1e4": med(runs, "seed_cost") / 1e4,
                         "final_median_1e4": med(runs, "final_cost") / 1e4,
                         "lloyd_updates_mean": float(np.mean([r["lloyd_updates"] for r in runs]))}
        t1[f"R={R:g}"] = row
        log(f"quality Table 1 R={R:g}: " + ", ".join(
            f"{m} {v['seed_median_1e4']:.1f}/{v['final_median_1e4']:.1f}" for m, v in row.items()))
    X = torch.from_numpy(synth.gauss_mixture(n, d, k, 10.0, seed=0)).to("cuda:0")
    f52 = {"kmeans++ final_median_1e4": med(gauss_runs(kmpar, torch, X, k, "kmeanspp", 0, 0, seeds),
                                             "final_cost") / 1e4}
    for ell in (k // 10, k // 2, k, 2 * k):
        f52[f"l={ell}"] = {str(r): med(gauss_runs(kmpar, torch, X, k, "par", ell, r, seeds),
                                       "final_cost") / 1e4 for r in (1, 2, 3, 5, 8, 12)}
    log(f"quality Figure 5.2: {f52}")
    t6 = {}
    for kk in (20, 50, 100):
        Xk = torch.from_numpy(synth.gauss_mixture(n, d, kk, 10.0, seed=1)).to("cuda:0")
        t6[f"k={kk}"] = {
            name: float(np.mean([r["lloyd_updates"] for r in
                                 gauss_runs(kmpar, torch, Xk, kk, method, ell, 5, range(10))]))
            for name, method, ell in (("kmeans++", "kmeanspp", 0),
                                      ("kmeans|| l=k/2 r=5", "par", kk // 2),
                                      ("kmeans|| l=2k r=5", "par", 2 * kk))}
    log(f"quality Table 6: {t6}")
    return {"workload": "GaussMixture n = 10,000, d = 15 (synthetic), medians over 11 seeds",
            "table1": t1, "figure5_2_final_median_1e4": f52, "table6_lloyd_updates_mean": t6}


# ------------------------------------------------------------ large C
def largec_leg(kmpar, synth, torch, seed):
    """The candidate-sharded assignment of Section 3.5 on a large center set
    and few points (KDDCup1999-shaped rows, n = 20,000, d = 42): against
    m = 16,384 centers (kmpar_assign's limit) one slice per point block and
    the sharded form, and against m = 1,000,000 centers sharded."""
    n, d = 20_000, 42
    X = torch.from_numpy(synth.heavy_tailed(n, d, seed=seed)).to("cuda:0")
    ctx = kmpar.Context(0)
    out = {"workload": f"KDDCup1999-shaped rows (synthetic), n = {n}, d = {d}"}
    for m, shards_list in ((16_384, (1, 8, 64)), (1_000_000, (64, 256))):
        C = torch.from_numpy(synth.heavy_tailed(m, d, seed=seed + 1)).to("cuda:0")
        ref = None
        for sh in shards_list:
            a, _, _ = ctx.assign_sharded(X, C, sh)
            torch.cuda.synchronize()
            if ref is None:
                ref = a
            assert torch.equal(a, ref)
            ms = timed_ms(torch, lambda: ctx.assign_sharded(X, C, sh), 3)
            e = 2.0 * d * n * m / (ms / 1e3) / 1e12
            out[f"m={m} shards={sh}"] = {"ms": ms, "tflops": e, "frac_fp32": e / PEAK_FP32_VECTOR_TFLOPS}
            log(f"large C: m={m} shards={sh}: {ms:.2f} ms, {e:.1f} TFLOP/s")
        if m <= 16_384:
            a0, _ = ctx.assign(X, C)
            torch.cuda.synchronize()
            assert torch.equal(a0, ref)
            out[f"m={m} kmpar_assign_ms"] = timed_ms(torch, lambda: ctx.assign(X, C), 3)
    return out


# ----------------------------------------------------------------------- C2
def c2_leg(kmpar, synth, torch, seed, steps=2):
    """BF16-refined vs plain FP32 on the precision workload: n = 16M, d = 128,
    1,000 Gaussian components (centers N(0, 25 I), sigma logU[0.5, 4]), X in
    bf16, k = 1000, ell = 2k, r = 5."""
    n, d, k, rounds = 16_000_000, 128, 1000, 5
    ell = 2.0 * k
    log("C2: generating 16M x 128 bf16 on the device")
    Xb = synth.gauss_mixture_sigma_torch(n, d, 1000, seed=seed, device="cuda:0",
                                         out_dtype=torch.bfloat16)
    out = {"workload": "Gaussian mixture, 1,000 components, bf16 storage (synthetic)", "n": n,
           "d": d, "k": k, "ell": ell, "rounds": rounds}
    res = {}
    for name, mode in (("refined_bf16", kmpar.MODE_REFINED), ("plain_fp32", kmpar.MODE_PLAIN_FP32)):
        ctx = kmpar.Context(0, mode)
        r = ctx.init(Xb, k=k, ell=ell, rounds=rounds, seed=seed)
        torch.cuda.synchronize()
        ms = timed_ms(torch, lambda: ctx.init(Xb, k=k, ell=ell, rounds=rounds, seed=seed,
                                              check=False), steps)
        res[name] = (ms, r)
        out[f"{name}_ms"] = ms
        out[f"{name}_evals_per_s"] = float(n) * r.stats["n_candidates"] / (ms / 1e3)
        log(f"C2 {name}: {ms:.2f} ms/init, |C|={r.stats['n_candidates']}")
        if mode == kmpar.MODE_REFINED:
            ctx.profile(True)
            rp = ctx.init(Xb, k=k, ell=ell, rounds=rounds, seed=seed)
            torch.cuda.synchronize()
            out["roofline"] = screen_roofline(kmpar, ctx, d, "profiles/screen_c2_bf16_kernel_stats.md")
            ctx.profile(False)
            out["flagged_draws"] = rp.stats["flagged_draws"]
            out["flagged_picks"] = rp.stats["flagged_picks"]
            out["flagged_argmins"] = rp.stats["flagged_argmins"]
            log(f"C2 screen: {out['roofline']['achieved']:.1f} TFLOP/s "
                f"({100 * out['roofline']['frac']:.1f}% of the bf16 peak)")
        del ctx
    (mr, rr), (mp, rp_) = res["refined_bf16"], res["plain_fp32"]
    phi_r, phi_p = rr.stats["phi"][-1], rp_.stats["phi"][-1]
    out["speedup_refined_vs_plain"] = mp / mr
    out["final_phi_rel_diff"] = abs(phi_r - phi_p) / max(abs(phi_p), 1e-300)
    out["centers_bitwise_equal"] = bool(torch.equal(rr.centers, rp_.centers))
    out["rescanned_points"] = rr.stats["n_rescanned"]
    del Xb
    torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------------- C3
def c3_leg(kmpar, synth, torch, seed, steps=2, with_plain=True, lloyd_iters=10):
    """FP8 workload: n = 50M, d = 256, e4m3 codes with per-row scales
    max|x|/448 from a 2,000-component Gaussian mixture (centers N(0, 25 I),
    sigma logU[0.5, 4]), k = 2000, ell = 2k, r = 5; REFINED init against
    PLAIN, then `lloyd_iters` Lloyd iterations with FP32 centroid sums from
    the REFINED centers in one kmpar_lloyd call (FP8 assignment passes run
    the direct form)."""
    n, d, k, rounds = 50_000_000, 256, 2000, 5
    ell = 2.0 * k
    log("C3: generating 50M x 256 e4m3 rows on the device")
    Q, S = synth.gauss_mixture_sigma_fp8_torch(n, d, 2000, seed=seed, device="cuda:0")
    out = {"workload": "Gaussian mixture, 2,000 components, e4m3 storage with row scales "
                       "(synthetic)", "n": n, "d": d, "k": k, "ell": ell, "rounds": rounds}
    ctx = kmpar.Context(0, kmpar.MODE_REFINED)
    r = ctx.init(Q, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=S)
    torch.cuda.synchronize()
    out["refined_init_ms"] = timed_ms(torch, lambda: ctx.init(Q, k=k, ell=ell, rounds=rounds,
                                                              seed=seed, row_scale=S, check=False),
                                      steps)
    out["n_candidates"] = r.stats["n_candidates"]
    out["refined_init_evals_per_s"] = float(n) * r.stats["n_candidates"] / (out["refined_init_ms"] / 1e3)
    log(f"C3 refined: init {out['refined_init_ms']:.1f} ms (|C|={r.stats['n_candidates']})")
    ctx.profile(True)
    rp = ctx.init(Q, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=S)
    torch.cuda.synchronize()
    out["roofline"] = screen_roofline(kmpar, ctx, d, "profiles/screen_c3_fp8_kernel_stats.md")
    ctx.profile(False)
    out["rescanned_points"] = rp.stats["n_rescanned"]
    out["flagged_draws"] = rp.stats["flagged_draws"]
    out["flagged_picks"] = rp.stats["flagged_picks"]
    out["flagged_argmins"] = rp.stats["flagged_argmins"]
    log(f"C3 screen: {out['roofline']['achieved']:.1f} TFLOP/s "
        f"({100 * out['roofline']['frac']:.1f}% of the bf16 peak)")
    if lloyd_iters > 0:
        C = r.centers.clone()
        holder = {}
        ms = timed_ms(torch, lambda: holder.__setitem__(
            "l", ctx.lloyd(Q, C, lloyd_iters, row_scale=S)), 1)
        phis = holder["l"][1].cpu().tolist()
        assert all(phis[i + 1] <= phis[i] * (1 + 1e-6) for i in range(len(phis) - 1))
        evals = float(n) * k
        out["lloyd"] = {"iterations": lloyd_iters, "ms_per_iter": ms / lloyd_iters,
                        "evals_per_s": evals / (ms / lloyd_iters / 1e3),
                        "phi_first_input": phis[0], "phi_last_input": phis[-1],
                        "assign_tflops": 2.0 * d * evals / (ms / lloyd_iters / 1e3) / 1e12}
        log(f"C3 Lloyd: {out['lloyd']['ms_per_iter']:.1f} ms per iteration, phi {phis[0]:.6g} -> "
            f"{phis[-1]:.6g}")
    del ctx
    if with_plain:
        pctx = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
        log("C3 plain: one init (about ten seconds)")
        holder = {}
        out["plain_init_ms"] = timed_ms(torch, lambda: holder.__setitem__(
            "r", pctx.init(Q, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=S)), 1)
        rpl = holder["r"]
        log(f"C3 plain: init {out['plain_init_ms']:.1f} ms")
        out["init_speedup"] = out["plain_init_ms"] / out["refined_init_ms"]
        out["init_centers_bitwise_equal"] = bool(torch.equal(r.centers, rpl.centers))
        out["init_phi_rel_diff"] = abs(r.stats["phi"][-1] - rpl.stats["phi"][-1]) / max(
            abs(rpl.stats["phi"][-1]), 1e-300)
        del pctx
    del Q, S
    torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------------- C4
def c4_leg(kmpar, synth, torch, seed, count, steps=2):
    """Many independent instances in one kmpar_init_batched call: n_i
    log-uniform in [2,000, 200,000], d_i uniform in {32, 64, 128},
    k_i = ceil(sqrt(n_i)/2), GaussMixture data (R = 10), ell = 2k_i, r = 5;
    FP32 and BF16 storage.  Timed with the tile shapes the tuner picks (its
    tuning call is the untimed first one) and with the fixed defaults; the
    grouped folds are timed live for the roofline entry."""
    ns, ds, ks = synth.batch_instances(count, seed=seed)
    ells = 2.0 * ks
    log(f"C4: generating {count} instances, sum n = {int(ns.sum())}")
    Xs = synth.batch_gauss_mixture_torch(ns, ds, ks, seed=seed, device="cuda:0")
    out = {"workload": f"{count} independent GaussMixture instances (synthetic)",
           "instances": count, "sum_n": int(ns.sum()), "mean_d": float(ds.mean()),
           "k_range": [int(ks.min()), int(ks.max())], "rounds": 5}
    tuned = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
    fixed = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
    fixed.set_option(kmpar.OPT_BATCH_AUTOTUNE, 0)
    for name, conv in (("fp32", None), ("bf16", torch.bfloat16)):
        Xv = Xs if conv is None else [X.to(conv) for X in Xs]
        for label, ctx in (("", tuned), ("_fixed", fixed)):
            _, sts, _ = ctx.init_batched(Xv, ks, ells, 5, seed=seed)    # raises on a non-OK status
            evals = float(sum(int(n) * s_["n_candidates"] for n, s_ in zip(ns, sts)))
            flops = float(sum(2.0 * int(d) * int(n) * s_["n_candidates"]
                              for n, d, s_ in zip(ns, ds, sts)))
            torch.cuda.synchronize()
            ms = timed_ms(torch, lambda: ctx.init_batched(Xv, ks, ells, 5, seed=seed, check=False),
                          steps)
            out[f"{name}{label}_ms"] = ms
            out[f"{name}{label}_evals_per_s"] = evals / (ms / 1e3)
            if label == "":
                out[f"{name}_flagged_draws"] = int(sum(s_["flagged_draws"] for s_ in sts))
                out[f"{name}_flagged_picks"] = int(sum(s_["flagged_picks"] for s_ in sts))
                ctx.profile(True)
                ctx.init_batched(Xv, ks, ells, 5, seed=seed)
                torch.cuda.synchronize()
                p = ctx.profile_read(kmpar.SLOT_BATCH_FOLD)
                ctx.profile(False)
                # every grouped fold launch of the batch (first pass and
                # rounds, all row-length groups): their summed algorithmic
                # flops over their summed duration
                e = roofline_entry("kb_fold* (grouped direct-form folds)", flops / p["launches"],
                                   p["ms"] / p["launches"] * 1e3, "alu", p["launches"], None,
                                   "profiles/batched_c4_kernel_stats.md")
                e["fold_ms_per_batch"] = p["ms"]
                out[f"{name}_roofline"] = e
                log(f"C4 {name}: folds {p['ms']:.1f} ms of {ms:.1f} ms, "
                    f"{e['achieved']:.1f} TFLOP/s ({100 * e['frac']:.1f}% of FP32 peak)")
            log(f"C4 {name}{label}: {ms:.1f} ms per batch, {evals / (ms / 1e3):.3e} evals/s")
        if conv is not None:
            del Xv
    out["roofline"] = out["fp32_roofline"]
    out["tuned_tiles"] = [{"dtype": dt, "padded_d": dp, "candidates_per_step": 1 if cb == 200 else cb,
                           "row_split_over_two_waves": cb == 200}
                          for dt, dp, cb in tuned.batch_tiles()]
    del Xs
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------- CPU oracle
def cpu_baseline_leg(X, k, ell, rounds, seed, rows, c0):
    """The FP64 oracle (test infrastructure, run only here): timed on the
    first `rows` rows of the C1 input, and the replay of the GPU's C0 init,
    whose flagged decisions are reported (a bad one fails the benchmark)."""
    from oracle import oracle as O
    O.lib()
    Xs = X[:rows].astype("float64")
    t0 = time.perf_counter()
    r = O.kmeans_parallel_init(Xs, k, ell, rounds, seed)
    dt = time.perf_counter() - t0
    evals = rows * len(r.cand_point)
    base = {"value": evals / dt, "unit": UNIT, "cores": O.num_threads(), "kind": "oracle",
            "sample": f"oracle kmeans_parallel_init on rows [0, {rows}) of the C1 input "
                      f"(k={k}, ell={ell:g}, r={rounds}); {evals:.3e} evals in {dt:.1f} s"}
    replay = None
    if c0 is not None:
        import numpy as np
        Xh, g, c0_seed = c0
        tr = {key: v.cpu().numpy() for key, v in g.trace.items()}
        st = g.stats
        rs, start = [], 1
        for c in st["round_count"][1:]:
            rs.append(tr["cand_point"][start:start + c])
            start += c
        o = O.kmeans_parallel_init(Xh.astype("float64"), 50, 100.0, 5, c0_seed,
                                   follow={"rounds": rs, "assign": tr["assign"],
                                           "picks": tr["center_cand"]})
        assert sum(o.bad.values()) == 0, o.bad
        assert np.array_equal(o.cand_point, tr["cand_point"]) and np.array_equal(o.picks, tr["center_cand"])
        replay = {"workload": "GaussMixture n = 10,000, d = 15, k = 50, ell = 2k, r = 5 (REFINED)",
                  "oracle_flagged": o.flags, "oracle_bad": o.bad,
                  "gpu_flagged_draws": st["flagged_draws"], "gpu_flagged_picks": st["flagged_picks"],
                  "gpu_flagged_argmins": st["flagged_argmins"],
                  "phi_rel_diff": abs(st["phi"][-1] - o.phi[-1]) / o.phi[-1]}
    return base, replay


def pmc_probe(kmpar, synth, torch, args):
    """Counter-collection workload: a plain 1 GiB device copy of known size
    (calibrates FETCH_SIZE / WRITE_SIZE), then one REFINED step."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    X = synth.heavy_tailed(args.n, args.d, seed=args.seed)
    Xd = torch.from_numpy(X).to("cuda:0")
    ctx = kmpar.Context(0, kmpar.MODE_REFINED)
    ctx.init(Xd, k=args.k, ell=args.ell_mult * args.k, rounds=args.rounds, seed=args.seed)
    torch.cuda.synchronize()
    log("pmc probe done")


def lloyd_probe(kmpar, synth, torch, args, iters=4):
    """Profiling workload for row a9 at full size: one REFINED init on the
    C1 input, then `iters` Lloyd steps from its centers (`iters` lloyd_step
    calls, or with --lloyd-one-call one kmpar_lloyd call)."""
    X = synth.heavy_tailed(args.n, args.d, seed=args.seed)
    Xd = torch.from_numpy(X).to("cuda:0")
    ctx = kmpar.Context(0, kmpar.MODE_REFINED)
    r = ctx.init(Xd, k=args.k, ell=args.ell_mult * args.k, rounds=args.rounds, seed=args.seed)
    C = r.centers.clone()
    torch.cuda.synchronize()
    if args.lloyd_one_call:
        _, phis = ctx.lloyd(Xd, C, iters)
        phi = phis[-1]
    else:
        for _ in range(iters):
            _, phi = ctx.lloyd_step(Xd, C)
    torch.cuda.synchronize()
    log(f"lloyd probe done: {iters} steps, phi {float(phi.item()):.6g}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4_800_000)
    ap.add_argument("--d", type=int, default=42)
    ap.add_argument("--k", type=int, default=500)
    ap.add_argument("--ell-mult", type=float, default=2.0)
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=["plain", "refined"], default="refined")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma list of legs to run: " + ", ".join(LEGS) + " (c1 always runs "
                         "when c1lloyd or the CPU baseline does)")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the C1 input the oracle baseline runs on (0: all of them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c3-lloyd", type=int, default=10,
                    help="Lloyd iterations of the FP8 leg (the workload's 10)")
    ap.add_argument("--c3-no-plain", action="store_true", help="FP8 leg: REFINED only (profiling)")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--recluster-path", type=int, default=0, choices=[0, 1, 2])
    ap.add_argument("--lloyd-probe", action="store_true",
                    help="profiling workload: one REFINED init then 4 Lloyd steps on the C1 input")
    ap.add_argument("--lloyd-one-call", action="store_true",
                    help="with --lloyd-probe: the 4 iterations as one kmpar_lloyd call")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run only a 1 GiB copy (counter calibration) and one step, for rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); a row-sharded "
              "multi-GPU path is not part of this library.", file=sys.stderr)
        sys.exit(2)
    legs = {x.strip() for x in args.legs.split(",") if x.strip()}
    unknown = legs - set(LEGS)
    if unknown:
        ap.error(f"unknown legs {sorted(unknown)}")

    import torch

    from paper_1203_6402_amd import kmpar, synth

    if args.pmc_probe:
        pmc_probe(kmpar, synth, torch, args)
        return
    if args.lloyd_probe:
        lloyd_probe(kmpar, synth, torch, args)
        return
    n, d, k, rounds = args.n, args.d, args.k, args.rounds
    ell = args.ell_mult * k
    need_c1 = "c1" in legs or "c1lloyd" in legs or not args.no_cpu_baseline
    X = c1 = None
    if need_c1:
        log(f"C1: generating heavy-tailed input n={n} d={d}")
        X = synth.heavy_tailed(n, d, seed=args.seed)
        c1 = c1_leg(kmpar, synth, torch, args, X)
    c1_lloyd = c1_lloyd_leg(kmpar, torch, c1) if "c1lloyd" in legs else None
    sweep = sweep_leg(kmpar, torch, c1["Xd"]) if "sweep" in legs and c1 is not None else None
    c0 = c0_leg(kmpar, synth, torch, args.seed) if "c0" in legs else None
    quality = quality_leg(kmpar, synth, torch) if "quality" in legs else None
    largec = largec_leg(kmpar, synth, torch, args.seed) if "largec" in legs else None
    c0_trace = c0.pop("_trace") if c0 else None
    if c1 is not None:
        del c1["Xd"], c1["ctx"], c1["r"]
        torch.cuda.empty_cache()
    c2 = c2_leg(kmpar, synth, torch, args.seed) if "c2" in legs else None
    c3 = c3_leg(kmpar, synth, torch, args.seed, with_plain=not args.c3_no_plain,
                lloyd_iters=args.c3_lloyd) if "c3" in legs else None
    c4 = c4_leg(kmpar, synth, torch, args.seed, args.batch_count) if "c4" in legs else None

    cpu = replay = None
    if not args.no_cpu_baseline:
        rows = args.cpu_rows if 0 < args.cpu_rows < n else n
        log(f"cpu baseline on {rows} rows, and the oracle replay of the C0 init")
        cpu, replay = cpu_baseline_leg(X, k, ell, rounds, args.seed, rows, c0_trace)
        log(f"cpu baseline {cpu['value']:.3e} evals/s on {cpu['cores']} threads")

    out = {"metric": METRIC, "value": None, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    if c1 is not None:
        st = c1["stats"]
        out.update({"value": c1["evals"] / (c1["ms"] / 1e3), "ms_per_step": c1["ms"]})
        out["config"] = {"workload": "KDDCup1999-shaped heavy-tailed mixture (synthetic), one "
                                     "kmpar_init on one stream",
                         "n": n, "d": d, "k": k, "ell": ell, "rounds": rounds, "mode": args.mode,
                         "n_candidates": st["n_candidates"], "evals_per_step": c1["evals"],
                         "rescanned_points": c1["rescanned_points"],
                         "flagged_draws": st["flagged_draws"], "flagged_picks": st["flagged_picks"],
                         "flagged_argmins": st["flagged_argmins"],
                         "graph_replay_ms_per_step": c1["graph_replay_ms"],
                         "three_streams": c1["three_streams"], "ell_half_k": c1["ell_half_k"],
                         "kmeanspp_same_input": c1["kmeanspp"],
                         "parallelism": "single GPU"}
        out["roofline"] = c1["roofline"]
    out["cpu_baseline"] = cpu
    out["oracle_replay_c0"] = replay
    out["c1_lloyd"] = c1_lloyd
    out["few_centers_sweep"] = sweep
    out["c0_lloyd"] = c0
    out["quality"] = quality
    out["large_candidate_set"] = largec
    out["precision"] = c2
    out["fp8"] = c3
    out["batched"] = c4
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
