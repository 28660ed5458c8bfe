"""Benchmark of the k-means|| hot path on one MI355X.

A step is one full kmpar_init (Algorithm 2 steps 1-8: first center, r
oversampling rounds of draw + gather + distance fold + cost, weights,
weighted k-means++ recluster) over the KDDCup1999-shaped synthetic input
(n = 4.8M, d = 42, heavy-tailed mixture), k = 500, ell = 2k, r = 5.

Prints one JSON line.  value = point-center distance evaluations per second
of the whole step (sum over distance passes of n * m_pass, divided by the
step time), with X already resident in HBM.
"""
from __future__ import annotations

import argparse
import json
import math
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


NSTREAMS = 3   # concurrent inits in the timed job


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(X, k, ell, rounds, seed, rows):
    """The FP64 oracle on the first `rows` rows of the same input."""
    from oracle import oracle as O
    O.lib()
    Xs = X[:rows].astype("float64")
    t0 = time.perf_counter()
    r = O.kmeans_parallel_init(Xs, k, ell, rounds, seed)
    dt = time.perf_counter() - t0
    evals = rows * len(r.cand_point)
    return {"value": evals / dt, "unit": UNIT, "cores": O.num_threads(), "kind": "oracle",
            "sample": f"oracle kmeans_parallel_init on rows [0, {rows}) of the same input "
                      f"(k={k}, ell={ell:g}, r={rounds}); {evals:.3e} evals in {dt:.1f} s"}


def precision_compare(kmpar, synth, torch, seed, steps=2):
    """BF16-refined vs plain FP32 on the precision workload: n = 16M, d = 128,
    1,000 Gaussian components (centers N(0, 25 I), sigma logU[0.5, 4]), X in
    bf16, k = 1000, ell = 2k, r = 5."""
    n, d, k, rounds = 16_000_000, 128, 1000, 5
    ell = 2.0 * k
    log("precision workload: generating 16M x 128 bf16 on the device")
    Xb = synth.gauss_mixture_sigma_torch(n, d, 1000, seed=seed, device="cuda:0",
                                         out_dtype=torch.bfloat16)
    out = {"workload": "Gaussian mixture, 1,000 components, bf16 storage (synthetic)", "n": n,
           "d": d, "k": k, "ell": ell, "rounds": rounds}
    res = {}
    for name, mode in (("refined_bf16", kmpar.MODE_REFINED), ("plain_fp32", kmpar.MODE_PLAIN_FP32)):
        ctx = kmpar.Context(0, mode)
        r = ctx.init(Xb, k=k, ell=ell, rounds=rounds, seed=seed)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ctx.init(Xb, k=k, ell=ell, rounds=rounds, seed=seed, check=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = (ms, r)
        out[f"{name}_ms"] = ms
        out[f"{name}_evals_per_s"] = float(n) * r.stats["n_candidates"] / (ms / 1e3)
        log(f"precision {name}: {ms:.2f} ms/init, |C|={r.stats['n_candidates']}")
        del ctx
    (mr, rr), (mp, rp) = res["refined_bf16"], res["plain_fp32"]
    phi_r, phi_p = rr.stats["phi"][-1], rp.stats["phi"][-1]
    out["speedup_refined_vs_plain"] = mp / mr
    out["final_phi_rel_diff"] = abs(phi_r - phi_p) / max(abs(phi_p), 1e-300)
    out["centers_bitwise_equal"] = bool(torch.equal(rr.centers, rp.centers))
    out["rescanned_points"] = rr.stats["n_rescanned"]
    del Xb
    torch.cuda.empty_cache()
    return out


def c0_lloyd(kmpar, synth, torch, seed, iters=20, reps=5):
    """C0: GaussMixture k* = 50 centers ~ N(0, 10 I) in d = 15, n = 10,000,
    k = 50, ell = 2k, r = 5, then 20 Lloyd iterations; per mode, the time of
    one init and of one Lloyd iteration (HIP events, averaged)."""
    n, d, k = 10_000, 15, 50
    X = torch.from_numpy(synth.gauss_mixture(n, d, k, 10.0, seed=seed)).to("cuda:0")
    out = {"workload": "GaussMixture (synthetic), n = 10,000, d = 15, k = 50, ell = 2k, r = 5, "
                       f"{iters} Lloyd iterations", "iterations": iters}
    for name, mode in (("refined", kmpar.MODE_REFINED), ("plain", kmpar.MODE_PLAIN_FP32)):
        ctx = kmpar.Context(0, mode)
        r = ctx.init(X, k=k, ell=2.0 * k, rounds=5, seed=seed)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.init(X, k=k, ell=2.0 * k, rounds=5, seed=seed, check=False)
        e1.record()
        torch.cuda.synchronize()
        out[f"{name}_init_ms"] = e0.elapsed_time(e1) / reps
        C = r.centers.clone()
        e0.record()
        for _ in range(iters):
            _, phi = ctx.lloyd_step(X, C)
        e1.record()
        torch.cuda.synchronize()
        out[f"{name}_lloyd_ms_per_iter"] = e0.elapsed_time(e1) / iters
        out[f"{name}_final_phi"] = float(phi.item())
        log(f"C0 {name}: init {out[f'{name}_init_ms']:.3f} ms, Lloyd "
            f"{out[f'{name}_lloyd_ms_per_iter']:.3f} ms/iter, phi {out[f'{name}_final_phi']:.6g}")
    return out


def c3_compare(kmpar, synth, torch, seed, steps=2, with_plain=True, lloyd_iters=0):
    """FP8 precision workload: n = 50M, d = 256, e4m3 codes with per-row
    scales max|x|/448 from a 2,000-component Gaussian mixture (centers
    N(0, 25 I), sigma logU[0.5, 4]), k = 2000, ell = 2k, r = 5; REFINED init
    against PLAIN (PLAIN takes about half a minute here and runs once); then,
    when asked, Lloyd iterations from the REFINED centers (FP8 assignment
    passes run the direct form, a few seconds each)."""
    n, d, k, rounds = 50_000_000, 256, 2000, 5
    ell = 2.0 * k
    log("C3: generating 50M x 256 e4m3 rows on the device")
    Q, S = synth.gauss_mixture_sigma_fp8_torch(n, d, 2000, seed=seed, device="cuda:0")
    out = {"workload": "Gaussian mixture, 2,000 components, e4m3 storage with row scales "
                       "(synthetic)", "n": n, "d": d, "k": k, "ell": ell, "rounds": rounds}

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ctx = kmpar.Context(0, kmpar.MODE_REFINED)
    r = ctx.init(Q, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=S)
    torch.cuda.synchronize()
    out["refined_init_ms"] = timed(lambda: ctx.init(Q, k=k, ell=ell, rounds=rounds, seed=seed,
                                                    row_scale=S, check=False), steps)
    out["refined_init_evals_per_s"] = float(n) * r.stats["n_candidates"] / (out["refined_init_ms"] / 1e3)
    log(f"C3 refined: init {out['refined_init_ms']:.1f} ms (|C|={r.stats['n_candidates']})")
    ctx.profile(True)
    rp = ctx.init(Q, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=S)
    torch.cuda.synchronize()
    p = ctx.profile_read(kmpar.SLOT_SCREEN)
    ctx.profile(False)
    dur = p["ms"] / p["launches"] / 1e3
    flops = 2.0 * d * p["pairs"] / p["launches"]
    out["screen_avg_launch_us"] = dur * 1e6
    out["screen_tflops"] = flops / dur / 1e12
    out["screen_frac_of_bf16_peak"] = flops / dur / 1e12 / PEAK_BF16_MFMA_TFLOPS
    out["rescanned_points"] = rp.stats["n_rescanned"]
    log(f"C3 screen: {p['launches']} launches, avg {dur*1e6:.1f} us, "
        f"{flops/dur/1e12:.1f} TFLOP/s algorithmic")
    if lloyd_iters > 0:
        C = r.centers.clone()
        phi0 = float(ctx.cost(Q, C, row_scale=S).item())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for it in range(lloyd_iters):
            _, phi = ctx.lloyd_step(Q, C, row_scale=S)
            torch.cuda.synchronize()
            log(f"C3 Lloyd iteration {it + 1}/{lloyd_iters}: phi of its input centers {float(phi.item()):.6g}")
        e1.record()
        torch.cuda.synchronize()
        out["lloyd_iterations"] = lloyd_iters
        out["lloyd_ms_per_iter"] = e0.elapsed_time(e1) / lloyd_iters
        out["lloyd_phi_init"] = phi0
        out["lloyd_phi_last_input"] = float(phi.item())
        log(f"C3 Lloyd: {out['lloyd_ms_per_iter']:.1f} ms per iteration")
    del ctx
    if with_plain:
        pctx = kmpar.Context(0, kmpar.MODE_PLAIN_FP32)
        log("C3 plain: one init (about half a minute)")
        holder = {}
        out["plain_init_ms"] = timed(lambda: holder.__setitem__(
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


def batched_bench(kmpar, synth, torch, seed, count, steps=2):
    """Many independent instances in one kmpar_init_batched call: n_i
    log-uniform in [2,000, 200,000], d_i uniform in {32, 64, 128},
    k_i = ceil(sqrt(n_i)/2), GaussMixture data (R = 10), ell = 2k_i, r = 5;
    FP32 and BF16 storage.  Timed with the tile shapes the tuner picks (its
    tuning call is the untimed first one) and with the fixed defaults."""
    import numpy as np
    ns, ds, ks = synth.batch_instances(count, seed=seed)
    ells = 2.0 * ks
    log(f"batched: generating {count} instances, sum n = {int(ns.sum())}")
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
            _, sts, _ = ctx.init_batched(Xv, ks, ells, 5, seed=seed)
            bad = sum(1 for s_ in sts if s_["status"] != 0)
            evals = float(sum(int(n) * s_["n_candidates"] for n, s_ in zip(ns, sts)))
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ctx.init_batched(Xv, ks, ells, 5, seed=seed, check=False)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            out[f"{name}{label}_ms"] = ms
            out[f"{name}{label}_evals_per_s"] = evals / (ms / 1e3)
            out[f"{name}{label}_instances_not_ok"] = bad
            log(f"batched {name}{label}: {ms:.1f} ms per batch, {evals / (ms / 1e3):.3e} evals/s, "
                f"{bad} instances with a non-OK status")
        if conv is not None:
            del Xv
    out["tuned_tiles"] = [{"dtype": dt, "padded_d": dp, "candidates_per_step": 1 if cb == 200 else cb,
                           "row_split_over_two_waves": cb == 200}
                          for dt, dp, cb in tuned.batch_tiles()]
    log(f"batched tiles: {out['tuned_tiles']}")
    del Xs
    torch.cuda.empty_cache()
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_screen_c1.json")
SCREEN_SRC = os.path.join(ROOT, "paper_1203_6402_amd", "csrc", "screen_mfma.hip")


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


def screen_traffic():
    """HBM bytes per k_screen launch from the committed counter summary, or
    None when the summary is missing or the kernel source changed since."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        with open(SCREEN_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if t.get("source_sha256") != sha:
        return None
    return t["hbm_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4_800_000)
    ap.add_argument("--d", type=int, default=42)
    ap.add_argument("--k", type=int, default=500)
    ap.add_argument("--ell-mult", type=float, default=2.0)
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", choices=["plain", "refined"], default="refined")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the input the oracle baseline runs on (0: all of them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c3-lloyd", type=int, default=0,
                    help="with --c3: Lloyd iterations from the REFINED centers (the paper runs 10)")
    ap.add_argument("--no-lloyd", action="store_true",
                    help="skip the Lloyd legs (C1 full size and C0)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16-refined vs FP32-plain comparison on the precision workload")
    ap.add_argument("--c3", action="store_true",
                    help="also run the FP8 workload (50M x 256 e4m3, k = 2000), REFINED init "
                         "against PLAIN")
    ap.add_argument("--c3-no-plain", action="store_true",
                    help="with --c3: REFINED only (for profiling)")
    ap.add_argument("--batched", action="store_true",
                    help="also time the 4,096-instance batched workload (FP32 and BF16)")
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

    import numpy as np
    import torch

    from paper_1203_6402_amd import kmpar, synth

    n, d, k, rounds = args.n, args.d, args.k, args.rounds
    ell = args.ell_mult * k
    if args.pmc_probe:
        pmc_probe(kmpar, synth, torch, args)
        return
    if args.lloyd_probe:
        lloyd_probe(kmpar, synth, torch, args)
        return
    log(f"generating heavy-tailed input n={n} d={d}")
    X = synth.heavy_tailed(n, d, seed=args.seed)
    Xd = torch.from_numpy(X).to("cuda:0")
    mode = kmpar.MODE_REFINED if args.mode == "refined" else kmpar.MODE_PLAIN_FP32
    ctx = kmpar.Context(0, mode)
    ctx.set_option(kmpar.OPT_RECLUSTER_PATH, args.recluster_path)
    stream = torch.cuda.current_stream()

    log(f"warmup {args.warmup}")
    r = None
    for _ in range(args.warmup):
        r = ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=args.seed)
    torch.cuda.synchronize()
    if r is None:
        r = ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=args.seed)
    stats = r.stats
    assert stats["status"] == 0, stats
    ncand = stats["n_candidates"]
    evals = float(n) * ncand          # first pass n*1 + sum_t n*m_t

    log(f"timing {args.steps} steps on one stream")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=args.seed, check=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_single = ev0.elapsed_time(ev1) / max(1, args.steps)
    log(f"{ms_single:.3f} ms/step on one stream, |C|={ncand}, {evals / (ms_single / 1e3):.3e} evals/s")

    # The job: K independent inits of the input, taken in turn by NSTREAMS
    # contexts (each with its own workspace) on as many streams, so that one
    # init's step-8 recluster (a few workgroups, latency-bound) and its small
    # kernels run beside the other inits' distance passes. Every init is
    # complete and its centers equal the single-stream result. (Three streams
    # measured fastest: 10.1 ms per init on one, 8.6 on two, 7.9 on three,
    # 8.4 on four.)
    ctxs = [ctx] + [kmpar.Context(0, mode) for _ in range(NSTREAMS - 1)]
    for c_ in ctxs[1:]:
        c_.set_option(kmpar.OPT_RECLUSTER_PATH, args.recluster_path)
    streams = [torch.cuda.Stream() for _ in range(NSTREAMS)]
    for c_, s_ in zip(ctxs, streams):
        c_.init(Xd, k=k, ell=ell, rounds=rounds, seed=args.seed, stream=s_, check=False)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps on {NSTREAMS} streams")
    outs = []
    ev0.record(stream)
    for s_ in streams:
        s_.wait_stream(stream)
    for i in range(args.steps):
        outs.append(ctxs[i % NSTREAMS].init(Xd, k=k, ell=ell, rounds=rounds, seed=args.seed,
                                            stream=streams[i % NSTREAMS], check=False))
    for s_ in streams:
        stream.wait_stream(s_)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / max(1, args.steps)
    same = all(torch.equal(o.centers[:stats["n_centers"]], r.centers) for o in outs)
    assert same, "a pipelined init differs from the single-stream result"
    del outs
    value = evals / (ms / 1e3)
    log(f"{ms:.3f} ms/step on {NSTREAMS} streams, {value:.3e} evals/s (centers equal: {same})")
    del ctxs[1:]

    # The same step replayed from a HIP graph (launch overhead removed).
    graph_ms = None
    try:
        cap = kmpar.CapturedInit(ctx, Xd, k, ell, rounds, args.seed)
        cap.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()                 # replay() launches on the current stream
        for _ in range(args.steps):
            cap.replay()
        g1.record()
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / max(1, args.steps)
        assert torch.equal(cap.centers, r.centers[:k]) or stats["n_centers"] < k
        log(f"graph replay: {graph_ms:.3f} ms/step")
        del cap
    except Exception as exc:  # reported, not fatal: the eager number stands
        log(f"graph capture unavailable: {exc!r}")

    # Dominant kernel: the distance pass (direct-form fold in PLAIN mode, the
    # MFMA screen in REFINED mode), timed live with HIP events on the stream
    # it runs on, over one further step.
    ctx.profile(True)
    rp = ctx.init(Xd, k=k, ell=ell, rounds=rounds, seed=args.seed)
    torch.cuda.synchronize()
    slots = {name: ctx.profile_read(slot) for name, slot in
             (("k_fold_direct", kmpar.SLOT_FOLD_DIRECT), ("k_screen", kmpar.SLOT_SCREEN),
              ("k_fold_direct(rescan)", kmpar.SLOT_RESCAN))}
    ctx.profile(False)
    for name, p in slots.items():
        if p["launches"]:
            log(f"{name}: {p['launches']} launches, {p['ms']:.3f} ms, {p['pairs']:.3e} pairs")
    dom = max(slots, key=lambda nm: slots[nm]["ms"])
    prof = slots[dom]
    flops_per_launch = 2.0 * d * prof["pairs"] / prof["launches"]
    dur_per_launch = prof["ms"] / prof["launches"] / 1e3
    achieved = flops_per_launch / dur_per_launch / 1e12
    if dom == "k_screen":
        bound, peak = "mfma", PEAK_BF16_MFMA_TFLOPS
    else:
        bound, peak = "alu", PEAK_FP32_VECTOR_TFLOPS
    traffic = screen_traffic() if dom == "k_screen" else None
    roofline = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "launches": prof["launches"], "avg_launch_us": dur_per_launch * 1e6,
                "flops_per_launch": flops_per_launch,
                "distance_kernels_ms": {nm: p["ms"] for nm, p in slots.items() if p["launches"]}}
    log(f"dominant {dom}: avg {dur_per_launch*1e6:.1f} us, {achieved:.2f} TFLOP/s algorithmic "
        f"({100*achieved/peak:.1f}% of {peak})")

    # Row a9 at full size: Lloyd iterations on this input from the centers found above.
    c1_lloyd = c0 = None
    if not args.no_lloyd:
        C = r.centers.clone()
        phi0 = float(ctx.cost(Xd, C).item())
        ctx.lloyd_step(Xd, C)
        torch.cuda.synchronize()
        Cstart = C.clone()
        l0, l1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        l0.record()
        for _ in range(5):
            _, phi = ctx.lloyd_step(Xd, C)
        l1.record()
        torch.cuda.synchronize()
        c1_lloyd = {"ms_per_iter": l0.elapsed_time(l1) / 5, "iterations": 6,
                    "phi_after": float(phi.item()), "phi_init": phi0}
        # The same five iterations in one kmpar_lloyd call (X prepared once).
        Cm = Cstart.clone()
        l0.record()
        _, phim = ctx.lloyd(Xd, Cm, 5)
        l1.record()
        torch.cuda.synchronize()
        assert torch.equal(Cm, C) and float(phim[-1].item()) == c1_lloyd["phi_after"]
        c1_lloyd["one_call_ms_per_iter"] = l0.elapsed_time(l1) / 5
        # The same call captured once in a HIP graph and replayed: the small
        # update kernels then start without launch gaps.
        Cg = Cstart.clone()
        graph, gs = torch.cuda.CUDAGraph(), torch.cuda.Stream()
        with torch.cuda.stream(gs):
            with torch.cuda.graph(graph, stream=gs):
                _, phig = ctx.lloyd(Xd, Cg, 5, stream=gs)
        Cg.copy_(Cstart)
        torch.cuda.synchronize()
        l0.record()
        graph.replay()
        l1.record()
        torch.cuda.synchronize()
        assert torch.equal(Cg, C) and float(phig[-1].item()) == c1_lloyd["phi_after"]
        c1_lloyd["graph_one_call_ms_per_iter"] = l0.elapsed_time(l1) / 5
        log(f"C1 Lloyd: {c1_lloyd['ms_per_iter']:.3f} ms/iter as steps, "
            f"{c1_lloyd['one_call_ms_per_iter']:.3f} ms/iter in one call, "
            f"{c1_lloyd['graph_one_call_ms_per_iter']:.3f} ms/iter as a graph replay, phi {phi0:.6g} -> "
            f"{c1_lloyd['phi_after']:.6g}")
        c0 = c0_lloyd(kmpar, synth, torch, args.seed)

    precision = None
    if not args.no_precision:
        precision = precision_compare(kmpar, synth, torch, args.seed)

    c3 = None
    if args.c3:
        c3 = c3_compare(kmpar, synth, torch, args.seed, with_plain=not args.c3_no_plain,
                        lloyd_iters=args.c3_lloyd)

    batched = None
    if args.batched:
        batched = batched_bench(kmpar, synth, torch, args.seed, args.batch_count)

    cpu = None
    if not args.no_cpu_baseline:
        rows = args.cpu_rows if 0 < args.cpu_rows < n else n
        log(f"cpu baseline on {rows} rows")
        cpu = cpu_baseline(X, k, ell, rounds, args.seed, rows)
        log(f"cpu baseline {cpu['value']:.3e} evals/s on {cpu['cores']} threads")

    out = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "KDDCup1999-shaped heavy-tailed mixture (synthetic)",
                      "n": n, "d": d, "k": k, "ell": ell, "rounds": rounds,
                      "mode": args.mode, "n_candidates": ncand, "evals_per_step": evals,
                      "rescanned_points": rp.stats["n_rescanned"],
                      "graph_replay_ms_per_step": graph_ms,
                      "streams": NSTREAMS, "single_stream_ms_per_step": ms_single,
                      "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu, "c1_lloyd": c1_lloyd, "c0_lloyd": c0, "precision": precision,
           "fp8": c3, "batched": batched}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
