"""Host-side tests of the C ABI (no GPU): the library loads, exports every
function include/kmpar.h declares, validates arguments before any HIP call,
and sizes workspaces."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kmpar.h")


@pytest.fixture(scope="module")
def K():
    from paper_1203_6402_amd import kmpar
    return kmpar


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_exports(K):
    declared = _declared_functions()
    assert "kmpar_init" in declared and "lloyd_step" in declared
    lib = ctypes.CDLL(K.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in kmpar.h but not exported"
    assert sorted(K.EXPORTED) == declared


def test_stats_layout(K):
    assert K._lib.kmpar_sizeof_stats() == ctypes.sizeof(K.Stats)
    assert ctypes.sizeof(K.Stats) % 8 == 0


def test_strerror(K):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert K._lib.kmpar_strerror(code).decode() != "unknown status"
    assert K._lib.kmpar_strerror(-99).decode() == "unknown status"


def test_max_candidates(K):
    # capacity min(n, L + 12 isqrt(L) + 76), L = ceil(ell): >= ell + 12 sqrt(ell) + 64
    assert K.max_candidates(10**6, 1000.0, 5) == 1 + 5 * (1000 + 12 * math.isqrt(1000) + 76)
    assert K.max_candidates(10**6, 999.5, 1) == 1 + (1000 + 12 * math.isqrt(1000) + 76)
    for ell in (1.0, 7.3, 250.0, 4000.0):
        assert K.max_candidates(10**9, ell, 1) - 1 >= ell + 12 * math.sqrt(ell) + 64
    assert K.max_candidates(50, 1e12, 1) == 51              # capped at n per round
    assert K.max_candidates(50, 3.0, 0) == 1
    with pytest.raises(K.KmparError):
        K.max_candidates(10, float("nan"), 1)
    with pytest.raises(K.KmparError):
        K.max_candidates(10, 2.0, K.MAX_ROUNDS + 1)


def test_host_only_context_and_workspace(K):
    ctx = K.Context(None)
    b_init = ctx.workspace_size(K.OP_INIT, 4_800_000, 42, 500, 1000.0, 5)
    assert b_init > 4_800_000 * 8                            # D2 + assignment at least
    assert ctx.workspace_size(K.OP_LLOYD, 10000, 15, 50) > ctx.workspace_size(K.OP_ASSIGN, 10000, 15, 50)
    for bad in [dict(n=0), dict(d=0), dict(d=257), dict(k=0), dict(k=20000), dict(n=2**31)]:
        args = dict(n=1000, d=8, k=10)
        args.update(bad)
        with pytest.raises(K.KmparError) as e:
            ctx.workspace_size(K.OP_ASSIGN, args["n"], args["d"], args["k"])
        assert e.value.status == K.E_INVAL
    with pytest.raises(K.KmparError):
        ctx.workspace_size(K.OP_INIT, 100, 8, 101, 10.0, 5)    # k > n
    with pytest.raises(K.KmparError):
        ctx.workspace_size(K.OP_INIT, 100, 8, 10, -1.0, 5)     # ell <= 0


def _call_init(K, ctx, **kw):
    a = dict(X=16, rs=None, dt=K.F32, n=100, d=8, k=10, ell=20.0, rounds=5, seed=0,
             centers=4096, ws=8192, wsb=1 << 30, stats=None, trace=None)
    a.update(kw)
    return K._lib.kmpar_init(ctx._h, a["X"], a["rs"], a["dt"], a["n"], a["d"], a["k"], a["ell"],
                             a["rounds"], a["seed"], a["centers"], a["ws"], a["wsb"], a["stats"],
                             a["trace"], None)


def test_init_validation_before_any_device_work(K):
    # Pointers here are never dereferenced: validation rejects first, and a
    # context without a device refuses to launch.
    ctx = K.Context(None)
    assert _call_init(K, ctx) == K.E_NODEVICE
    cases = [dict(X=None), dict(X=17), dict(n=0), dict(d=0), dict(d=300), dict(k=0), dict(k=101),
             dict(ell=0.0), dict(ell=float("inf")), dict(rounds=-1), dict(rounds=65),
             dict(centers=None), dict(centers=4100), dict(ws=None), dict(dt=7),
             dict(rs=32), dict(dt=K.FP8_E4M3), dict(stats=4097)]
    for c in cases:
        assert _call_init(K, ctx, **c) == K.E_INVAL, c
    assert _call_init(K, ctx, wsb=100) == K.E_WORKSPACE


def test_assign_cost_lloyd_validation(K):
    ctx = K.Context(None)
    L = K._lib
    h = ctx._h
    assert L.kmpar_cost(h, 16, None, K.F32, 100, 8, 32, 5, 64, 8192, 1 << 30, None) == K.E_NODEVICE
    assert L.kmpar_cost(h, 16, None, K.F32, 100, 8, 32, 0, 64, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_cost(h, 16, None, K.F32, 100, 8, 32, 5, None, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_cost(h, 16, None, K.F32, 100, 8, 32, 5, 64, 8192, 10, None) == K.E_WORKSPACE
    assert L.kmpar_assign(h, 16, None, K.F32, 100, 8, 32, 5, None, None, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_assign(h, 16, None, K.F32, 100, 8, 32, 5, 48, 52, 8192, 1 << 30, None) == K.E_INVAL
    assert L.lloyd_step(h, 16, None, K.F32, 100, 8, 32, 101, None, None, 8192, 1 << 30, None) == K.E_INVAL
    assert L.lloyd_step(h, 16, None, K.F32, 100, 8, 32, 5, None, 12, 8192, 1 << 30, None) == K.E_INVAL
    assert L.lloyd_step(h, 16, None, K.F32, 100, 8, 32, 5, None, None, 8192, 1 << 30, None) == K.E_NODEVICE
    assert L.kmpar_lloyd(h, 16, None, K.F32, 100, 8, 32, 5, -1, None, None, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_lloyd(h, 16, None, K.F32, 100, 8, 32, 101, 3, None, None, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_lloyd(h, 16, None, K.F32, 100, 8, 32, 5, 3, 20, None, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_lloyd(h, 16, None, K.F32, 100, 8, 32, 5, 3, None, 12, 8192, 1 << 30, None) == K.E_INVAL
    assert L.kmpar_lloyd(h, 16, None, K.F32, 100, 8, 32, 5, 3, None, None, 8192, 10, None) == K.E_WORKSPACE
    assert L.kmpar_lloyd(h, 16, None, K.F32, 100, 8, 32, 5, 3, None, None, 8192, 1 << 30, None) == K.E_NODEVICE
    assert L.kmpar_last_error(h).decode() != ""


def test_batched_validation(K):
    import numpy as np
    ctx = K.Context(None)
    desc = np.zeros(3, dtype=K.INSTANCE_DTYPE)
    for i in range(3):
        desc[i]["X"], desc[i]["centers"] = 4096 * (i + 1), 8192 * (i + 1)
        desc[i]["n"], desc[i]["d"], desc[i]["k"], desc[i]["ell"], desc[i]["rounds"] = 1000, 32, 10, 20.0, 5
    out = ctypes.c_size_t(0)
    L = K._lib
    assert L.kmpar_workspace_size_batched(ctx._h, desc.ctypes.data, 3, K.F32, ctypes.byref(out)) == 0
    assert out.value > 3 * 1000 * 8
    assert L.kmpar_init_batched(ctx._h, desc.ctypes.data, 4096, 3, K.F32, 0, 64, out.value, None, None) == K.E_NODEVICE
    assert L.kmpar_init_batched(ctx._h, desc.ctypes.data, 4096, 3, K.F32, 0, 64, 10, None, None) == K.E_WORKSPACE
    bad = desc.copy(); bad[1]["rounds"] = 4          # rounds must agree across the batch
    assert L.kmpar_workspace_size_batched(ctx._h, bad.ctypes.data, 3, K.F32, ctypes.byref(out)) == K.E_INVAL
    bad = desc.copy(); bad[2]["k"] = 1001             # k > n
    assert L.kmpar_workspace_size_batched(ctx._h, bad.ctypes.data, 3, K.F32, ctypes.byref(out)) == K.E_INVAL
    bad = desc.copy(); bad[0]["X"] = 4100             # misaligned X
    assert L.kmpar_init_batched(ctx._h, bad.ctypes.data, 4096, 3, K.F32, 0, 64, 1 << 40, None, None) == K.E_INVAL
    assert L.kmpar_init_batched(ctx._h, desc.ctypes.data, 4100, 3, K.F32, 0, 64, 1 << 40, None, None) == K.E_INVAL
    assert L.kmpar_workspace_size_batched(ctx._h, desc.ctypes.data, 0, K.F32, ctypes.byref(out)) == K.E_INVAL


def test_create_rejects_bad_arguments(K):
    h = ctypes.c_void_p()
    assert K._lib.kmpar_create(0, 5, ctypes.byref(h)) == K.E_INVAL
    assert K._lib.kmpar_create(-2, 0, ctypes.byref(h)) == K.E_INVAL
    assert K._lib.kmpar_create(0, 0, None) == K.E_INVAL


def test_set_option_validation(K):
    ctx = K.Context(None)
    for path in (0, 1, 2, 3):
        assert K._lib.kmpar_set_option(ctx._h, K.OPT_RECLUSTER_PATH, path) == 0
    assert K._lib.kmpar_set_option(ctx._h, K.OPT_RECLUSTER_PATH, 4) == K.E_INVAL
    assert K._lib.kmpar_set_option(ctx._h, K.OPT_RECLUSTER_PATH, -1) == K.E_INVAL
    assert K._lib.kmpar_set_option(ctx._h, 7, 0) == K.E_INVAL
    for v in (0, 1):
        assert K._lib.kmpar_set_option(ctx._h, K.OPT_BATCH_AUTOTUNE, v) == 0
    assert K._lib.kmpar_set_option(ctx._h, K.OPT_BATCH_AUTOTUNE, 2) == K.E_INVAL


def test_batch_tiles_empty_before_any_batch(K):
    ctx = K.Context(None)
    assert ctx.batch_tiles() == []
    cnt = ctypes.c_int32(0)
    assert K._lib.kmpar_batch_tiles(ctx._h, None, None, None, -1, ctypes.byref(cnt)) == K.E_INVAL
    assert K._lib.kmpar_batch_tiles(ctx._h, None, None, None, 4, ctypes.byref(cnt)) == K.E_INVAL


def test_init_rejects_candidate_capacity_overflow(K):
    # 1 + rounds * per-round capacity must fit an int32 (validated before any
    # device work, so a host-only context reports it)
    ctx = K.Context(None)
    assert _call_init(K, ctx, n=2**30, d=8, k=10, ell=1e12, rounds=64, wsb=1 << 62) == K.E_INVAL


def test_noalloc_cost_validation(K):
    # kmpar_cost_noalloc validates and sizes before any HIP call: a call that
    # needs more than the fixed scratch is refused, a fitting one reaches the
    # device check of a host-only context.
    L, ctx = K._lib, K.Context(None)
    h = ctx._h
    assert L.kmpar_cost_noalloc(h, 16, None, K.F32, 1000, 8, 32, 5, 64, None) == K.E_NODEVICE
    assert L.kmpar_cost_noalloc(h, 16, None, K.F32, 9_000_000, 8, 32, 5, 64, None) == K.E_WORKSPACE
    assert "fixed" in L.kmpar_last_error(h).decode()
    assert L.kmpar_cost_noalloc(h, 16, None, K.F32, 1000, 8, 32, 0, 64, None) == K.E_INVAL
    assert L.kmpar_cost_noalloc(h, 16, None, K.F32, 1000, 8, 32, 5, 68, None) == K.E_INVAL
    assert L.kmpar_cost_noalloc(h, 17, None, K.F32, 1000, 8, 32, 5, 64, None) == K.E_INVAL
    refined = K.Context(None, K.MODE_REFINED)     # REFINED also sizes the screen's operands
    assert L.kmpar_cost_noalloc(refined._h, 16, None, K.F32, 400_000, 42, 32, 500, 64,
                                None) == K.E_WORKSPACE
