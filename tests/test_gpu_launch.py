"""Launch modes of the static chain (GPU): replayed HIP graphs, kernel-by-
kernel launches and every autotuner launch shape give bit-identical results.

Graph replays are interleaved with eager queries of other sizes and with
host synchronisation, and every replay is compared with the eager result.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


@pytest.fixture(scope="module")
def packing():
    return synth.cfg2_scene(run=3, n=300, phi=0.45, subdivs=(1, 2))


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _run(ctx, pairs, flags):
    t = ctx.query_pairs(pairs, flags=flags)
    pr, con = ctx.fetch(t)
    st = ctx.stats(t)
    ctx.release(t)
    return pr, con, st


def _same(a, b):
    return a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()


@pytest.mark.parametrize("flags_name", ["Q_MIXED", "Q_FP64"])
def test_graph_replay_equals_eager(mcd, packing, flags_name):
    sc = packing
    flags = getattr(mcd, flags_name)
    rng = np.random.default_rng(7)
    subsets = [sc.pairs, sc.pairs[:17], sc.pairs[rng.choice(sc.pairs.shape[0], 200, replace=False)],
               sc.pairs[:1]]
    with mcd.Context(flags=mcd.CFG_NO_GRAPHS | mcd.CFG_NO_TUNE) as ref_ctx:
        ref_ctx.load_scene(sc)
        ref = [_run(ref_ctx, p, flags) for p in subsets]
    with mcd.Context(flags=mcd.CFG_NO_TUNE) as ctx:
        ctx.load_scene(sc)
        for rep in range(3):
            for k, p in enumerate(subsets):
                _say("graph", flags_name, rep, k, p.shape[0])
                got = _run(ctx, p, flags)
                assert _same(got, ref[k]), (rep, k)
                # eager work in between replays
                timed = _run(ctx, p, flags | mcd.Q_TIMING)
                assert _same(timed, ref[k])
                assert timed[2]["near_ms"] > 0 and timed[2]["main_ms"] > 0


def test_autotuner_shapes_identical(mcd, packing):
    """The first queries of a bucket run every candidate shape (twice); the
    results never depend on the shape."""
    sc = packing
    with mcd.Context(flags=mcd.CFG_NO_GRAPHS | mcd.CFG_NO_TUNE) as ref_ctx:
        ref_ctx.load_scene(sc)
        ref = _run(ref_ctx, sc.pairs, mcd.Q_MIXED)
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for k in range(16):
            _say("tune", k)
            got = _run(ctx, sc.pairs, mcd.Q_MIXED)
            assert _same(got, ref), k


def test_tune_cache_persists(mcd, packing, tmp_path):
    """The autotuner's choice survives the context: a second context reading
    the same cache file starts tuned (no trial shapes), with bit-identical
    results; a file from another device model or shape set is ignored."""
    path = str(tmp_path / "tune.txt")
    with mcd.Context(tune_cache=path) as ctx:
        ctx.load_scene(packing)
        first = None
        for _ in range(40):
            t = ctx.query_pairs(packing.pairs)
            pr, con = ctx.fetch(t)
            st = ctx.stats(t)
            ctx.release(t)
            first = first or (pr.tobytes(), con.tobytes())
            if st["tune_pending"] == 0:
                break
        assert st["tune_pending"] == 0
    text = open(path).read().splitlines()
    assert text[0].startswith("mcd-tune 1 ") and len(text) >= 2
    with mcd.Context(tune_cache=path) as ctx:
        ctx.load_scene(packing)
        t = ctx.query_pairs(packing.pairs)
        pr, con = ctx.fetch(t)
        assert ctx.stats(t)["tune_pending"] == 0
        assert (pr.tobytes(), con.tobytes()) == first
    with open(path, "w") as f:
        f.write("mcd-tune 1 another-device shapes 1/1\n0 0\n")
    with mcd.Context(tune_cache=path) as ctx:
        ctx.load_scene(packing)
        t = ctx.query_pairs(packing.pairs)
        ctx.fetch(t)
        assert ctx.stats(t)["tune_pending"] > 0


def test_time_stamp_graph_replay_equals_eager(mcd):
    """The time-stamp chain: launched eagerly the first time its shape is
    met, captured the second time, replayed after that; interleaved with a
    query of another size. Every result equals the eager launches of a
    context without graphs, bit for bit."""
    mv = synth.cfg4_scene(run=3, n=400, subdivs=(1, 2), proxy_r=1.0)
    other = mv.pairs[: mv.pairs.shape[0] // 3]
    with mcd.Context(flags=mcd.CFG_NO_GRAPHS) as ctx:
        ctx.load_scene(mv)
        t = ctx.query_pairs(mv.pairs, dt=mv.dt)
        ref = ctx.fetch(t)
        t = ctx.query_pairs(other, dt=mv.dt)
        ref_other = ctx.fetch(t)
    assert (ref[0]["status"] == mcd.COLLIDES).any()
    with mcd.Context(streams=1) as ctx:
        ctx.load_scene(mv)
        for k in range(5):
            _say("time-stamp replay", k)
            t = ctx.query_pairs(mv.pairs, dt=mv.dt)
            got = ctx.fetch(t)
            ctx.release(t)
            assert _same(got, ref), k
            t = ctx.query_pairs(other, dt=mv.dt)
            got = ctx.fetch(t)
            ctx.release(t)
            assert _same(got, ref_other), k
        # per-stage times come with MCD_Q_TIMING (kernel by kernel)
        t = ctx.query_pairs(mv.pairs, dt=mv.dt, flags=mcd.Q_MIXED | mcd.Q_TIMING)
        got = ctx.fetch(t)
        st = ctx.stats(t)
        assert _same(got, ref) and st["near_ms"] > 0 and st["endgame_ms"] > 0
