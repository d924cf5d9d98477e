"""GPU parity of the paper's narrowing estimate (MCD_Q_NARROW: section 5,
"Collision time detection"; translation only) against the oracle's
narrowing: statuses equal, time stamps within 1e-9 * dt, the reported
triangle pair and the contact set at the time stamp equal, closest points
checked at that time with the same translation-only motion."""

import numpy as np
import pytest

import oracle
import synth
from parity import assert_contact_order, check_points, contact_set
from test_oracle_narrow import BIG, SPIKE, DELTA, _pair_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _gpu(mcd, sc, dt, flags=0):
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        t = ctx.query_pairs(sc.pairs, dt=dt, flags=flags | mcd.Q_NARROW)
        pr, con = ctx.fetch(t)
        st = ctx.stats(t)
        tn = ctx.cluster_time(t)
    return pr, con, st, tn


def _no_spin(sc):
    st = sc.state.copy()
    st[:, 10:13] = 0.0
    return synth.Scene(meshes=sc.meshes, halo=sc.halo, mesh_of=sc.mesh_of, state=st, pairs=sc.pairs, dt=sc.dt)


def check_narrow(mcd, sc, dt, pr, con):
    ref, rcon, rounds = oracle.narrow_pairs(sc, dt)
    assert np.array_equal(pr["status"], ref["status"]), (pr["status"], ref["status"])
    hit = ref["status"] > 0
    assert np.all(np.abs(pr["toi"][hit] - ref["toi"][hit]) <= 1e-9 * dt)
    assert np.all(np.isinf(pr["toi"][~hit]))
    assert np.array_equal(pr["tri_a"][hit], ref["tri_a"][hit]) and np.array_equal(pr["tri_b"][hit], ref["tri_b"][hit])
    assert contact_set(con) == contact_set(rcon)
    assert_contact_order(con)
    assert np.array_equal(con["t"], pr["toi"][con["pair"]])
    times = np.where(np.isfinite(pr["toi"]), pr["toi"], 0.0)
    sel = con if con.shape[0] <= 3000 else con[:: con.shape[0] // 3000 + 1]
    check_points(_no_spin(sc), sc.pairs, sel, times=times)
    return ref, rounds


def test_closed_forms(mcd):
    h, v = 0.3, 2.0
    sc = _pair_scene(*BIG, *SPIKE, [0, 0, 0], [0, 0, h], [0, 0, 0], [0, 0, -v])
    _say("narrow: vertex onto face")
    pr, con, st, tn = _gpu(mcd, sc, 0.5)
    assert pr["status"][0] == mcd.COLLIDES and abs(pr["toi"][0] - h / v) <= 1e-12 and tn == pr["toi"][0]
    check_narrow(mcd, sc, 0.5, pr, con)
    pr, con, _, _ = _gpu(mcd, sc, (h - 2 * DELTA) / v)
    assert pr["status"][0] == mcd.NONE and con.shape[0] == 0
    A = ([[-2, 0, 0], [2, 0, 0], [0.7, -1.0, 0]], [[0, 1, 2]])
    B = ([[0, -2, 0], [0, 2, 0], [-0.7, 0, 1.0]], [[0, 1, 2]])
    g0, u, dt = 0.5, 1.0, 1.0
    sc = _pair_scene(*A, *B, [0, 0, 0], [0, 0, g0], [0, 0, 0], [0, 0, -u])
    _say("narrow: crossed edges")
    pr, con, st, _ = _gpu(mcd, sc, dt)
    t_true = (g0 - DELTA) / u
    k = 0
    while dt / 2 ** (k + 1) >= t_true:
        k += 1
    assert pr["toi"][0] == dt / 2 ** k and st["candidates"] == k + 1
    check_narrow(mcd, sc, dt, pr, con)


@pytest.mark.parametrize("run", [0, 1])
def test_random_pairs_and_spin_ignored(mcd, run):
    rng = np.random.default_rng(700 + run)
    V, F = synth.icosphere(1)
    n = 12
    meshes = [(synth.perturb_radial(V, rng, 0.1), F) for _ in range(2 * n)]
    st = np.zeros((2 * n, 13))
    st[:, 3:7] = synth.random_quaternions(2 * n, rng)
    u = synth.random_unit_vectors(n, rng)
    for p in range(n):
        st[2 * p, :3] = [10.0 * p, 0, 0]
        st[2 * p + 1, :3] = st[2 * p, :3] + rng.uniform(2.05, 2.3) * u[p]
        st[2 * p + 1, 7:10] = -rng.uniform(0.5, 3.0) * u[p] + 0.3 * rng.normal(size=3)
    st[:, 10:13] = rng.normal(size=(2 * n, 3)) * 5.0     # spin: neglected by the estimate
    pairs = np.stack([np.arange(0, 2 * n, 2), np.arange(1, 2 * n, 2)], 1).astype(np.int32)
    sc = synth.Scene(meshes=meshes, halo=np.full(2 * n, DELTA / 2), mesh_of=np.arange(2 * n, dtype=np.int32),
                     state=st, pairs=pairs)
    dt = 0.3
    _say("narrow: random pairs", run)
    pr, con, stats, tn = _gpu(mcd, sc, dt)
    ref, _ = check_narrow(mcd, sc, dt, pr, con)
    assert (ref["status"] == 2).sum() >= 4
    coll = ref["status"] == 2
    assert abs(tn - (ref["toi"][coll].min() if coll.any() else dt)) <= 1e-9 * dt
    # the exact first contact without spin is never later than the estimate
    ns = _no_spin(sc)
    with mcd.Context() as ctx:
        ctx.load_scene(ns)
        t = ctx.query_pairs(ns.pairs, dt=dt)
        ex, _ = ctx.fetch(t)
    both = (ex["status"] > 0) & (pr["status"] > 0)
    assert np.all(pr["status"][pr["status"] > 0] > 0) and np.all(ex["status"][pr["status"] > 0] > 0)
    assert np.all(ex["toi"][both] <= pr["toi"][both] + 1e-6 * dt)


def test_moving_packing(mcd):
    """400 moving perturbed icospheres, every candidate pair against the
    oracle's narrowing."""
    sc = synth.cfg4_scene(run=1, n=400, subdivs=(1, 2), proxy_r=1.0)
    _say("narrow: moving packing", sc.pairs.shape[0], sc.dt)
    pr, con, st, tn = _gpu(mcd, sc, sc.dt)
    ref, rounds = check_narrow(mcd, sc, sc.dt, pr, con)
    assert (ref["status"] == 2).sum() >= 3 and rounds.max() >= 2
