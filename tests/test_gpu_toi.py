"""GPU parity of collision time stamps against the FP64 oracle.

Time stamps agree within 1e-6 * dt (the bisection tolerance); statuses are
equal; the reported triangle pair attains the minimum; contact sets at the
time stamp equal the oracle's at the GPU's own time stamp, with closest
points checked at that time.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from parity import assert_contact_order, check_points, contact_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _state(x, q, v=(0, 0, 0), w=(0, 0, 0)):
    return np.concatenate([x, q, v, w]).astype(np.float64)


def _gpu_toi(mcd, sc, pairs, dt, S=64, tol_rel=1e-6, flags=0):
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        t = ctx.query_pairs(pairs, dt=dt, flags=flags, samples=S, tol_rel=tol_rel)
        pr, con = ctx.fetch(t)
        st = ctx.stats(t)
        tn = ctx.cluster_time(t)
    return pr, con, st, tn


def check_toi(sc, pairs, dt, pr, con, ref, rcon, rtol=1e-6):
    """Statuses equal; time stamps within rtol * dt; the winning triangle pair
    in contact at the GPU's time stamp; the contact set of every pair with a
    time stamp equal to the oracle's static contact set at the GPU's own time
    stamp (the oracle's records when both times are the same number), every
    record's closest points checked at that time."""
    n = pairs.shape[0]
    assert np.array_equal(pr["status"], ref["status"]), (pr["status"], ref["status"])
    halo = sc.halo[sc.mesh_of]
    delta = halo[pairs[:, 0]] + halo[pairs[:, 1]]
    same_t = np.zeros(n, bool)
    exp = set()
    rset = contact_set(rcon)
    for p in range(n):
        if ref["status"][p] == oracle.STATUS_NONE:
            assert not np.isfinite(pr["toi"][p]) and pr["tri_a"][p] == -1
            continue
        assert abs(pr["toi"][p] - ref["toi"][p]) <= rtol * dt, (p, pr["toi"][p], ref["toi"][p])
        same_t[p] = pr["toi"][p] == ref["toi"][p]
        assert pr["contact"][p] == 1 and pr["dmin"][p] <= delta[p] * (1 + 1e-9)
        # the winning triangle pair is in contact at the GPU's time stamp (oracle check)
        ia, ib = pairs[p]
        Va, Fa = sc.meshes[sc.mesh_of[ia]]
        Vb, Fb = sc.meshes[sc.mesh_of[ib]]
        ta = oracle.world_tris(Va, Fa[[pr["tri_a"][p]]], sc.state[ia], pr["toi"][p])
        tb = oracle.world_tris(Vb, Fb[[pr["tri_b"][p]]], sc.state[ib], pr["toi"][p])
        d, *_ = oracle.tri_tri(ta[0], tb[0])
        assert abs(d - pr["dmin"][p]) <= rtol * delta[p]
        if same_t[p] and (pr["tri_a"][p], pr["tri_b"][p]) == (ref["tri_a"][p], ref["tri_b"][p]):
            assert np.abs(pr["pa"][p] - ref["pa"][p]).max() <= 1e-6 * delta[p] * 10
        if same_t[p]:
            exp |= {c for c in rset if c[0] == p}
        else:
            # the oracle's static query at the GPU's time stamp
            _, rc = oracle.static_pairs(sc, pairs=pairs[[p]], t=float(pr["toi"][p]))
            exp |= {(p, int(c["tri_a"]), int(c["tri_b"])) for c in rc}
    got = contact_set(con)
    assert got == exp, (sorted(exp - got)[:8], sorted(got - exp)[:8])
    assert_contact_order(con)
    if "t" in con.dtype.names:
        assert np.array_equal(con["t"], pr["toi"][con["pair"]])
    times = np.where(np.isfinite(pr["toi"]), pr["toi"], 0.0)
    sel = con
    if con.shape[0] > 3000:
        rng = np.random.default_rng(len(con))
        sel = con[np.sort(rng.choice(con.shape[0], size=3000, replace=False))]
    check_points(sc, pairs, sel, times=times, rtol=rtol)
    return same_t


def test_translation_closed_form(mcd):
    V, F = synth.icosphere(0)
    u = V[0] / np.linalg.norm(V[0])
    eps, sep, vr, dt = 0.01, 2.3, 1.7, 0.25
    sc = synth.pair_test_scene((V, F), (V, F), _state(np.zeros(3), [1, 0, 0, 0]),
                               _state(sep * u, [1, 0, 0, 0], v=-vr * u), eps)
    _say("toi translation")
    for flags in (0, 1):
        pr, con, st, tn = _gpu_toi(mcd, sc, sc.pairs, dt, flags=flags)
        t_true = (sep - 2 - 2 * eps) / vr
        assert pr["status"][0] == mcd.COLLIDES
        assert -1e-15 <= pr["toi"][0] - t_true <= 1e-6 * dt + 1e-15
        assert tn == pr["toi"][0]
        ref, rcon, _ = oracle.toi_pairs(sc, dt)
        check_toi(sc, sc.pairs, dt, pr, con, ref, rcon)


@pytest.mark.parametrize("phi0,omega", [(-1.0, 2.0), (-2.0, 3.0)])
def test_spinning_vertex(mcd, phi0, omega):
    c, eps = 0.95, 0.01
    ca, sa_ = math.cos(phi0), math.sin(phi0)
    Rz = np.array([[ca, -sa_, 0], [sa_, ca, 0], [0, 0, 1]])
    VA = np.array([[1.0, 0, 0], [-0.1, 0.05, 0], [-0.1, -0.05, 0]]) @ Rz.T
    VB = np.array([[0, -5, -5], [0, 5, -5], [0, 0, 5.0]])
    F1 = np.array([[0, 1, 2]], np.int32)
    sc = synth.pair_test_scene((VA, F1), (VB, F1), _state(np.zeros(3), [1, 0, 0, 0], w=[0, 0, omega]),
                               _state([c, 0, 0], [1, 0, 0, 0]), eps)
    t_true = (-math.acos(c - 2 * eps) - phi0) / omega
    dt = 1.5 * t_true
    _say("toi spin", phi0, omega)
    pr, con, st, tn = _gpu_toi(mcd, sc, sc.pairs, dt)
    assert pr["status"][0] == mcd.COLLIDES
    assert -1e-15 <= pr["toi"][0] - t_true <= 1e-6 * dt + 1e-15
    ref, rcon, _ = oracle.toi_pairs(sc, dt)
    check_toi(sc, sc.pairs, dt, pr, con, ref, rcon)


def _random_pairs_scene(run, n_pairs=10, subdiv=1):
    rng = np.random.default_rng(4400 + run)
    V, F = synth.icosphere(subdiv)
    meshes = [(synth.perturb_radial(V, rng, 0.1), F) for _ in range(2 * n_pairs)]
    st = np.zeros((2 * n_pairs, 13))
    q = synth.random_quaternions(2 * n_pairs, rng)
    u = synth.random_unit_vectors(n_pairs, rng)
    for p in range(n_pairs):
        st[2 * p, :3] = [10.0 * p, 0, 0]
        st[2 * p + 1, :3] = st[2 * p, :3] + rng.uniform(2.05, 2.4) * u[p]
        st[2 * p + 1, 7:10] = -rng.uniform(0.5, 3.0) * u[p] + rng.normal(size=3) * 0.3
        st[2 * p, 7:10] = rng.normal(size=3) * 0.3
        st[:, 10:13] = rng.normal(size=(2 * n_pairs, 3)) * 5.0
    st[:, 3:7] = q
    if run % 2 == 1:   # one pair starts in contact
        st[1, :3] = st[0, :3] + 1.9 * u[0]
    pairs = np.stack([np.arange(0, 2 * n_pairs, 2), np.arange(1, 2 * n_pairs, 2)], 1).astype(np.int32)
    return synth.Scene(meshes=meshes, halo=np.full(2 * n_pairs, 0.01),
                       mesh_of=np.arange(2 * n_pairs, dtype=np.int32), state=st, pairs=pairs)


@pytest.mark.parametrize("run", [0, 1, 2])
@pytest.mark.parametrize("flags", [0, 1], ids=["mixed", "fp64"])
def test_random_rotating_pairs(mcd, run, flags):
    sc = _random_pairs_scene(run)
    dt = 0.12
    _say("toi random", run, flags)
    pr, con, st, tn = _gpu_toi(mcd, sc, sc.pairs, dt, S=32, flags=flags)
    ref, rcon, _ = oracle.toi_pairs(sc, dt, S=32)
    assert (ref["status"] == oracle.STATUS_COLLIDES).sum() >= 2
    check_toi(sc, sc.pairs, dt, pr, con, ref, rcon)
    coll = ref["status"] == oracle.STATUS_COLLIDES
    exp_t = ref["toi"][coll].min() if coll.any() else dt
    assert abs(tn - exp_t) <= 1e-6 * dt


def test_reduced_moving_packing(mcd):
    """400 moving perturbed icospheres (80/320 triangles); dt calibrated with
    nominal-radius spheres, which gives about 8% colliding pairs here."""
    sc = synth.cfg4_scene(run=1, n=400, subdivs=(1, 2), proxy_r=1.0)
    _say("toi packing-400", sc.pairs.shape[0], sc.dt)
    pr, con, st, tn = _gpu_toi(mcd, sc, sc.pairs, sc.dt)
    ref, rcon, _ = oracle.toi_pairs(sc, sc.dt)
    assert (ref["status"] == oracle.STATUS_COLLIDES).sum() >= 3
    same = check_toi(sc, sc.pairs, sc.dt, pr, con, ref, rcon)
    assert same[ref["status"] > 0].mean() >= 0.9


def test_regrow_equals_default(mcd):
    """First-phase candidates beyond a tiny initial capacity: the overflow is
    found after the second phase has run on the incomplete time stamps, and
    both phases run again with larger buffers. The result equals, bit for
    bit, that of a context whose buffers fit."""
    sc = synth.cfg4_scene(run=1, n=400, subdivs=(1, 2), proxy_r=1.0)
    _say("toi regrow", sc.pairs.shape[0])
    pr, con, st, _ = _gpu_toi(mcd, sc, sc.pairs, sc.dt)
    assert st["retries"] == 0 and (pr["status"] > 0).sum() >= 3
    with mcd.Context(contact_cap=8) as ctx:
        ctx.load_scene(sc)
        t = ctx.query_pairs(sc.pairs, dt=sc.dt)
        pr2, con2 = ctx.fetch(t)
        st2 = ctx.stats(t)
    assert st2["retries"] >= 1
    assert pr2.tobytes() == pr.tobytes()
    assert con2.tobytes() == con.tobytes()


def test_full_size_sampled(mcd):
    """10,000 moving particles (320/1280 triangles), all candidate pairs in one
    query; the oracle recomputes a sample (colliding pairs and others)."""
    sc = synth.cfg4_scene(run=0)
    _say("toi full", sc.pairs.shape[0], sc.dt)
    pr, con, st, tn = _gpu_toi(mcd, sc, sc.pairs, sc.dt)
    rng = np.random.default_rng(5)
    coll = np.where(pr["status"] > 0)[0]
    assert coll.size >= 20
    nt = sc.tri_counts()[sc.mesh_of]
    cost = nt[sc.pairs[:, 0]] * nt[sc.pairs[:, 1]]
    small = np.where(cost <= 320 * 1280)[0]
    pick = set(rng.choice(coll, size=min(6, coll.size), replace=False).tolist())
    pick |= set(rng.choice(small, size=6, replace=False).tolist())
    # the largest meshes of the packing: 1,280 x 1,280 pairs, colliding ones first
    big = np.where(cost == 1280 * 1280)[0]
    big_hit = np.intersect1d(big, coll)
    pick |= set(rng.choice(big_hit, size=min(2, big_hit.size), replace=False).tolist())
    pick |= set(rng.choice(big, size=2, replace=False).tolist())
    idx = np.array(sorted(pick))
    ref, rcon, _ = oracle.toi_pairs(sc, sc.dt, pairs=sc.pairs[idx])
    pos = {int(p): k for k, p in enumerate(idx)}
    sel = np.array([c for c in con if int(c["pair"]) in pos], dtype=con.dtype)
    for c in sel:
        c["pair"] = pos[int(c["pair"])]
    check_toi(sc, sc.pairs[idx], sc.dt, pr[idx], sel, ref, rcon)


def test_edge_cases(mcd):
    """Empty query; no relative motion (L = 0) out of and in contact; a
    common velocity and spin (rigid together: never closer); the extreme
    sample counts and the smallest tolerance. Checked against the oracle."""
    V, F = synth.icosphere(1)
    rng = np.random.default_rng(11)
    q = synth.random_quaternions(8, rng)
    st = np.zeros((8, 13))
    st[:, 3:7] = q
    st[0, :3] = [0, 0, 0]; st[1, :3] = [2.3, 0, 0]            # static, apart
    st[2, :3] = [10, 0, 0]; st[3, :3] = [11.9, 0, 0]          # static, overlapping
    st[4, :3] = [20, 0, 0]; st[5, :3] = [22.05, 0.1, 0]       # moving together
    st[4, 7:10] = st[5, 7:10] = [3.0, -1.0, 0.5]
    st[6, :3] = [30, 0, 0]; st[7, :3] = [32.4, 0, 0]          # approaching, spinning
    st[7, 7:10] = [-6.0, 0, 0]; st[6, 10:13] = [0, 0, 4.0]; st[7, 10:13] = [3.0, 0, 0]
    sc = synth.Scene(meshes=[(V, F)], halo=np.array([0.01]), mesh_of=np.zeros(8, np.int32),
                     state=st, pairs=np.array([[0, 1], [2, 3], [4, 5], [6, 7]], np.int32))
    dt = 0.1
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        _say("toi edge: empty")
        t = ctx.query_pairs(np.zeros((0, 2), np.int32), dt=dt)
        pr, con = ctx.fetch(t)
        assert pr.shape[0] == 0 and con.shape[0] == 0
        assert ctx.cluster_time(t) == dt
        for S, tol in ((64, 1e-6), (1, 1e-6), (128, 1e-6), (64, 1e-7)):
            _say("toi edge: S", S, "tol", tol)
            t = ctx.query_pairs(sc.pairs, dt=dt, samples=S, tol_rel=tol)
            pr, con = ctx.fetch(t)
            ref, rcon, _ = oracle.toi_pairs(sc, dt, S=S, tol_rel=tol)
            assert pr["status"].tolist() == [0, 1, 0, 2], pr["status"]
            check_toi(sc, sc.pairs, dt, pr, con, ref, rcon, rtol=max(tol, 1e-6))
