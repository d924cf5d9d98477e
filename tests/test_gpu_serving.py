"""Batching, cluster queries and admission through the C ABI (GPU).

A query's results must be the same alone and in a mix of concurrently
submitted queries (bit-identical records); cluster queries form their
candidate pairs inside the library and are checked against a brute-force
bounding-sphere test written here and against the oracle.
"""

import numpy as np
import pytest

import oracle
import synth
from parity import assert_contact_order, check_static

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def packing():
    return synth.cfg2_scene(run=3, n=300, phi=0.45, subdivs=(1, 2))


def _clusters(sc, k, rng, sizes=(1, 2, 5, 12, 40)):
    x = sc.state[:, :3]
    seeds = rng.choice(sc.n_particles, size=k, replace=False)
    szs = rng.choice(np.asarray(sizes), size=k)
    return synth.cluster_members(x, seeds, szs)


def _brute_pairs(sc, members, delta_of, dt=0.0):
    """Every pair of cluster members whose bounding spheres (radius = largest
    vertex distance) come within R_a + R_b + delta at the start (dt = 0) or
    at the closest approach of the linear centre paths over [0, dt]; listed
    in cluster order (position a < b). delta_of(i, j) takes index arrays."""
    R = np.array([synth.mesh_radius(V) for V, _ in sc.meshes])[sc.mesh_of]
    x, v = sc.state[:, :3], sc.state[:, 7:10]
    m = np.asarray(members)
    a, b = np.triu_indices(len(m), k=1)
    i, j = m[a], m[b]
    d, dv = x[j] - x[i], v[j] - v[i]
    t = np.zeros(len(a))
    if dt > 0:
        vv = (dv * dv).sum(1)
        nz = vv > 0
        t[nz] = np.clip(-(d[nz] * dv[nz]).sum(1) / vv[nz], 0.0, dt)
    c = d + dv * t[:, None]
    keep = np.sqrt((c * c).sum(1)) <= R[i] + R[j] + delta_of(i, j)
    return np.stack([i[keep], j[keep]], 1).astype(np.int32).reshape(-1, 2)


def test_batch_equals_alone(mcd, packing):
    sc = packing
    rng = np.random.default_rng(1)
    groups = [sc.pairs[rng.choice(sc.pairs.shape[0], size=int(s), replace=False)]
              for s in (1, 3, 17, 60, 2, 33)]
    with mcd.Context(streams=2) as ctx:
        ctx.load_scene(sc)
        _say("alone")
        alone = []
        for g in groups:
            t = ctx.query_pairs(g)
            alone.append(ctx.fetch(t))
        _say("mixed submit")
        tickets = [ctx.query_pairs(g) for g in groups]
        mixed = [ctx.fetch(t) for t in tickets]
    for (pa, ca), (pm, cm) in zip(alone, mixed):
        assert pa.tobytes() == pm.tobytes()
        assert ca.tobytes() == cm.tobytes()
        assert_contact_order(ca)


def test_cluster_query_static(mcd, packing):
    sc = packing
    rng = np.random.default_rng(2)
    halo = sc.halo[sc.mesh_of]
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for members in _clusters(sc, 6, rng):
            _say("cluster", len(members))
            t = ctx.query_cluster(members)
            pr, con, pp = ctx.fetch(t, with_pairs=True)
            exp = _brute_pairs(sc, members, lambda i, j: halo[i] + halo[j])
            assert {tuple(p) for p in pp.tolist()} == {tuple(p) for p in exp.tolist()}
            if pp.shape[0]:
                ref, rcon = oracle.static_pairs(sc, pairs=pp)
                check_static(sc, pp, pr, con, ref, rcon, 1e-6, dense=False)
            assert ctx.cluster_time(t) == 0.0


def test_cluster_query_time_stamps(mcd):
    sc = synth.cfg4_scene(run=2, n=300, subdivs=(1, 2), proxy_r=1.0)
    rng = np.random.default_rng(3)
    halo = sc.halo[sc.mesh_of]
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for members in _clusters(sc, 4, rng, sizes=(8, 20, 40)):
            _say("toi cluster", len(members))
            t = ctx.query_cluster(members, dt=sc.dt)
            pr, con, pp = ctx.fetch(t, with_pairs=True)
            exp = _brute_pairs(sc, members, lambda i, j: halo[i] + halo[j], dt=sc.dt)
            assert {tuple(p) for p in pp.tolist()} == {tuple(p) for p in exp.tolist()}
            if pp.shape[0] == 0:
                continue
            ref, rcon, _ = oracle.toi_pairs(sc, sc.dt, pairs=pp)
            assert np.array_equal(pr["status"], ref["status"])
            assert_contact_order(con)
            coll = ref["status"] == 2
            assert np.all(np.abs(pr["toi"][coll] - ref["toi"][coll]) <= 1e-6 * sc.dt)
            t_new = ctx.cluster_time(t)
            exp_t = ref["toi"][coll].min() if coll.any() else sc.dt
            assert abs(t_new - exp_t) <= 1e-6 * sc.dt


def test_cluster_new_states_and_duplicates(mcd, packing):
    sc = packing
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        members = np.array([0, 1, 2], np.int32)
        st = sc.state[members].copy()
        st[1, :3] = st[0, :3] + [2.0, 0, 0]       # move particle 1 next to 0
        _say("cluster with states")
        t = ctx.query_cluster(members, states=st)
        pr, con, pp = ctx.fetch(t, with_pairs=True)
        assert [0, 1] in pp.tolist()
        with pytest.raises(mcd.MCDError):
            ctx.query_cluster(np.array([0, 0], np.int32))


def test_admission_budget_and_timeout(mcd, packing):
    sc = packing
    with mcd.Context(mem_budget=1 << 12) as ctx:
        ctx.load_scene(sc)
        _say("admission refusal")
        with pytest.raises(mcd.MCDError) as e:
            ctx.query_pairs(sc.pairs)
        assert e.value.code == -4
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        t = ctx.query_pairs(sc.pairs, flags=mcd.Q_FP64 | mcd.Q_DENSE)
        _say("timeout")
        try:
            ctx.wait(t, timeout_ns=0)
            timed_out = False
        except mcd.MCDError as e:
            assert e.code == -5
            timed_out = True
        ctx.wait(t)
        assert ctx.poll(t)
        pr, con = ctx.fetch(t)
        assert pr.shape[0] == sc.pairs.shape[0]
        print("timed out before completion:", timed_out)


def test_cfg5_clusters_at_full_residency(mcd):
    """Cluster queries against the full serving population (100,000 resident
    particles, 4,096 distinct meshes of 80-1,280 triangles): cluster sizes
    from the power law plus a 2,000-particle cluster, submitted together so
    they share batches. Candidate pairs equal a brute-force bounding-sphere
    test; a seeded sample of every cluster's pairs is compared with the
    oracle."""
    sc = synth.cfg5_scene(run=0)
    rng = np.random.default_rng(55)
    sizes = list(synth.cluster_sizes(6, rng)) + [2000]
    seeds = rng.integers(0, sc.n_particles, size=len(sizes))
    members = synth.cluster_members(sc.state[:, :3], seeds, sizes)
    halo = sc.halo[sc.mesh_of]
    _say("cfg5 population", sc.n_particles, "clusters", [len(m) for m in members])
    with mcd.Context(streams=2) as ctx:
        ctx.load_scene(sc)
        tickets = [ctx.query_cluster(m) for m in members]
        res = [ctx.fetch(t, with_pairs=True) for t in tickets]
    for members_k, (pr, con, pp) in zip(members, res):
        exp = _brute_pairs(sc, members_k, lambda i, j: halo[i] + halo[j])
        assert {tuple(p) for p in pp.tolist()} == {tuple(p) for p in exp.tolist()}
        assert_contact_order(con)
        if pp.shape[0] == 0:
            continue
        k = min(12, pp.shape[0])
        idx = np.sort(rng.choice(pp.shape[0], size=k, replace=False))
        touching = np.where(pr["contact"] == 1)[0]
        idx = np.union1d(idx, touching[:3])
        ref, rcon = oracle.static_pairs(sc, pairs=pp[idx])
        pos = {int(p): j for j, p in enumerate(idx)}
        sel = np.array([c for c in con if int(c["pair"]) in pos], dtype=con.dtype)
        for c in sel:
            c["pair"] = pos[int(c["pair"])]
        check_static(sc, pp[idx], pr[idx], sel, ref, rcon, 1e-6, dense=False)


def _oracle_bp(sc, members, dt):
    """The oracle's broad phase on the members' bounding spheres (radius =
    largest vertex distance + halo), mapped back to particle ids."""
    R = np.array([synth.mesh_radius(V) for V, _ in sc.meshes])[sc.mesh_of]
    halo = sc.halo[sc.mesh_of]
    m = np.asarray(members)
    p, lab, _ = oracle.broad_phase(sc.state[m, :3], sc.state[m, 7:10], (R + halo)[m], dt)
    return m[p], lab


def test_broad_phase_and_clusters(mcd):
    """mcd_broad_phase on the device against the oracle's (checks 1 and 2 of
    section 3, then min-labelling): the same pairs in the same order and the
    same clusters, static and moving, for 300 and 10,000 particles."""
    counts = []
    for sc, dt in ((synth.cfg2_scene(run=3, n=300, phi=0.45, subdivs=(1, 2)), 0.0),
                   (synth.cfg4_scene(run=2, n=300, subdivs=(1, 2), proxy_r=1.0), None),
                   (synth.cfg4_scene(run=0), None)):
        dt = sc.dt if dt is None else dt
        rng = np.random.default_rng(7)
        members = rng.permutation(sc.n_particles).astype(np.int32)
        _say("broad phase", sc.n_particles, dt)
        with mcd.Context() as ctx:
            ctx.load_scene(sc)
            lab, k, pairs = ctx.broad_phase(members, dt=dt)
        exp_pairs, exp_lab = _oracle_bp(sc, members, dt)
        assert pairs.tolist() == exp_pairs.tolist()
        # clusters numbered by their first member: the oracle's labels are
        # those first members' positions
        first = {}
        exp_id = np.array([first.setdefault(int(l), len(first)) for l in exp_lab])
        assert np.array_equal(lab, exp_id) and k == len(first)
        counts.append((k, len(members)))
    # the dense static packing percolates into one cluster; the sparse moving
    # packings split into many
    assert counts[0][0] >= 1 and all(1 < k < m for k, m in counts[1:])


def test_device_cluster_batches(mcd):
    """Static cluster queries whose pairs are found on the device, submitted
    together so that they share batches: each result equals the same query
    alone, the pairs equal the oracle's broad phase, and sampled pairs equal
    the oracle's contact query."""
    sc = synth.cfg2_scene(run=3, n=300, phi=0.45, subdivs=(1, 2))
    rng = np.random.default_rng(12)
    clusters = _clusters(sc, 12, rng, sizes=(1, 2, 3, 8, 30, 60))
    with mcd.Context(streams=1) as ctx:
        ctx.load_scene(sc)
        alone = []
        for m in clusters:
            t = ctx.query_cluster(m)
            alone.append(ctx.fetch(t, with_pairs=True))
            ctx.release(t)
        tickets = [ctx.query_cluster(m) for m in clusters]
        mixed = [ctx.fetch(t, with_pairs=True) for t in tickets]
        batched = max(ctx.stats(t)["batch_queries"] for t in tickets)
    assert batched > 1
    for m, (pa, ca, ppa), (pm, cm, ppm) in zip(clusters, alone, mixed):
        assert pa.tobytes() == pm.tobytes() and ca.tobytes() == cm.tobytes() and ppa.tobytes() == ppm.tobytes()
        exp, _ = _oracle_bp(sc, m, 0.0)
        assert ppa.tolist() == exp.tolist()
        if ppa.shape[0]:
            idx = np.arange(min(8, ppa.shape[0]))
            ref, rcon = oracle.static_pairs(sc, pairs=ppa[idx])
            sel = ca[ca["pair"] < len(idx)]
            check_static(sc, ppa[idx], pa[idx], sel, ref, rcon, 1e-6, dense=False)


def test_capture_counter_on_empty_queries(mcd, packing):
    """graph_captures is the context's running count on every completed
    query, also on queries with nothing to evaluate (a one-particle cluster,
    an empty pair list), which complete at submission."""
    sc = packing
    with mcd.Context(streams=1) as ctx:
        ctx.load_scene(sc)
        _say("capture counter, empty queries")
        counts = []
        # the first runs of a size class measure launch shapes (eager
        # launches); the chain is captured once the shape is chosen
        for _ in range(200):
            t = ctx.query_pairs(sc.pairs[:50])
            ctx.wait(t)
            counts.append(ctx.stats(t)["graph_captures"])
            ctx.release(t)
            if counts[-1] >= 1:
                break
        assert counts[-1] >= 1 and counts == sorted(counts)
        for t in (ctx.query_cluster(np.array([0], np.int32)), ctx.query_pairs(np.zeros((0, 2), np.int32))):
            ctx.wait(t)
            st = ctx.stats(t)
            assert st["batch_queries"] == 0 and st["graph_captures"] == counts[-1]
            ctx.release(t)
