"""GPU parity of the static contact query against the FP64 oracle.

Every call goes through libmcd.so (C ABI). Tolerances: FP64 outputs within
1e-6 relative in the form |x - x_ref| <= 1e-6 * max(|x_ref|, delta); contact
sets and flags bit-exact.
"""

import numpy as np
import pytest

import oracle
import synth
from parity import assert_contact_order, check_static, contact_set

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _run(m, ctx, scene, pairs, flags):
    t = ctx.query_pairs(pairs, flags=flags)
    pr, con = ctx.fetch(t)
    st = ctx.stats(t)
    ctx.release(t)
    return pr, con, st


MODES = [("fp64-dense", 1 | 4), ("mixed-dense", 2 | 4), ("fp64-culled", 1), ("mixed-culled", 2)]


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_cfg1_all_modes(mcd, mode):
    name, flags = mode
    sc = synth.cfg1_scene(run=0)
    ref, rcon = oracle.static_pairs(sc)
    _say("cfg1", name, "pairs", sc.pairs.shape[0])
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        pr, con, st = _run(mcd, ctx, sc, sc.pairs, flags)
    check_static(sc, sc.pairs, pr, con, ref, rcon, RTOL, dense=bool(flags & 4))
    if flags & 4:
        assert st["tile_pairs_kept"] == st["tile_pairs_total"] == 16 * 25


def _ragged_scene(run, n_pairs=12, tmin=20, tmax=700, eps=0.005):
    rng = np.random.default_rng(9000 + run)
    T = rng.integers(tmin, tmax, size=2 * n_pairs)
    meshes = [synth.uv_sphere(int(t)) for t in T]
    # perturb so that meshes are not all symmetric copies
    meshes = [(synth.perturb_radial(V, rng, 0.05), F) for V, F in meshes]
    n = 2 * n_pairs
    q = synth.random_quaternions(n, rng)
    u = synth.random_unit_vectors(n_pairs, rng)
    g = rng.uniform(0.0, 2 * eps, size=n_pairs)
    x = np.zeros((n, 3))
    x[0::2, 0] = 10.0 * np.arange(n_pairs)
    R = np.array([synth.mesh_radius(V) for V, _ in meshes])
    x[1::2] = x[0::2] + (R[0::2] + R[1::2] + g)[:, None] * u - 0.08 * u
    st = np.zeros((n, 13))
    st[:, :3] = x
    st[:, 3:7] = q
    pairs = np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], axis=1).astype(np.int32)
    return synth.Scene(meshes=meshes, halo=np.full(n, eps), mesh_of=np.arange(n, dtype=np.int32),
                       state=st, pairs=pairs)


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_ragged_tiles_all_modes(mcd, mode):
    """Triangle counts that are not multiples of the 64-triangle tile, and
    pairs that interpenetrate a little (intersecting triangles, d = 0)."""
    name, flags = mode
    sc = _ragged_scene(1)
    ref, rcon = oracle.static_pairs(sc)
    assert ref["contact"].sum() >= 3 and (ref["d"] == 0).sum() >= 1
    _say("ragged", name)
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        pr, con, st = _run(mcd, ctx, sc, sc.pairs, flags)
    check_static(sc, sc.pairs, pr, con, ref, rcon, RTOL, dense=bool(flags & 4))


def test_edge_cases(mcd):
    V, F = synth.icosphere(1)
    tri1 = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]]), np.array([[0, 1, 2]], np.int32))
    with mcd.Context() as ctx:
        a = ctx.mesh_load(V, F, 0.01)
        b = ctx.mesh_load(*tri1, 0.01)
        st = np.zeros((4, 13))
        st[:, 3] = 1.0
        st[1, :3] = [5.0, 0, 0]          # far from 0: every tile pair culled
        st[2, :3] = [0.0, 0, 1.005]      # single triangle just above the sphere
        st[3, :3] = [0.0, 0, 0.5]        # single triangle cutting through the sphere
        ctx.particles_set([0, 1, 2, 3], [a, a, b, b], st)
        _say("edge: empty query")
        t = ctx.query_pairs(np.zeros((0, 2), np.int32))
        pr, con = ctx.fetch(t)
        assert pr.shape[0] == 0 and con.shape[0] == 0
        _say("edge: culled / touching / intersecting")
        pairs = np.array([[0, 1], [0, 2], [0, 3], [3, 0]], np.int32)
        for flags in (1, 2, 5, 6):
            t = ctx.query_pairs(pairs, flags=flags)
            pr, con = ctx.fetch(t)
            sc = synth.Scene(meshes=[(V, F), tri1], halo=np.array([0.01, 0.01]),
                             mesh_of=np.array([0, 0, 1, 1], np.int32), state=st, pairs=pairs)
            ref, rcon = oracle.static_pairs(sc)
            check_static(sc, pairs, pr, con, ref, rcon, RTOL, dense=bool(flags & 4))
            assert pr["contact"].tolist() == [0, 1, 1, 1]
            assert pr["dmin"][2] == 0.0 and pr["dmin"][3] == 0.0
        _say("edge: invalid input")
        with pytest.raises(mcd.MCDError):
            ctx.query_pairs(np.array([[0, 0]], np.int32))
        with pytest.raises(mcd.MCDError):
            ctx.query_pairs(np.array([[0, 99]], np.int32))
        # a long list is prepared in several host threads: the lowest bad pair
        # is the one named, whichever thread meets it
        big = np.tile(pairs, (1500, 1))
        bad = big.copy()
        bad[4100] = [0, 99]
        bad[5000] = [1, 1]
        with pytest.raises(mcd.MCDError, match="pair 4100"):
            ctx.query_pairs(bad)
        bad[2000] = [2, 2]
        with pytest.raises(mcd.MCDError, match="pair 2000 repeats"):
            ctx.query_pairs(bad)
        t = ctx.query_pairs(big, flags=2)
        pr, con = ctx.fetch(t)
        assert pr["contact"].tolist() == [0, 1, 1, 1] * 1500
        with pytest.raises(mcd.MCDError):
            ctx.mesh_load(np.zeros((3, 3)), np.array([[0, 1, 2]], np.int32), 0.01)
        with pytest.raises(mcd.MCDError):
            ctx.mesh_load(V, F + 1000, 0.01)
        # non-finite or negative inputs are rejected on the host, before any launch
        Vn = V.copy()
        Vn[3, 1] = np.nan
        with pytest.raises(mcd.MCDError):
            ctx.mesh_load(Vn, F, 0.01)
        for eps in (-0.01, np.inf):
            with pytest.raises(mcd.MCDError):
                ctx.mesh_load(V, F, eps)
        sn = st[:1].copy()
        sn[0, 7] = np.inf                 # velocity
        with pytest.raises(mcd.MCDError):
            ctx.particles_set([0], [a], sn)
        for dt in (-0.1, np.nan):
            with pytest.raises(mcd.MCDError):
                ctx.query_pairs(pairs, dt=dt)
        # the context is still usable after rejected calls
        t = ctx.query_pairs(pairs, flags=2)
        pr, con = ctx.fetch(t)
        assert pr["contact"].tolist() == [0, 1, 1, 1]


def test_determinism_and_overflow_regrow(mcd):
    sc = _ragged_scene(2)
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        _say("determinism")
        a = _run(mcd, ctx, sc, sc.pairs, 2)
        b = _run(mcd, ctx, sc, sc.pairs, 2)
        assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()
    with mcd.Context(contact_cap=8) as ctx:
        ctx.load_scene(sc)
        _say("overflow regrow")
        c = _run(mcd, ctx, sc, sc.pairs, 2)
        assert c[2]["retries"] >= 1
        assert c[0].tobytes() == a[0].tobytes() and c[1].tobytes() == a[1].tobytes()


def test_device_pair_list(mcd):
    """Pair lists in device memory: read on the device after the work queued
    on the caller's stream (the list is written there by an asynchronous copy
    right before the call), the pair sources gathered from the device
    particle and mesh tables. Results equal the host-list query's bit for bit
    (static, several modes, and time stamps); a particles_set after the
    submission does not change the query's result; bad lists fail the ticket."""
    import torch
    sc = synth.cfg2_scene(run=3, n=300, phi=0.45, subdivs=(1, 2))
    ref, rcon = oracle.static_pairs(sc, pairs=sc.pairs[:40])
    stream = torch.cuda.current_stream()
    with mcd.Context(stream=stream.cuda_stream) as ctx:
        ids = ctx.load_scene(sc)
        for flags in (2, 1, 2 | 4):
            _say("device pair list", flags)
            host = _run(mcd, ctx, sc, sc.pairs, flags)
            pin = torch.from_numpy(sc.pairs.copy()).pin_memory()
            d = torch.empty_like(pin, device="cuda")
            d.copy_(pin, non_blocking=True)      # queued on the caller's stream
            t = ctx.query_pairs_dev(d.data_ptr(), d.shape[0], flags=flags, stream=stream.cuda_stream)
            pr, con, pp = ctx.fetch(t, with_pairs=True)
            ctx.release(t)
            assert np.array_equal(pp, sc.pairs)
            assert pr.tobytes() == host[0].tobytes() and con.tobytes() == host[1].tobytes()
        check_static(sc, sc.pairs[:40], pr[:40], con[con["pair"] < 40], ref, rcon, RTOL)
        # a state update right after the submission waits for the query
        d = torch.from_numpy(sc.pairs.copy()).cuda()
        base = _run(mcd, ctx, sc, sc.pairs, 2)
        t = ctx.query_pairs_dev(d.data_ptr(), d.shape[0], flags=2)
        moved = sc.state.copy()
        moved[:, :3] += 0.05
        moved[:, 3:7] = synth.random_quaternions(sc.n_particles, np.random.default_rng(3))
        ctx.particles_set(np.arange(sc.n_particles, dtype=np.int32), ids[sc.mesh_of], moved)
        pr, con = ctx.fetch(t)
        assert pr.tobytes() == base[0].tobytes() and con.tobytes() == base[1].tobytes()
        ctx.particles_set(np.arange(sc.n_particles, dtype=np.int32), ids[sc.mesh_of], sc.state)
        # time stamps from a device list
        mv = synth.cfg4_scene(run=3, n=200, subdivs=(1,), proxy_r=1.0)
        with mcd.Context() as c2:
            c2.load_scene(mv)
            hp, hc = c2.fetch(c2.query_pairs(mv.pairs, dt=mv.dt))
            dm = torch.from_numpy(mv.pairs.copy()).cuda()
            torch.cuda.synchronize()
            t = c2.query_pairs_dev(dm.data_ptr(), dm.shape[0], dt=mv.dt)
            dp_, dc_ = c2.fetch(t)
            assert (hp["status"] == mcd.COLLIDES).any()
            assert dp_.tobytes() == hp.tobytes() and dc_.tobytes() == hc.tobytes()
        # bad lists: unknown id, repeated particle; the context stays usable
        for bad, code in (([[0, 5000]], -3), ([[7, 7]], -1)):
            db = torch.tensor(bad, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            t = ctx.query_pairs_dev(db.data_ptr(), 1, flags=2)
            with pytest.raises(mcd.MCDError) as e:
                ctx.fetch(t)
            assert e.value.code == code
        empty = ctx.query_pairs_dev(0, 0, flags=2)
        pr, con = ctx.fetch(empty)
        assert pr.shape[0] == 0 and con.shape[0] == 0
        again = _run(mcd, ctx, sc, sc.pairs, 2)
        assert again[0].tobytes() == base[0].tobytes()


def test_device_pair_list_regrow(mcd):
    """A device list whose tile pairs exceed the first estimate (64 per pair):
    the gather counts them on the device, the query reruns with larger
    buffers, and the result equals the host list's."""
    import torch
    V, F = synth.icosphere(4)      # 5,120 triangles: 80 x 80 tile pairs per pair
    rng = np.random.default_rng(21)
    n = 6
    st = np.zeros((2 * n, 13))
    st[:, 3:7] = synth.random_quaternions(2 * n, rng)
    for p in range(n):
        st[2 * p, :3] = [8.0 * p, 0, 0]
        st[2 * p + 1, :3] = [8.0 * p + 2.0 + 0.002 * p, 0, 0]
    pairs = np.stack([np.arange(0, 2 * n, 2), np.arange(1, 2 * n, 2)], 1).astype(np.int32)
    sc = synth.Scene(meshes=[(V, F)], halo=np.array([0.005]), mesh_of=np.zeros(2 * n, np.int32),
                     state=st, pairs=pairs)
    # the device list first, on a fresh context whose buffers have not grown
    with mcd.Context(streams=1) as ctx:
        ctx.load_scene(sc)
        d = torch.from_numpy(pairs.copy()).cuda()
        torch.cuda.synchronize()
        _say("device pair list regrow")
        t = ctx.query_pairs_dev(d.data_ptr(), n, flags=2)
        pr, con = ctx.fetch(t)
        assert ctx.stats(t)["retries"] >= 1
        assert ctx.stats(t)["tile_pairs_total"] == n * 80 * 80
        host = _run(mcd, ctx, sc, pairs, 2)
    assert pr.tobytes() == host[0].tobytes() and con.tobytes() == host[1].tobytes()


@pytest.fixture(scope="module")
def cfg2():
    return synth.cfg2_scene(run=0)


def _sample_pairs(sc, ref_contact_pairs, k, rng, max_tri2=1280 * 1280, n_large=3):
    """k seeded random pairs of at most max_tri2 triangle pairs, the first six
    pairs in contact, and n_large pairs with the largest meshes (one
    5,120 x 5,120 pair when there is one, then 5,120 x 1,280 pairs), so the
    biggest tiles of the packing are compared at full size too."""
    nt = sc.tri_counts()[sc.mesh_of]
    na, nb = nt[sc.pairs[:, 0]], nt[sc.pairs[:, 1]]
    small = np.where(na * nb <= max_tri2)[0]
    pick = set(rng.choice(small, size=min(k, small.size), replace=False).tolist())
    pick |= set(ref_contact_pairs[:6])
    big = np.where((na == 5120) & (nb == 5120))[0]
    mid = np.where(np.maximum(na, nb) == 5120)[0]
    mid = mid[np.minimum(na[mid], nb[mid]) <= 1280]
    large = list(rng.choice(big, size=min(1, big.size), replace=False)) if big.size else []
    if mid.size:
        large += list(rng.choice(mid, size=min(n_large - len(large), mid.size), replace=False))
    pick |= {int(x) for x in large}
    return np.array(sorted(pick))


@pytest.mark.parametrize("flags", [2, 1, 2 | 4], ids=["mixed", "fp64", "mixed-dense"])
def test_cfg2_full_size_sampled(mcd, cfg2, flags):
    """The benchmark's workloads at full size (2,000 particles, all candidate
    pairs in one query; the dense one evaluates every triangle pair and reports
    every pair's exact minimum); the oracle recomputes a sample of pairs."""
    sc = cfg2
    dense = bool(flags & 4)
    _say("cfg2 full", "flags", flags, "pairs", sc.pairs.shape[0])
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        pr, con, st = _run(mcd, ctx, sc, sc.pairs, flags)
    if dense:
        assert st["tile_pairs_kept"] == st["tile_pairs_total"]
        assert st["tri_pairs_evaluated"] == st["tri_pairs_covered"]
        assert np.all(np.isfinite(pr["dmin"]))
    else:
        assert st["tile_pairs_kept"] < st["tile_pairs_total"]
    # every record of the full list in (pair, tri_a, tri_b) order, including
    # the pairs with more than 64 contacts (the LDS sort of long segments)
    assert_contact_order(con)
    seg = np.bincount(con["pair"], minlength=sc.pairs.shape[0])
    _say("largest contact segment", int(seg.max()), "pairs above 64", int((seg > 64).sum()))
    assert seg.max() > 64
    rng = np.random.default_rng(77)
    touching = np.where(pr["contact"] == 1)[0]
    idx = _sample_pairs(sc, touching.tolist(), 10, rng)
    nt = sc.tri_counts()[sc.mesh_of]
    assert (np.maximum(nt[sc.pairs[idx, 0]], nt[sc.pairs[idx, 1]]) == 5120).sum() >= 3
    sub = sc.pairs[idx]
    ref, rcon = oracle.static_pairs(sc, pairs=sub)
    # restrict GPU results to the sample and renumber
    pos = {int(p): k for k, p in enumerate(idx)}
    sel = np.array([c for c in con if int(c["pair"]) in pos], dtype=con.dtype)
    for c in sel:
        c["pair"] = pos[int(c["pair"])]
    check_static(sc, sub, pr[idx], sel, ref, rcon, RTOL, dense=dense)


@pytest.mark.parametrize("flags", [2, 1], ids=["mixed", "fp64"])
def test_uneven_pair_queries_batched(mcd, flags):
    """Pairs of UV spheres of 20-5,120 triangles (ragged and single tiles),
    each submitted as its own query; the scheduler runs them as batches on
    two streams. Every query's result is checked against the oracle."""
    sc = synth.cfg3_scene(run=1, n_pairs=64)
    _say("uneven queries", flags, sc.pairs.shape[0])
    with mcd.Context(streams=2) as ctx:
        ctx.load_scene(sc)
        tickets = [ctx.query_pairs(sc.pairs[i:i + 1], flags=flags) for i in range(sc.pairs.shape[0])]
        res = [ctx.fetch(t) for t in tickets]
        batched = max(ctx.stats(t)["batch_queries"] for t in tickets)
    ref, rcon = oracle.static_pairs(sc)
    assert ref["contact"].sum() >= 5 and (~ref["contact"].astype(bool)).sum() >= 5
    pr = np.concatenate([r[0] for r in res])
    con = []
    for i, (_, c) in enumerate(res):
        c = c.copy()
        c["pair"] = i
        con.append(c)
    con = np.concatenate(con)
    check_static(sc, sc.pairs, pr, con, ref, rcon, RTOL, dense=False)
    assert batched > 1


def _marginal_scene(seed=0):
    """Pairs of one-triangle meshes: A is a right triangle of leg s, B a thin
    triangle with an edge crossing A's plane at a point a relative distance t
    inside (t < 0) or outside (t > 0) A's hypotenuse, or near a vertex; both
    placed far from the origin and rotated together. The halo is tiny, so
    contact means intersection (or a gap below 2e-9)."""
    rng = np.random.default_rng(9100 + seed)
    ts = [-1e-3, -1e-5, -1e-7, 1e-7, 1e-5, 1e-3]
    meshes, states, pairs = [], [], []
    for t in ts:
        for where in ("edge", "vertex"):
            for _ in range(3):
                s = 10.0 ** rng.uniform(-1, 0.5)
                A = np.array([[0, 0, 0], [s, 0, 0], [0, s, 0.0]])
                if where == "edge":
                    c = np.array([0.5 * s, 0.5 * s]) * (1 + t)
                else:
                    c = np.array([s, 0.0]) + np.array([t, t * 0.3]) * s * np.sign(t) * -1
                h = 0.2 * s
                side = rng.normal(size=2)
                side = 0.1 * s * side / np.linalg.norm(side)
                B = np.array([[c[0], c[1], -h], [c[0], c[1], h], [c[0] + side[0], c[1] + side[1], 0.3 * h]])
                F = np.array([[0, 1, 2]], np.int32)
                q = synth.random_quaternions(1, rng)[0]
                x = rng.uniform(-50, 50, size=3)
                for V in (A, B):
                    meshes.append((V, F))
                    st = np.zeros(13)
                    st[:3] = x
                    st[3:7] = q
                    states.append(st)
                pairs.append([len(states) - 2, len(states) - 1])
    n = len(states)
    return synth.Scene(meshes=meshes, halo=np.full(n, 1e-9), mesh_of=np.arange(n, dtype=np.int32),
                       state=np.array(states), pairs=np.array(pairs, np.int32))


@pytest.mark.parametrize("seed", [0, 1])
def test_marginal_intersections(mcd, seed):
    """The FP32 filter's intersection test must pass every FP64 intersection:
    edges crossing a triangle 1e-7 (relative) inside its boundary, at
    coordinates up to 50 where FP32 resolves only about 4e-6. Contact flags
    and sets are compared exactly and distances to 1e-6 relative; closest
    points at |x| ~ 50 carry FP64 rounding of about 1e-14 |x| whatever the
    (here 2e-9) threshold, so their tolerance is set by that scale."""
    sc = _marginal_scene(seed)
    ref, rcon = oracle.static_pairs(sc)
    assert 0 < ref["contact"].sum() < sc.pairs.shape[0]
    _say("marginal intersections", seed)
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for flags in (2, 1, 6):
            pr, con, st = _run(mcd, ctx, sc, sc.pairs, flags)
            assert pr["contact"].tolist() == ref["contact"].tolist(), flags
            check_static(sc, sc.pairs, pr, con, ref, rcon, RTOL, dense=bool(flags & 4), rtol_pts=0.1)


def test_largest_meshes(mcd):
    """Two UV spheres of 65,024 triangles each (the largest mesh is 65,535),
    0.0005 apart, in random rotations: triangle ids use all 16 bits. The
    oracle checks the contact region (triangles with a vertex within 0.2 of
    the touching point cover every pair within the halo)."""
    V, F = synth.uv_sphere(65000)
    assert F.shape[0] == 65024
    rng = np.random.default_rng(77)
    q = synth.random_quaternions(2, rng)
    g, eps = 0.0005, 0.002
    st = np.zeros((2, 13))
    st[:, 3:7] = q
    st[1, :3] = [2.0 + g, 0, 0]
    sc = synth.Scene(meshes=[(V, F)], halo=np.array([eps]), mesh_of=np.zeros(2, np.int32), state=st,
                     pairs=np.array([[0, 1]], np.int32))
    _say("largest meshes")
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        pr, con, stats = _run(mcd, ctx, sc, sc.pairs, 2)
    assert con.shape[0] > 10
    # oracle on the triangles near the touching point (world x within 0.2 of it)
    Wa = oracle.world_tris(V, F, st[0]).reshape(-1, 3, 3)
    Wb = oracle.world_tris(V, F, st[1]).reshape(-1, 3, 3)
    sa = np.where(Wa[:, :, 0].max(1) > 0.8)[0]
    sb = np.where(Wb[:, :, 0].min(1) < 1.2 + g)[0]
    sub = synth.Scene(meshes=[(V, F[sa]), (V, F[sb])], halo=np.array([eps, eps]),
                      mesh_of=np.array([0, 1], np.int32), state=st, pairs=sc.pairs)
    ref, rcon = oracle.static_pairs(sub)
    exp = {(0, int(sa[c["tri_a"]]), int(sb[c["tri_b"]])) for c in rcon}
    got = contact_set(con)
    assert got == exp, (len(got), len(exp), sorted(got ^ exp)[:8])
    assert abs(pr["dmin"][0] - ref["d"][0]) <= RTOL * max(ref["d"][0], 2 * eps)
    assert (int(pr["tri_a"][0]), int(pr["tri_b"][0])) == (int(sa[ref["tri_a"][0]]), int(sb[ref["tri_b"][0]]))


def test_coincident_particles(mcd):
    """Two particles with the same mesh and the same state: every pair of
    coincident or adjacent triangles is in contact (coplanar overlap and
    shared edges), compared with the oracle in every mode."""
    V, F = synth.icosphere(1)
    rng = np.random.default_rng(5)
    st = np.zeros((2, 13))
    st[:, 3:7] = synth.random_quaternions(1, rng)[0]
    st[:, :3] = [3.0, -2.0, 1.0]
    sc = synth.Scene(meshes=[(V, F)], halo=np.array([0.01]), mesh_of=np.zeros(2, np.int32), state=st,
                     pairs=np.array([[0, 1]], np.int32))
    ref, rcon = oracle.static_pairs(sc)
    assert ref["d"][0] == 0.0 and rcon.shape[0] >= F.shape[0]
    _say("coincident particles")
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for flags in (2, 1, 6, 5):
            pr, con, _ = _run(mcd, ctx, sc, sc.pairs, flags)
            check_static(sc, sc.pairs, pr, con, ref, rcon, RTOL, dense=bool(flags & 4))


@pytest.mark.gpu
def test_contacts_beyond_segment_capacity(mcd):
    """A pair with more contacts than one per-pair LDS segment holds (two
    coincident 1,280-triangle spheres): the contact records are then ordered
    by the device-wide radix sort instead; the set and order must still
    equal the oracle's."""
    V, F = synth.icosphere(3)
    rng = np.random.default_rng(11)
    st = np.zeros((3, 13))
    st[:, 3:7] = synth.random_quaternions(1, rng)[0]
    st[:2, :3] = [1.0, 2.0, -1.0]
    st[2, :3] = [1.0, 2.0, 1.0]      # a third particle touching the first: a second, small segment
    sc = synth.Scene(meshes=[(V, F)], halo=np.array([0.01]), mesh_of=np.zeros(3, np.int32), state=st,
                     pairs=np.array([[0, 1], [0, 2]], np.int32))
    ref, rcon = oracle.static_pairs(sc)
    assert int((rcon["pair"] == 0).sum()) > 4096
    _say("contacts beyond the segment capacity")
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for flags in (2, 1):
            pr, con, _ = _run(mcd, ctx, sc, sc.pairs, flags)
            check_static(sc, sc.pairs, pr, con, ref, rcon, RTOL, dense=False)


def test_cfg3_full_batch_sampled(mcd):
    """The full 4,096-query batch of uneven UV-sphere pairs (20-5,120
    triangles), every pair its own query, batched by the scheduler on two
    streams; every result is self-consistent (flag = dmin within the halo,
    records in order and within the halo) and a seeded sample of 48 queries,
    including the largest meshes, is compared with the oracle."""
    sc = synth.cfg3_scene(run=0)
    n = sc.pairs.shape[0]
    assert n == 4096
    _say("cfg3 full batch", n)
    with mcd.Context(streams=2) as ctx:
        ctx.load_scene(sc)
        tickets = [ctx.query_pairs(sc.pairs[i:i + 1]) for i in range(n)]
        res = [ctx.fetch(t) for t in tickets]
        batched = max(ctx.stats(t)["batch_queries"] for t in tickets)
        for t in tickets:
            ctx.release(t)
    assert batched > 1
    delta = 2 * 0.005
    for pr, con in res:
        assert pr.shape[0] == 1
        assert pr["contact"][0] == (1 if np.isfinite(pr["dmin"][0]) and pr["dmin"][0] <= delta else 0)
        assert con.shape[0] == 0 or (pr["contact"][0] == 1 and np.all(con["d"] <= delta))
        assert_contact_order(con)
    nt = sc.tri_counts()[sc.mesh_of]
    cost = nt[sc.pairs[:, 0]] * nt[sc.pairs[:, 1]]
    rng = np.random.default_rng(33)
    pick = set(rng.choice(n, size=44, replace=False).tolist())
    pick |= set(np.argsort(cost)[-4:].tolist())
    idx = np.array(sorted(pick))
    ref, rcon = oracle.static_pairs(sc, pairs=sc.pairs[idx])
    pr = np.concatenate([res[i][0] for i in idx])
    con = []
    for k, i in enumerate(idx):
        c = res[i][1].copy()
        c["pair"] = k
        con.append(c)
    con = np.concatenate(con)
    check_static(sc, sc.pairs[idx], pr, con, ref, rcon, RTOL, dense=False)


def test_bounding_radius_packing(mcd):
    """The 2,000-particle packing on the bounding radius 1.1 (no two bounding
    spheres overlap): no triangle pair comes within the halo, in the culled
    and in the dense query, and the dense query's exact minima of a sample
    of pairs (including the largest meshes) equal the oracle's."""
    sc = synth.cfg2_scene(run=0, pack_r=1.1)
    _say("bounding-radius packing", sc.pairs.shape[0])
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        pr, con, st = _run(mcd, ctx, sc, sc.pairs, 2)
        assert con.shape[0] == 0 and not pr["contact"].any()
        prd, cond, _ = _run(mcd, ctx, sc, sc.pairs, 2 | 4)
    assert cond.shape[0] == 0 and np.all(np.isfinite(prd["dmin"]))
    assert prd["dmin"].min() > 0.01
    rng = np.random.default_rng(78)
    idx = _sample_pairs(sc, [], 10, rng)
    ref, rcon = oracle.static_pairs(sc, pairs=sc.pairs[idx])
    check_static(sc, sc.pairs[idx], prd[idx], cond[:0], ref, rcon, RTOL, dense=True)
