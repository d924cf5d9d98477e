"""Particle interaction (section 6) on the device, mcd_impulses, against the
oracle's Picard solve on the fused contacts of a static packing whose
particles carry random velocities."""

import numpy as np
import pytest

import oracle
import synth

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
def setup(mcd):
    """Fused contacts of 200 candidate pairs of the static packing, particles
    with random velocities; the oracle's mass properties of every mesh."""
    import torch
    sc = synth.cfg2_scene(run=0)
    rng = np.random.default_rng(11)
    states = sc.state.copy()
    states[:, 7:10] = rng.normal(size=(sc.n_particles, 3))
    states[:, 10:13] = rng.normal(scale=0.5, size=(sc.n_particles, 3))
    ctx = mcd.Context(stream=torch.cuda.current_stream().cuda_stream)
    ids = ctx.load_scene(sc)
    ctx.particles_set(np.arange(sc.n_particles, dtype=np.int32), ids[sc.mesh_of], states)
    t = ctx.query_pairs(sc.pairs[:200], flags=mcd.Q_MIXED | mcd.Q_FUSE)
    pr, con, pp = ctx.fetch(t, with_pairs=True)
    ctx.release(t)
    con, pp = con.copy(), pp.copy()
    assert con.shape[0] > 100
    props = {}
    for m in np.unique(sc.mesh_of):
        props[int(m)] = oracle.mass_properties(*sc.meshes[m])
    yield ctx, sc, states, con, pp[con["pair"]], props
    ctx.close()


def _oracle(sc, states, con, pid_pairs, props, **kw):
    flat = pid_pairs.reshape(-1)
    _, first = np.unique(flat, return_index=True)
    pids = flat[np.sort(first)]
    local = {int(p): i for i, p in enumerate(pids)}
    ab = np.array([[local[int(a)], local[int(b)]] for a, b in pid_pairs])
    mass = np.array([props[int(sc.mesh_of[p])][0] for p in pids])
    com = np.array([props[int(sc.mesh_of[p])][1] for p in pids])
    inertia = np.array([props[int(sc.mesh_of[p])][2] for p in pids])
    imp, vel, it, col = oracle.impulses(mass, com, inertia, states[pids], ab, con["pa"], con["pb"], **kw)
    return imp, pids, vel, it


@pytest.mark.parametrize("kw", [dict(), dict(restitution=0.5), dict(friction=0.4), dict(restitution=0.2, friction=1.0,
                                                                                        relax=0.7)],
                         ids=["plain", "restitution", "friction", "all"])
def test_fixed_sweeps_match_the_oracle(setup, kw):
    ctx, sc, states, con, pid_pairs, props = setup
    _say("impulses, 25 sweeps", con.shape[0], kw)
    imp, pids, vel, sw = ctx.impulses(pid_pairs, con, tol=1e-300, max_iter=25, **kw)
    oimp, opids, ovel, oit = _oracle(sc, states, con, pid_pairs, props, tol=1e-300, max_iter=25, **kw)
    assert sw == oit == 25
    assert np.array_equal(pids, opids)
    scale = np.abs(oimp).max()
    assert np.allclose(imp, oimp, rtol=1e-9, atol=1e-10 * scale)
    assert np.allclose(vel, ovel, rtol=1e-9, atol=1e-10 * np.abs(ovel).max())


def test_converged_solve(setup):
    ctx, sc, states, con, pid_pairs, props = setup
    _say("impulses, converged", con.shape[0])
    imp, pids, vel, sw = ctx.impulses(pid_pairs, con, friction=0.3, max_iter=100000)
    oimp, opids, ovel, oit = _oracle(sc, states, con, pid_pairs, props, friction=0.3, max_iter=100000)
    assert sw < 100000 and abs(sw - oit) <= 1
    assert np.all(imp[:, 0] >= 0.0)
    assert np.all(np.linalg.norm(imp[:, 1:], axis=1) <= 0.3 * imp[:, 0] * (1 + 1e-12) + 1e-300)
    # both stop within the relative tolerance of the same solution
    assert np.allclose(vel, ovel, rtol=0, atol=1e-2 * np.abs(ovel).max())


def test_errors_and_empty_input(setup, mcd):
    ctx, sc, states, con, pid_pairs, props = setup
    _say("impulses, errors")
    imp, pids, vel, sw = ctx.impulses(np.zeros((0, 2), np.int32), con[:0])
    assert imp.shape == (0, 4) and pids.shape == (0,) and sw == 0
    bad = pid_pairs[:4].copy()
    bad[1, 1] = bad[1, 0]                               # a particle with itself
    with pytest.raises(mcd.MCDError):
        ctx.impulses(bad, con[:4])
    bad = pid_pairs[:4].copy()
    bad[2, 0] = 10 ** 7                                 # unknown id
    with pytest.raises(mcd.MCDError):
        ctx.impulses(bad, con[:4])
    for kw in (dict(restitution=1.5), dict(friction=-1.0), dict(relax=2.0), dict(max_iter=-3)):
        with pytest.raises(mcd.MCDError):
            ctx.impulses(pid_pairs[:4], con[:4], **kw)


def test_many_clusters_match_the_oracle(mcd):
    """Clusters sharing no particle (a particle with its neighbours), one
    device workgroup each, converged on their own: against the oracle."""
    import torch
    sc = synth.cfg2_scene(run=0)
    rng = np.random.default_rng(21)
    owner = np.full(sc.n_particles, -1)
    nbr = [[] for _ in range(sc.n_particles)]
    for a, b in sc.pairs:
        nbr[a].append(b)
        nbr[b].append(a)
    k = 0
    for s in rng.permutation(sc.n_particles)[:150]:
        if owner[s] >= 0:
            continue
        owner[s] = k
        for b in nbr[s]:
            if owner[b] < 0:
                owner[b] = k
        k += 1
    keep = (owner[sc.pairs[:, 0]] >= 0) & (owner[sc.pairs[:, 0]] == owner[sc.pairs[:, 1]])
    pairs = sc.pairs[keep]
    states = sc.state.copy()
    states[:, 7:10] = rng.normal(size=(sc.n_particles, 3))
    states[:, 10:13] = rng.normal(scale=0.5, size=(sc.n_particles, 3))
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ids = ctx.load_scene(sc)
        ctx.particles_set(np.arange(sc.n_particles, dtype=np.int32), ids[sc.mesh_of], states)
        t = ctx.query_pairs(pairs, flags=mcd.Q_MIXED | mcd.Q_FUSE)
        _, con, pp = ctx.fetch(t, with_pairs=True)
        con, pid_pairs = con.copy(), pp[con["pair"]].copy()
        ctx.release(t)
        _say("impulses, clusters", k, "contacts", con.shape[0])
        props = {int(m): oracle.mass_properties(*sc.meshes[m]) for m in np.unique(sc.mesh_of)}
        for kw in (dict(tol=1e-300, max_iter=40), dict(friction=0.5, restitution=0.3, tol=1e-300, max_iter=40)):
            imp, pids, vel, sw = ctx.impulses(pid_pairs, con, **kw)
            oimp, opids, ovel, oit = _oracle(sc, states, con, pid_pairs, props, **kw)
            assert sw == oit == 40 and np.array_equal(pids, opids)
            assert np.allclose(imp, oimp, rtol=1e-9, atol=1e-10 * np.abs(oimp).max())
            assert np.allclose(vel, ovel, rtol=1e-9, atol=1e-10 * np.abs(ovel).max())
        imp, pids, vel, sw = ctx.impulses(pid_pairs, con, max_iter=20000)
        oimp, opids, ovel, oit = _oracle(sc, states, con, pid_pairs, props, max_iter=20000)
        assert sw < 20000 and abs(sw - oit) <= 1
        assert np.allclose(vel, ovel, rtol=0, atol=1e-2 * np.abs(ovel).max())
