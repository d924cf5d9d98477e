"""Pins of the oracle's narrowing time stamp (section 5, "Collision time
detection": analytic vertex-triangle test, edge-edge distances sampled at
the start, middle and end of the span, the span narrowed to the earliest
contact until nothing earlier is found; translation only)."""

import numpy as np

import oracle
import synth

DELTA = 0.02


def _pair_scene(VA, FA, VB, FB, xa, xb, va, vb, wa=(0, 0, 0), wb=(0, 0, 0)):
    st = np.zeros((2, 13))
    st[:, 3] = 1.0
    st[0, :3], st[1, :3] = xa, xb
    st[0, 7:10], st[1, 7:10] = va, vb
    st[0, 10:13], st[1, 10:13] = wa, wb
    return synth.Scene(meshes=[(np.asarray(VA, float), np.asarray(FA, np.int32)),
                               (np.asarray(VB, float), np.asarray(FB, np.int32))],
                       halo=np.array([DELTA / 2, DELTA / 2]), mesh_of=np.array([0, 1], np.int32),
                       state=st, pairs=np.array([[0, 1]], np.int32))


BIG = ([[-5, -5, 0], [5, -5, 0], [0, 5, 0]], [[0, 1, 2]])
# a small triangle whose lowest vertex points down
SPIKE = ([[0, 0, 0], [-0.3, 0.2, 0.6], [0.3, 0.2, 0.6]], [[0, 1, 2]])


def test_vertex_onto_face_closed_forms():
    h, v = 0.3, 2.0
    # passes the plane inside the span: the time is the plane crossing h / v
    sc = _pair_scene(*BIG, *SPIKE, [0, 0, 0], [0, 0, h], [0, 0, 0], [0, 0, -v])
    pr, con, rounds = oracle.narrow_pairs(sc, dt=0.5)
    assert pr["status"][0] == 2 and abs(pr["toi"][0] - h / v) <= 1e-15 and con.shape[0] >= 1
    # stops inside the halo before the plane: contact only at the end of the span
    dt = (h - 0.5 * DELTA) / v
    pr, _, _ = oracle.narrow_pairs(sc, dt=dt)
    assert pr["status"][0] == 2 and pr["toi"][0] == dt
    # stops short of the halo: no contact
    pr, _, _ = oracle.narrow_pairs(sc, dt=(h - 2 * DELTA) / v)
    assert pr["status"][0] == 0 and np.isinf(pr["toi"][0])
    # in contact at the start
    sc0 = _pair_scene(*BIG, *SPIKE, [0, 0, 0], [0, 0, 0.5 * DELTA], [0, 0, 0], [0, 0, -v])
    pr, _, _ = oracle.narrow_pairs(sc0, dt=0.5)
    assert pr["status"][0] == 1 and pr["toi"][0] == 0.0


def test_edge_edge_dyadic_closed_form():
    """Two crossed edges approaching at speed u (gap g(t) = g0 - u t, no
    vertex feature within reach): each round halves the span while the
    middle sample is in contact, so the time is the smallest dt / 2^k that
    is not earlier than the true contact time (g0 - delta) / u."""
    A = ([[-2, 0, 0], [2, 0, 0], [0.7, -1.0, 0]], [[0, 1, 2]])
    B = ([[0, -2, 0], [0, 2, 0], [-0.7, 0, 1.0]], [[0, 1, 2]])
    g0, u, dt = 0.5, 1.0, 1.0
    sc = _pair_scene(*A, *B, [0, 0, 0], [0, 0, g0], [0, 0, 0], [0, 0, -u])
    pr, _, rounds = oracle.narrow_pairs(sc, dt=dt)
    t_true = (g0 - DELTA) / u
    k = 0
    while dt / 2 ** (k + 1) >= t_true:
        k += 1
    assert pr["status"][0] == 2 and pr["toi"][0] == dt / 2 ** k
    assert rounds[0] == k + 1


def test_invariances_and_symmetry():
    """A common velocity changes nothing, nor does spin (rotation is
    neglected); swapping the particles gives the same time."""
    rng = np.random.default_rng(3)
    V, F = synth.icosphere(1)
    for run in range(4):
        q = synth.random_quaternions(2, rng)
        u = synth.random_unit_vectors(1, rng)[0]
        sc = _pair_scene(V, F, V, F, [0, 0, 0], 2.15 * u, [0, 0, 0], -1.5 * u + 0.2 * rng.normal(size=3))
        sc.state[:, 3:7] = q
        base, _, _ = oracle.narrow_pairs(sc, dt=0.2)
        moved = synth.Scene(**{**sc.__dict__, "state": sc.state.copy()})
        moved.state[:, 7:10] += rng.normal(size=3)
        moved.state[:, 10:13] = rng.normal(size=(2, 3)) * 5
        pr, _, _ = oracle.narrow_pairs(moved, dt=0.2)
        assert pr["status"][0] == base["status"][0]
        assert abs(pr["toi"][0] - base["toi"][0]) <= 1e-12 or pr["toi"][0] == base["toi"][0]
        sw, _, _ = oracle.narrow_pairs(sc, dt=0.2, pairs=np.array([[1, 0]], np.int32))
        assert sw["status"][0] == base["status"][0]
        assert sw["toi"][0] == base["toi"][0] or abs(sw["toi"][0] - base["toi"][0]) <= 1e-12


def test_never_before_the_exact_time():
    """Translation only: whenever the narrowing reports a time, the two
    particles are in contact then (the distance at that time is within the
    threshold), so the exact first contact time of the sampler is not later."""
    rng = np.random.default_rng(9)
    V, F = synth.icosphere(1)
    n_hit = 0
    for run in range(12):
        Va = synth.perturb_radial(V, rng, 0.1)
        Vb = synth.perturb_radial(V, rng, 0.1)
        q = synth.random_quaternions(2, rng)
        u = synth.random_unit_vectors(1, rng)[0]
        sc = _pair_scene(Va, F, Vb, F, [0, 0, 0], rng.uniform(2.05, 2.3) * u, [0, 0, 0],
                         -rng.uniform(0.5, 3.0) * u + 0.3 * rng.normal(size=3))
        sc.state[:, 3:7] = q
        dt = 0.3
        nar, ncon, _ = oracle.narrow_pairs(sc, dt=dt)
        ex, _, _ = oracle.toi_pairs(sc, dt, S=64)
        if nar["status"][0] == 0:
            continue
        n_hit += 1
        assert ex["status"][0] > 0
        assert ex["toi"][0] <= nar["toi"][0] + 1e-6 * dt
        # the reported pair is within the threshold at the reported time
        assert nar["d"][0] <= DELTA * (1 + 1e-12) and ncon.shape[0] >= 1
    assert n_hit >= 8
