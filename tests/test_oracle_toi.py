"""Pins for the oracle's rigid motion and collision time stamps.

Expected values: scipy's rotation routines for the pose, closed-form first
contact times (translation along a vertex axis; a spinning vertex reaching a
plane), Galilean invariance, and brute-force dense sampling in time.
"""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth


def _state(x, q_wxyz, v=(0, 0, 0), w=(0, 0, 0)):
    return np.concatenate([x, q_wxyz, v, w]).astype(np.float64)


def test_pose_matches_scipy():
    rng = np.random.default_rng(31)
    for _ in range(200):
        R0 = Rotation.random(random_state=rng)
        q = R0.as_quat()
        x0, v, w = rng.normal(size=3), rng.normal(size=3), rng.normal(size=3) * 4
        t = rng.uniform(-1, 1)
        R, x = oracle.pose(_state(x0, [q[3], *q[:3]], v, w), t)
        Rref = (Rotation.from_rotvec(w * t) * R0).as_matrix()   # spin about a world axis
        assert np.allclose(R, Rref, atol=1e-13)
        assert np.allclose(x, x0 + v * t, atol=1e-14)
    # an unnormalised quaternion is normalised
    R, _ = oracle.pose(_state(np.zeros(3), [2.0, 0, 0, 0]), 0.0)
    assert np.allclose(R, np.eye(3))


def _scene(meshA, meshB, sa, sb, eps):
    return synth.pair_test_scene(meshA, meshB, sa, sb, eps)


def test_translation_along_vertex_axis():
    """Two icosahedra approach along a vertex axis: d(t) = sep - v t - 2, so the
    first contact is t = (sep - 2 - delta) / v; the search returns the end of
    a bracket of width <= tol that contains it."""
    V, F = synth.icosphere(0)
    u = V[0] / np.linalg.norm(V[0])
    eps, sep, vr, dt = 0.01, 2.3, 1.7, 0.25
    delta = 2 * eps
    sa = _state(np.zeros(3), [1, 0, 0, 0])
    sb = _state(sep * u, [1, 0, 0, 0], v=-vr * u)
    sc = _scene((V, F), (V, F), sa, sb, eps)
    pr, con, diag = oracle.toi_pairs(sc, dt, S=64, tol_rel=1e-6)
    t_true = (sep - 2 - delta) / vr
    tol = 1e-6 * dt
    assert pr["status"][0] == oracle.STATUS_COLLIDES
    assert -1e-15 <= pr["toi"][0] - t_true <= tol + 1e-15
    assert pr["d"][0] <= delta
    # contact records at t*: only triangles around the two facing vertices
    assert len(con) > 0 and (con["d"] <= delta).all()
    ia = {i for i, f in enumerate(F) if 0 in f}
    assert {int(c) for c in con["tri_a"]} <= ia


@pytest.mark.parametrize("phi0,omega", [(-1.0, 2.0), (-0.7, 5.0), (-2.0, 3.0)])
def test_spinning_vertex_reaches_plane(phi0, omega):
    """A triangle with one vertex at radius 1 spins about z; a large static
    triangle lies in the plane x = c. The vertex height over the plane is
    c - cos(phi0 + omega t), so contact starts at
    t = (-arccos((c - delta)/1) - phi0) / omega."""
    c, eps = 0.95, 0.01
    delta = 2 * eps
    ca, sa_ = math.cos(phi0), math.sin(phi0)
    Rz = np.array([[ca, -sa_, 0], [sa_, ca, 0], [0, 0, 1]])
    VA = np.array([[1.0, 0, 0], [-0.1, 0.05, 0], [-0.1, -0.05, 0]]) @ Rz.T
    FA = np.array([[0, 1, 2]], np.int32)
    VB = np.array([[0, -5, -5], [0, 5, -5], [0, 0, 5.0]])
    FB = np.array([[0, 1, 2]], np.int32)
    sa = _state(np.zeros(3), [1, 0, 0, 0], w=[0, 0, omega])
    sb = _state([c, 0, 0], [1, 0, 0, 0])
    t_true = (-math.acos(c - delta) - phi0) / omega
    dt = 1.5 * t_true
    sc = _scene((VA, FA), (VB, FB), sa, sb, eps)
    pr, con, diag = oracle.toi_pairs(sc, dt, S=64, tol_rel=1e-6)
    assert pr["status"][0] == oracle.STATUS_COLLIDES
    assert -1e-15 <= pr["toi"][0] - t_true <= 1e-6 * dt + 1e-15
    # the Lipschitz constant uses the largest vertex radius about the centre
    L = omega * 1.0
    t1, _ = oracle.tri_pair_toi(VA.reshape(9), VB.reshape(9), sa, sb, delta, L, dt)
    assert t1 == pr["toi"][0]


def test_status_cases():
    V, F = synth.icosphere(0)
    u = V[0] / np.linalg.norm(V[0])
    eps = 0.01
    # overlapping halos at the start: contact at t = 0
    sc = _scene((V, F), (V, F), _state(np.zeros(3), [1, 0, 0, 0]),
                _state((2.01) * u, [1, 0, 0, 0], v=u), eps)
    pr, con, _ = oracle.toi_pairs(sc, 0.1)
    assert pr["status"][0] == oracle.STATUS_AT_START and pr["toi"][0] == 0.0
    assert len(con) > 0
    # moving apart: no contact in the step
    sc = _scene((V, F), (V, F), _state(np.zeros(3), [1, 0, 0, 0]),
                _state(2.1 * u, [1, 0, 0, 0], v=u), eps)
    pr, con, _ = oracle.toi_pairs(sc, 0.1)
    assert pr["status"][0] == oracle.STATUS_NONE and not np.isfinite(pr["toi"][0])
    assert len(con) == 0
    # approaching but too slowly to close the gap within the step
    sc = _scene((V, F), (V, F), _state(np.zeros(3), [1, 0, 0, 0]),
                _state(2.1 * u, [1, 0, 0, 0], v=-0.1 * u), eps)
    pr, con, _ = oracle.toi_pairs(sc, 0.1)
    assert pr["status"][0] == oracle.STATUS_NONE


def test_galilean_invariance():
    rng = np.random.default_rng(32)
    V, F = synth.icosphere(1)
    hits = 0
    for trial in range(6):
        qa, qb = synth.random_quaternions(2, rng)
        u = synth.random_unit_vectors(1, rng)[0]
        sa = _state(np.zeros(3), qa, v=rng.normal(size=3) * 0.2, w=rng.normal(size=3) * 3)
        sb = _state(2.08 * u, qb, v=-3 * u + rng.normal(size=3) * 0.2, w=rng.normal(size=3) * 3)
        sc = _scene((V, F), (V, F), sa, sb, 0.005)
        pr, _, _ = oracle.toi_pairs(sc, 0.1, S=32)
        vc = rng.normal(size=3) * 3
        sa2, sb2 = sa.copy(), sb.copy()
        sa2[7:10] += vc
        sb2[7:10] += vc
        sc2 = _scene((V, F), (V, F), sa2, sb2, 0.005)
        pr2, _, _ = oracle.toi_pairs(sc2, 0.1, S=32)
        assert pr["status"][0] == pr2["status"][0]
        if pr["status"][0] == oracle.STATUS_COLLIDES:
            hits += 1
            assert abs(pr["toi"][0] - pr2["toi"][0]) <= 1e-6 * 0.1 + 1e-15
    assert hits >= 2


def test_against_dense_time_sampling():
    """First contact from 4000 equidistant static queries in time versus the
    sampled/bisected search, on small meshes with rotation."""
    rng = np.random.default_rng(33)
    V, F = synth.icosphere(0)
    checked = 0
    for trial in range(12):
        qa, qb = synth.random_quaternions(2, rng)
        u = synth.random_unit_vectors(1, rng)[0]
        sa = _state(np.zeros(3), qa, v=rng.normal(size=3) * 0.3, w=rng.normal(size=3) * 4)
        sb = _state(2.2 * u, qb, v=-2 * u + rng.normal(size=3) * 0.3, w=rng.normal(size=3) * 4)
        sc = _scene((V, F), (V, F), sa, sb, 0.01)
        dt = 0.2
        pr, _, _ = oracle.toi_pairs(sc, dt, S=16)
        n = 4000
        ts = np.arange(n + 1) * dt / n
        first = None
        for t in ts:
            p, _ = oracle.static_pairs(sc, t=t, cap=0)
            if p["d"][0] <= 0.02:
                first = t
                break
        if first is None:
            assert pr["status"][0] == oracle.STATUS_NONE
            continue
        checked += 1
        assert pr["status"][0] in (oracle.STATUS_COLLIDES, oracle.STATUS_AT_START)
        # search result within one dense step of the dense first contact
        assert pr["toi"][0] <= first + 1e-6 * dt
        assert first <= pr["toi"][0] + dt / n
    assert checked >= 3
