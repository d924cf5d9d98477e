"""Pins for the oracle's particle-pair (mesh) queries.

Expected values come from the support function of convex icospheres, from an
independent QP solver over every triangle pair, or from invariants.
"""

import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from test_oracle_primitives import qp_distance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _two(meshA, meshB, xa, xb, qa=(1, 0, 0, 0), qb=(1, 0, 0, 0), eps=0.01):
    sa = np.concatenate([xa, qa, np.zeros(6)])
    sb = np.concatenate([xb, qb, np.zeros(6)])
    return synth.pair_test_scene(meshA, meshB, sa, sb, eps)


def _face_centre_dir(V, F, k=0):
    c = V[F[k]].mean(axis=0)
    return c / np.linalg.norm(c)


def _edge_mid_dir(V, F, k=0):
    m = 0.5 * (V[F[k][0]] + V[F[k][1]])
    return m / np.linalg.norm(m)


def test_icosahedron_constants():
    """Support of the unit icosahedron along a face normal (inradius) and an
    edge midpoint (midradius), from tests/golden/icosphere_support.json."""
    g = json.load(open(os.path.join(GOLDEN, "icosphere_support.json")))
    for s, h in g["face_centre"].items():
        V, F = synth.icosphere(int(s))
        u = _face_centre_dir(*synth.icosphere(0), k=0)
        assert (V @ u).max() == pytest.approx(h, abs=1e-9)
    V, F = synth.icosphere(0)
    assert (V @ _edge_mid_dir(V, F)).max() == pytest.approx(g["edge_mid_s0"], abs=1e-9)


@pytest.mark.parametrize("subdiv", [0, 1, 2])
@pytest.mark.parametrize("kind", ["vertex", "face", "edge"])
def test_icosphere_translated_copy_closed_form(subdiv, kind):
    """B = A + sep u. Both convex and centrally symmetric, so the distance is
    sep - 2 h(u) with h the support function, attained by antipodal features."""
    V, F = synth.icosphere(subdiv)
    V0, F0 = synth.icosphere(0)
    u = {"vertex": V0[0], "face": _face_centre_dir(V0, F0), "edge": _edge_mid_dir(V0, F0)}[kind]
    u = u / np.linalg.norm(u)
    h = (V @ u).max()
    rng = np.random.default_rng(21)
    for sep in (2 * h + 0.003, 2 * h + 0.0199, 2 * h + 0.5):
        R = Rotation.random(random_state=rng)
        q = R.as_quat()  # x, y, z, w
        qwxyz = np.array([q[3], q[0], q[1], q[2]])
        xa = rng.normal(size=3)
        xb = xa + sep * R.apply(u)
        sc = _two((V, F), (V, F), xa, xb, qwxyz, qwxyz)
        pr, con = oracle.static_pairs(sc)
        assert pr["d"][0] == pytest.approx(sep - 2 * h, abs=1e-12)
        assert bool(pr["contact"][0]) == (sep - 2 * h <= 0.02)
        assert (con["d"] <= 0.02).all()
        # closest points: on the two support planes
        pa, pb = pr["pa"][0], pr["pb"][0]
        assert np.linalg.norm(pb - pa) == pytest.approx(sep - 2 * h, abs=1e-12)


@pytest.mark.parametrize("kind", ["vertex", "face"])
def test_icosphere_overlap_gives_zero(kind):
    V, F = synth.icosphere(1)
    V0, F0 = synth.icosphere(0)
    u = V0[0] if kind == "vertex" else _face_centre_dir(V0, F0)
    u = u / np.linalg.norm(u)
    h = (V @ u).max()
    for sep in (0.3 * h, 1.0 * h, 1.9 * h):
        sc = _two((V, F), (V, F), np.zeros(3), sep * u)
        pr, con = oracle.static_pairs(sc)
        assert pr["d"][0] == 0.0
        assert pr["contact"][0] == 1


def _tetra(rng, scale=1.0):
    V = rng.normal(size=(4, 3)) * scale
    F = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)
    return V, F


def test_small_meshes_against_qp():
    """Contact sets and minima of tiny meshes against the QP solver applied to
    every triangle pair of the world-frame meshes (posed with scipy)."""
    rng = np.random.default_rng(22)
    for trial in range(30):
        A, B = _tetra(rng, 0.5), _tetra(rng, 0.5)
        RA, RB = Rotation.random(random_state=rng), Rotation.random(random_state=rng)
        xa = np.zeros(3)
        xb = rng.normal(size=3)
        xb *= rng.uniform(0.3, 1.5) / np.linalg.norm(xb)
        qa, qb = RA.as_quat(), RB.as_quat()
        eps = rng.uniform(0.01, 0.2)
        sc = _two(A, B, xa, xb, [qa[3], *qa[:3]], [qb[3], *qb[:3]], eps=eps)
        pr, con = oracle.static_pairs(sc)
        WA = RA.apply(A[0]) + xa
        WB = RB.apply(B[0]) + xb
        D = np.array([[qp_distance(WA[fa], WB[fb]) for fb in B[1]] for fa in A[1]])
        assert pr["d"][0] == pytest.approx(D.min(), abs=1e-9)
        i, j = np.unravel_index(np.argmin(D), D.shape)
        assert D[pr["tri_a"][0], pr["tri_b"][0]] == pytest.approx(D.min(), abs=1e-9)
        ref = {(a, b) for a in range(4) for b in range(4) if D[a, b] <= 2 * eps}
        got = {(int(c["tri_a"]), int(c["tri_b"])) for c in con}
        # the QP and the oracle can disagree only within rounding of delta
        band = {(a, b) for a in range(4) for b in range(4) if abs(D[a, b] - 2 * eps) < 1e-9}
        assert (ref ^ got) <= band
        for c in con:
            assert c["d"] == pytest.approx(D[c["tri_a"], c["tri_b"]], abs=1e-9)


def test_pair_symmetry():
    sc = synth.cfg1_scene(run=3, n_pairs=4)
    pr, con = oracle.static_pairs(sc)
    pr2, con2 = oracle.static_pairs(sc, pairs=sc.pairs[:, ::-1].copy())
    assert np.allclose(pr["d"], pr2["d"], rtol=1e-12, atol=1e-15)
    s1 = {(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"])) for c in con}
    s2 = {(int(c["pair"]), int(c["tri_b"]), int(c["tri_a"])) for c in con2}
    assert s1 == s2
    # the same winning triangle pair (no tie) gives the same closest points, swapped
    same = (pr["tri_a"] == pr2["tri_b"]) & (pr["tri_b"] == pr2["tri_a"])
    assert same.sum() >= 2
    assert np.allclose(pr["pa"][same], pr2["pb"][same], atol=1e-12)
    assert np.allclose(pr["pb"][same], pr2["pa"][same], atol=1e-12)


def test_lowest_index_wins_ties():
    """A mesh holding the same face twice: both copies tie, the lower id wins."""
    A = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]]), np.array([[0, 1, 2], [0, 1, 2]], np.int32))
    B = (np.array([[0, 0, 0.05], [1, 0, 0.05], [0, 1, 0.05]]) + [0.1, 0.1, 0],
         np.array([[0, 1, 2], [0, 1, 2]], np.int32))
    sc = _two(A, B, np.zeros(3), np.zeros(3))
    pr, con = oracle.static_pairs(sc)
    assert pr["d"][0] == pytest.approx(0.05, abs=1e-15)
    assert (pr["tri_a"][0], pr["tri_b"][0]) == (0, 0)
    assert len(con) == 0
    sc.halo[:] = 0.025   # delta = 0.05: closed threshold, every pair is a contact
    pr, con = oracle.static_pairs(sc)
    assert [(c["tri_a"], c["tri_b"]) for c in con] == [(0, 0), (0, 1), (1, 0), (1, 1)]


def test_common_rigid_motion_invariance():
    sc = synth.cfg1_scene(run=4, n_pairs=3)
    pr, con = oracle.static_pairs(sc)
    rng = np.random.default_rng(23)
    R = Rotation.random(random_state=rng)
    t = rng.normal(size=3) * 10
    st = sc.state.copy()
    st[:, 0:3] = R.apply(st[:, 0:3]) + t
    q = Rotation.from_quat(np.c_[st[:, 4:7], st[:, 3]])
    q2 = (R * q).as_quat()
    st[:, 3] = q2[:, 3]
    st[:, 4:7] = q2[:, :3]
    sc.state = st
    pr2, con2 = oracle.static_pairs(sc)
    assert np.allclose(pr["d"], pr2["d"], rtol=1e-10, atol=1e-12)
    assert len(con) == len(con2)
