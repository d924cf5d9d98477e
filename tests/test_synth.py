"""Generators: counts, closure, symmetry and perturbation bounds."""

import numpy as np
import pytest

import synth


def _edges_closed(F):
    e = {}
    for f in F:
        for k in range(3):
            a, b = int(f[k]), int(f[(k + 1) % 3])
            e[(a, b)] = e.get((a, b), 0) + 1
    # closed, consistently oriented 2-manifold: every directed edge once, with its reverse
    return all(c == 1 and e.get((b, a)) == 1 for (a, b), c in e.items())


@pytest.mark.parametrize("s", [0, 1, 2, 3])
def test_icosphere_counts_symmetry(s):
    V, F = synth.icosphere(s)
    assert V.shape == (10 * 4 ** s + 2, 3) and F.shape == (20 * 4 ** s, 3)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    assert _edges_closed(F)
    # centrally symmetric vertex set
    d = np.linalg.norm(V[:, None, :] + V[None, :, :], axis=2).min(axis=1)
    assert d.max() < 1e-12
    # outward orientation
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    assert ((n * V[F].mean(axis=1)).sum(axis=1) > 0).all()


@pytest.mark.parametrize("T", [20, 37, 300, 920, 5120])
def test_uv_sphere(T):
    V, F = synth.uv_sphere(T)
    m, k = synth.uv_sphere_size(T)
    assert F.shape[0] == 2 * m * k
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    assert _edges_closed(F)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    assert ((n * V[F].mean(axis=1)).sum(axis=1) > 0).all()


def test_perturbation_bounds_and_seed():
    V, F = synth.icosphere(2)
    a = synth.perturb_radial(V, np.random.default_rng(5))
    b = synth.perturb_radial(V, np.random.default_rng(5))
    r = np.linalg.norm(a, axis=1)
    assert np.array_equal(a, b)
    assert r.min() >= 0.9 and r.max() <= 1.1


def test_quaternions_unit_and_packing():
    rng = np.random.default_rng(6)
    q = synth.random_quaternions(1000, rng)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0)
    x, side = synth.relax_packing(200, 1.1, 0.5, rng)
    d = np.linalg.norm(x[:, None] - x[None], axis=2) + np.eye(200) * 10
    assert d.min() >= 2.2 - 1e-9
    assert (x >= 1.1 - 1e-12).all() and (x <= side - 1.1 + 1e-12).all()
    y, side2 = synth.rsa_packing(300, 1.1, 0.25, rng)
    d = np.linalg.norm(y[:, None] - y[None], axis=2) + np.eye(300) * 10
    assert d.min() >= 2.2


def test_cfg1_shape():
    sc = synth.cfg1_scene()
    assert sc.pairs.shape == (16, 2) and sc.dense_tri_pairs() == 16 * 320 * 320
    g = sc.info["gaps"]
    sep = np.linalg.norm(sc.state[1::2, :3] - sc.state[0::2, :3], axis=1)
    assert np.allclose(sep - 2, g) and (g >= 0).all() and (g <= 0.02).all()


def test_sphere_pairs_moving():
    x = np.array([[0, 0, 0], [5, 0, 0], [0, 10, 0.0]])
    v = np.array([[0, 0, 0], [-10, 0, 0], [0, 0, 0.0]])
    R = np.ones(3)
    assert synth.sphere_pairs(x, R, 0.01).shape[0] == 0
    p = synth.sphere_pairs(x, R, 0.01, v=v, dt=0.5)
    assert p.tolist() == [[0, 1]]
