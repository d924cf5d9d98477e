"""Pins of the oracle's particle interaction (section 6): mass properties of
closed meshes against textbook values, and the Picard impulse solve against
closed-form collisions of two bodies and the conservation laws any set of
internal impulses must obey."""

import numpy as np
import pytest

import oracle
import synth


def box(a, b, c, centre=(0.0, 0.0, 0.0)):
    """Closed box a x b x c about centre, outward triangles."""
    V = np.array([[x, y, z] for z in (-0.5, 0.5) for y in (-0.5, 0.5) for x in (-0.5, 0.5)])
    V = V * np.array([a, b, c]) + np.array(centre)
    F = np.array([[0, 2, 1], [1, 2, 3], [4, 5, 6], [5, 7, 6], [0, 1, 4], [1, 5, 4],
                  [2, 6, 3], [3, 6, 7], [0, 4, 2], [2, 4, 6], [1, 3, 5], [3, 7, 5]], dtype=np.int32)
    return V, F


def state(x, v=(0, 0, 0), w=(0, 0, 0), q=(1, 0, 0, 0)):
    return np.concatenate([x, q, v, w]).astype(float)


def test_mass_properties_of_boxes():
    m, c, I = oracle.mass_properties(*box(1, 1, 1, (0.5, 0.5, 0.5)))
    assert m == pytest.approx(1.0, rel=1e-12)
    assert np.allclose(c, 0.5, atol=1e-12)
    assert np.allclose(I, np.eye(3) / 6.0, atol=1e-12)
    a, b, cc = 2.0, 1.0, 0.5
    m, c, I = oracle.mass_properties(*box(a, b, cc))
    assert m == pytest.approx(a * b * cc, rel=1e-12)
    ref = m / 12.0 * np.diag([b * b + cc * cc, a * a + cc * cc, a * a + b * b])
    assert np.allclose(I, ref, atol=1e-12)
    # the same box inside out, and moved away from the origin
    V, F = box(a, b, cc, (3.0, -2.0, 1.0))
    for FF in (F, F[:, ::-1].copy()):
        m2, c2, I2 = oracle.mass_properties(V, FF)
        assert m2 == pytest.approx(m, rel=1e-12)
        assert np.allclose(c2, [3.0, -2.0, 1.0], atol=1e-12)
        assert np.allclose(I2, ref, atol=1e-10)


def test_mass_properties_of_a_fine_sphere():
    V, F = synth.meshes.icosphere(4)
    m, c, I = oracle.mass_properties(V, F)
    # the polyhedron lies between its inscribed and circumscribed spheres
    T = V[F]
    nrm = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    r_in = np.min(np.abs(np.einsum("ij,ij->i", nrm, T[:, 0])) / np.linalg.norm(nrm, axis=1))
    r_out = np.linalg.norm(V, axis=1).max()
    assert 4.0 / 3.0 * np.pi * r_in ** 3 < m < 4.0 / 3.0 * np.pi * r_out ** 3
    assert np.allclose(c, 0.0, atol=1e-12)
    # a solid ball: I = 2/5 m r^2 on the diagonal
    assert np.allclose(np.diag(I), 0.4 * m * r_out ** 2, rtol=5e-3)
    assert np.allclose(I - np.diag(np.diag(I)), 0.0, atol=1e-12)


def two_cubes(va, vb, sa=1.0, sb=1.0, gap=1e-3, **kw):
    """Two cubes on the x axis, faces apart by gap, one contact between the
    face centres (normal +x, through both centres of mass)."""
    props = [oracle.mass_properties(*box(s, s, s)) for s in (sa, sb)]
    mass = np.array([p[0] for p in props])
    com = np.array([p[1] for p in props])
    inertia = np.array([p[2] for p in props])
    xb = 0.5 * sa + 0.5 * sb + gap
    st = np.array([state([0, 0, 0], va), state([xb, 0, 0], vb)])
    pa = np.array([[0.5 * sa, 0, 0]])
    pb = np.array([[0.5 * sa + gap, 0, 0]])
    return oracle.impulses(mass, com, inertia, st, [[0, 1]], pa, pb, **kw), mass


def test_head_on_inelastic_and_elastic():
    (imp, vel, it, _), m = two_cubes([1, 0, 0], [-1, 0, 0])
    assert imp[0, 0] == pytest.approx(1.0, rel=1e-12)        # reduced mass 1/2 times closing speed 2
    assert np.allclose(vel[:, :3], 0.0, atol=1e-12)
    assert np.allclose(vel[:, 3:], 0.0, atol=1e-12)          # the impulse passes through both centres
    (imp, vel, it, _), m = two_cubes([1, 0, 0], [-1, 0, 0], restitution=1.0)
    assert imp[0, 0] == pytest.approx(2.0, rel=1e-12)
    assert np.allclose(vel[0, :3], [-1, 0, 0], atol=1e-12)
    assert np.allclose(vel[1, :3], [1, 0, 0], atol=1e-12)
    # unequal masses 8 and 1: common velocity (8 - 1) / 9
    (imp, vel, it, _), m = two_cubes([1, 0, 0], [-1, 0, 0], sa=2.0)
    assert np.allclose(vel[:, 0], 7.0 / 9.0, atol=1e-12)


def test_separating_contact_takes_no_impulse():
    (imp, vel, it, _), m = two_cubes([-1, 0, 0], [1, 0, 0])
    assert it == 1
    assert np.all(imp == 0.0)
    assert np.allclose(vel[:, :3], [[-1, 0, 0], [1, 0, 0]])


def test_friction_sticks_or_slides_on_the_cone():
    # B slides along +y relative to A while they close along x
    (imp, vel, it, _), m = two_cubes([1, 0, 0], [-1, 1, 0], friction=10.0, tol=1e-12, max_iter=1000)
    # contact point velocities after the solve: equal (sticking)
    xa, xb = np.zeros(3), np.array([1.001, 0, 0])
    X = np.array([0.5005, 0, 0])
    ua = vel[0, :3] + np.cross(vel[0, 3:], X - xa)
    ub = vel[1, :3] + np.cross(vel[1, 3:], X - xb)
    assert np.allclose(ua, ub, atol=1e-9)
    assert np.linalg.norm(imp[0, 1:]) <= 10.0 * imp[0, 0] + 1e-12
    (imp, vel, it, _), m = two_cubes([1, 0, 0], [-1, 1, 0], friction=0.1, tol=1e-12, max_iter=1000)
    assert np.linalg.norm(imp[0, 1:]) == pytest.approx(0.1 * imp[0, 0], rel=1e-9)   # on the cone
    assert imp[0, 2] < 0.0                                   # opposing B's sliding along +y


def random_cluster(rng, n=6, nc=12):
    props, st = [], []
    for i in range(n):
        dims = rng.uniform(0.5, 1.5, 3)
        props.append(oracle.mass_properties(*box(*dims)))
        q = rng.normal(size=4)
        st.append(state(rng.uniform(-2, 2, 3), rng.normal(size=3), rng.normal(size=3), q / np.linalg.norm(q)))
    mass = np.array([p[0] for p in props])
    com = np.array([p[1] for p in props])
    inertia = np.array([p[2] for p in props])
    ab = []
    for _ in range(nc):
        a, b = rng.choice(n, 2, replace=False)
        ab.append([a, b])
    ab = np.array(ab)
    st = np.array(st)
    mid = 0.5 * (st[ab[:, 0], :3] + st[ab[:, 1], :3]) + rng.normal(scale=0.2, size=(nc, 3))
    gap = 0.01 * rng.normal(size=(nc, 3))
    return mass, com, inertia, st, ab, mid - gap, mid + gap


def momenta(mass, inertia, st, vel):
    P, L = np.zeros(3), np.zeros(3)
    for i in range(len(mass)):
        q = st[i, 3:7]
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        P += mass[i] * vel[i, :3]                             # centres of mass at the origins
        L += np.cross(st[i, :3], mass[i] * vel[i, :3]) + R @ inertia[i] @ R.T @ vel[i, 3:]
    return P, L


@pytest.mark.parametrize("e,mu", [(0.0, 0.0), (0.5, 0.0), (0.0, 0.4), (0.3, 0.8)])
def test_internal_impulses_conserve_momentum(e, mu):
    rng = np.random.default_rng(int(10 * e + 100 * mu))
    mass, com, inertia, st, ab, pa, pb = random_cluster(rng)
    imp, vel, it, col = oracle.impulses(mass, com, inertia, st, ab, pa, pb, restitution=e, friction=mu)
    before = np.concatenate([st[:, 7:10], st[:, 10:13]], axis=1)
    P0, L0 = momenta(mass, inertia, st, before)
    P1, L1 = momenta(mass, inertia, st, vel)
    assert np.allclose(P0, P1, atol=1e-10)
    assert np.allclose(L0, L1, atol=1e-9)
    assert np.all(imp[:, 0] >= 0.0)
    assert np.all(np.linalg.norm(imp[:, 1:], axis=1) <= mu * imp[:, 0] + 1e-12)


def test_converged_solution_meets_the_constraints():
    rng = np.random.default_rng(7)
    mass, com, inertia, st, ab, pa, pb = random_cluster(rng, n=5, nc=8)
    imp, vel, it, col = oracle.impulses(mass, com, inertia, st, ab, pa, pb, tol=1e-13, max_iter=20000)
    assert it < 20000
    X = 0.5 * (pa + pb)
    n = (pb - pa) / np.linalg.norm(pb - pa, axis=1)[:, None]
    for c, (a, b) in enumerate(ab):
        ua = vel[a, :3] + np.cross(vel[a, 3:], X[c] - st[a, :3])
        ub = vel[b, :3] + np.cross(vel[b, 3:], X[c] - st[b, :3])
        un = (ub - ua) @ n[c]
        assert un >= -1e-9                                   # no contact still approaching
        if imp[c, 0] > 1e-9:
            assert abs(un) <= 1e-9                           # active contacts stop exactly


def test_damping_reaches_the_same_solution():
    rng = np.random.default_rng(3)
    args = random_cluster(rng, n=5, nc=8)
    a = oracle.impulses(*args, tol=1e-13, max_iter=50000)
    b = oracle.impulses(*args, relax=0.5, tol=1e-13, max_iter=50000)
    assert b[2] > a[2]
    assert np.allclose(a[1], b[1], atol=1e-8)


def test_colouring_is_greedy_in_contact_order():
    mass, com, inertia, st, ab, pa, pb = random_cluster(np.random.default_rng(1), n=4, nc=3)
    ab = np.array([[0, 1], [1, 2], [2, 3]])
    _, _, _, col = oracle.impulses(mass, com, inertia, st, ab, pa, pb)
    assert list(col) == [0, 1, 0]


def test_clusters_iterate_independently():
    """Two clusters with no particle in common, solved together, give what each
    gives alone, and the sweep count is the larger one."""
    rng = np.random.default_rng(5)
    m1, c1, i1, s1, ab1, pa1, pb1 = random_cluster(rng, n=4, nc=6)
    m2, c2, i2, s2, ab2, pa2, pb2 = random_cluster(rng, n=5, nc=9)
    one = oracle.impulses(m1, c1, i1, s1, ab1, pa1, pb1, tol=1e-6, max_iter=5000)
    two = oracle.impulses(m2, c2, i2, s2, ab2, pa2, pb2, tol=1e-6, max_iter=5000)
    both = oracle.impulses(np.concatenate([m1, m2]), np.concatenate([c1, c2]), np.concatenate([i1, i2]),
                           np.concatenate([s1, s2]), np.concatenate([ab1, ab2 + 4]), np.concatenate([pa1, pa2]),
                           np.concatenate([pb1, pb2]), tol=1e-6, max_iter=5000)
    assert np.array_equal(both[0], np.concatenate([one[0], two[0]]))
    assert np.array_equal(both[1], np.concatenate([one[1], two[1]]))
    assert both[2] == max(one[2], two[2]) and one[2] != two[2]
