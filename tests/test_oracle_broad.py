"""Pins of the oracle's broad phase and clustering (section 3: checks 1 and
2, then the unconnected subgraphs), against references other than itself."""

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle


def _scene(n, seed, box=12.0, vs=2.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, box, size=(n, 3))
    v = rng.normal(0, vs, size=(n, 3))
    r = rng.uniform(0.4, 1.1, size=n)
    return x, v, r


def test_static_is_sphere_overlap():
    """dt = 0: both checks reduce to |x_a - x_b| <= r_a + r_b."""
    x, v, r = _scene(300, 1)
    p, _, _ = oracle.broad_phase(x, v, r, 0.0)
    a, b = np.triu_indices(len(r), 1)
    keep = np.linalg.norm(x[a] - x[b], axis=1) <= r[a] + r[b]
    assert {tuple(q) for q in p.tolist()} == set(zip(a[keep].tolist(), b[keep].tolist()))
    # ordered by (a, b)
    assert p.tolist() == sorted(p.tolist())


def test_moving_against_dense_time_sampling():
    """The pair set equals the spheres' contact at any of 20,001 sample times,
    for every pair whose closest approach is not within the sampling error of
    the threshold."""
    x, v, r = _scene(200, 2)
    dt = 0.6
    p, _, _ = oracle.broad_phase(x, v, r, dt)
    got = {tuple(q) for q in p.tolist()}
    a, b = np.triu_indices(len(r), 1)
    d, w = x[b] - x[a], v[b] - v[a]
    ts = np.linspace(0.0, dt, 20001)
    dmin = np.full(a.size, np.inf)
    for t in ts[::1]:
        dmin = np.minimum(dmin, np.linalg.norm(d + w * t, axis=1))
    lim = r[a] + r[b]
    err = np.linalg.norm(w, axis=1) * dt / 20000
    clear = np.abs(dmin - lim) > 2 * err + 1e-12
    exp = {(int(i), int(j)) for i, j, k in zip(a, b, dmin <= lim) if k}
    for i, j, c in zip(a, b, clear):
        if c:
            assert ((int(i), int(j)) in got) == ((int(i), int(j)) in exp)
    assert clear.mean() > 0.99 and len(got) > 20


def test_boxes_overlap_tubes_do_not():
    """The paper's motivating cases for check 2: two spheres moving in
    parallel (the second takes the first's place later) and two spheres
    crossing the same point at different times have overlapping space-time
    boxes but never meet; a head-on pair meets in mid-step."""
    x = np.array([[0, 0, 0], [3, 0, 0],            # parallel, 3 apart
                  [10, 50, 0], [13, 53, 0],        # cross (13, 50, 0) at t = 0.3 and 0.6
                  [20, 100, 0], [26, 100, 0.0]])   # head-on, meet at t = 0.6
    v = np.array([[5, 0, 0], [5, 0, 0],
                  [10, 0, 0], [0, -5, 0],
                  [5, 0, 0], [-5, 0, 0.0]])
    r = np.full(6, 0.5)
    p, lab, _ = oracle.broad_phase(x, v, r, 1.0)
    assert p.tolist() == [[4, 5]]
    assert lab.tolist() == [0, 1, 2, 3, 4, 4]


def test_clusters_are_connected_components():
    x, v, r = _scene(400, 3, box=20.0)
    p, lab, sweeps = oracle.broad_phase(x, v, r, 0.3)
    n = len(r)
    g = coo_matrix((np.ones(len(p)), (p[:, 0], p[:, 1])), shape=(n, n))
    k, comp = connected_components(g, directed=False)
    assert len(set(lab.tolist())) == k
    # same partition, and each label is the smallest position of its subgraph
    for c in range(k):
        members = np.where(comp == c)[0]
        assert np.all(lab[members] == members.min())
    assert k < n and sweeps >= 2


def test_chain_needs_one_sweep_per_link():
    """A chain of touching spheres: the smallest label travels one link per
    sweep (plus the sweep that changes nothing)."""
    n = 12
    x = np.zeros((n, 3))
    x[:, 0] = np.arange(n) * 1.9
    p, lab, sweeps = oracle.broad_phase(x, np.zeros((n, 3)), np.ones(n), 0.0)
    assert len(p) == n - 1 and np.all(lab == 0) and sweeps == n
