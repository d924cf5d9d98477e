"""Pins for the oracle's geometric primitives and triangle-triangle distance.

Every expected value here comes from a closed form, an independent solver
(active-set enumeration of the convex quadratic program over the two
triangles, written below with numpy least squares) or an invariant, never
from the oracle itself.
"""

import itertools

import numpy as np
import pytest

import oracle

T0 = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0]])


# ---------------------------------------------------------------- point-triangle
@pytest.mark.parametrize("p,q", [
    ([0.5, 0.5, 0.7], [0.5, 0.5, 0.0]),     # face region: projection
    ([-1.0, -1.0, 0.3], [0.0, 0.0, 0.0]),   # vertex 0 region
    ([3.0, -0.5, 0.2], [2.0, 0.0, 0.0]),    # vertex 1 region
    ([-0.5, 3.0, -0.4], [0.0, 2.0, 0.0]),   # vertex 2 region
    ([1.0, -1.0, 0.5], [1.0, 0.0, 0.0]),    # edge v0-v1 region
    ([-1.0, 1.2, -0.5], [0.0, 1.2, 0.0]),   # edge v0-v2 region
    ([2.0, 2.0, 1.0], [1.0, 1.0, 0.0]),     # edge v1-v2 region
])
def test_point_triangle_regions(p, q):
    d, c = oracle.point_triangle(p, T0)
    assert np.allclose(c, q, atol=1e-14)
    assert d == pytest.approx(np.linalg.norm(np.subtract(p, q)), abs=1e-14)


# -------------------------------------------------------------- segment-segment
def test_segment_segment_cases():
    # perpendicular skew, offset h
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [1, 0, 0], [0.5, -1, 0.3], [0.5, 1, 0.3])
    assert d == pytest.approx(0.3, abs=1e-15)
    assert np.allclose(c1, [0.5, 0, 0]) and np.allclose(c2, [0.5, 0, 0.3])
    # parallel, overlapping, offset 0.2
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [1, 0, 0], [0.5, 0.2, 0], [2.0, 0.2, 0])
    assert d == pytest.approx(0.2, abs=1e-15)
    assert np.linalg.norm(c1 - c2) == pytest.approx(0.2, abs=1e-15)
    # collinear, disjoint, gap 0.25
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [1, 0, 0], [1.25, 0, 0], [3, 0, 0])
    assert d == pytest.approx(0.25, abs=1e-15)
    assert np.allclose(c1, [1, 0, 0]) and np.allclose(c2, [1.25, 0, 0])
    # crossing
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [2, 2, 0], [0, 2, 0], [2, 0, 0])
    assert d == pytest.approx(0.0, abs=1e-15)
    assert np.allclose(c1, [1, 1, 0]) and np.allclose(c2, [1, 1, 0])
    # closest point beyond the end of segment 2 (t clamps to 1, s recomputed)
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [4, 0, 0], [1, 1, 1], [1, 3, 1])
    assert d == pytest.approx(np.sqrt(2.0), abs=1e-14)
    assert np.allclose(c1, [1, 0, 0]) and np.allclose(c2, [1, 1, 1])
    # closest point before the start of segment 2 (t clamps to 0)
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [4, 0, 0], [3, -1, 0.5], [3, -4, 0.5])
    assert d == pytest.approx(np.hypot(1.0, 0.5), abs=1e-14)
    assert np.allclose(c1, [3, 0, 0]) and np.allclose(c2, [3, -1, 0.5])
    # s clamps to 1 at the end of segment 1
    d, c1, c2 = oracle.segment_segment([0, 0, 0], [1, 0, 0], [2, -1, 0], [2, 1, 0])
    assert d == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(c1, [1, 0, 0]) and np.allclose(c2, [2, 0, 0])


# ------------------------------------------------------------ segment-triangle
def test_segment_triangle_cases():
    hit, x = oracle.segment_triangle([0.5, 0.5, -1], [0.5, 0.5, 1], T0)
    assert hit and np.allclose(x, [0.5, 0.5, 0])
    hit, _ = oracle.segment_triangle([1.5, 1.5, -1], [1.5, 1.5, 1], T0)   # beside the face
    assert not hit
    hit, _ = oracle.segment_triangle([0.5, 0.5, 0.1], [0.5, 0.5, 1], T0)  # one side only
    assert not hit
    hit, x = oracle.segment_triangle([0.5, 0.5, 0.0], [0.5, 0.5, 1], T0)  # endpoint on face
    assert hit and np.allclose(x, [0.5, 0.5, 0])
    hit, x = oracle.segment_triangle([1.0, 1.0, -1], [1.0, 1.0, 1], T0)   # through an edge
    assert hit and np.allclose(x, [1, 1, 0])
    hit, _ = oracle.segment_triangle([0.2, 0.2, 0.3], [1.0, 0.2, 0.3], T0)  # parallel above
    assert not hit


# ---------------------------------------------- independent triangle distance
def qp_distance(A, B):
    """Exact distance of two triangles by enumerating the faces (vertex, edge,
    triangle) of both simplices, minimising on each pair of affine hulls with
    least squares and keeping feasible minimisers."""
    best = np.inf
    subsets = [s for r in (1, 2, 3) for s in itertools.combinations(range(3), r)]
    for sa in subsets:
        for sb in subsets:
            a0, b0 = A[sa[0]], B[sb[0]]
            cols = [A[k] - a0 for k in sa[1:]] + [-(B[k] - b0) for k in sb[1:]]
            r0 = a0 - b0
            if cols:
                M = np.stack(cols, axis=1)
                z, *_ = np.linalg.lstsq(M, -r0, rcond=None)
            else:
                z = np.zeros(0)
            al, be = z[:len(sa) - 1], z[len(sa) - 1:]
            la = np.concatenate([[1 - al.sum()], al])
            lb = np.concatenate([[1 - be.sum()], be])
            if (la < -1e-12).any() or (lb < -1e-12).any():
                continue
            P = (la[:, None] * A[list(sa)]).sum(axis=0)
            Q = (lb[:, None] * B[list(sb)]).sum(axis=0)
            best = min(best, np.linalg.norm(P - Q))
    return best


def _on_triangle(p, T, tol=1e-9):
    d, _ = oracle.point_triangle(p, T.reshape(9))
    return d <= tol


def test_tri_tri_parallel_faces():
    A = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]])
    B = A + [0.1, 0.1, 0.05]
    d, pa, pb, _ = oracle.tri_tri(A, B)
    assert d == pytest.approx(0.05, abs=1e-15)


def test_tri_tri_crossed_edges():
    A = np.array([[-1, 0, 0], [1, 0, 0], [0, 0, -1.0]])       # top edge on the x axis
    B = np.array([[0, -1, 0.3], [0, 1, 0.3], [0, 0, 1.3]])     # bottom edge along y at z=.3
    d, pa, pb, f = oracle.tri_tri(A, B)
    assert d == pytest.approx(0.3, abs=1e-15)
    assert np.allclose(pa, [0, 0, 0]) and np.allclose(pb, [0, 0, 0.3])
    assert 12 <= f <= 20


def test_tri_tri_intersecting_is_zero():
    A = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0.0]])
    B = np.array([[0, -0.5, -1], [0, -0.5, 1], [0, 2, 0.0]])  # pierces A
    d, pa, pb, f = oracle.tri_tri(A, B)
    assert d == 0.0 and f < 6
    assert np.allclose(pa, pb)
    assert _on_triangle(pa, A) and _on_triangle(pa, B)


def test_tri_tri_x_crossing_far_features():
    # Two long thin triangles crossing through each other's middle: all 15
    # vertex and edge-pair features are non-zero, only the intersection test
    # sees d = 0.
    A = np.array([[-5, 0, 0], [5, -0.3, 0], [5, 0.3, 0.0]])
    B = np.array([[0, -5, -0.5], [0.3, 5, 0.5], [-0.3, 5, 0.5]])
    d, pa, pb, f = oracle.tri_tri(A, B)
    assert d == 0.0 and f < 6
    assert qp_distance(A, B) < 1e-12
    feats = [oracle.point_triangle(A[k], B.reshape(9))[0] for k in range(3)]
    feats += [oracle.point_triangle(B[k], A.reshape(9))[0] for k in range(3)]
    feats += [oracle.segment_segment(A[k], A[(k + 1) % 3], B[l], B[(l + 1) % 3])[0]
              for k in range(3) for l in range(3)]
    assert min(feats) > 1e-3


def test_tri_tri_coplanar_overlap_is_zero():
    A = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]])
    B = np.array([[0.2, 0.2, 0], [1.2, 0.2, 0], [0.2, 1.2, 0.0]])
    d, pa, pb, f = oracle.tri_tri(A, B)
    assert d <= 1e-15          # exact zero up to the rounding of the face projection
    assert 6 <= f


def test_tri_tri_against_qp_random():
    rng = np.random.default_rng(11)
    worst = 0.0
    for k in range(3000):
        A = rng.normal(size=(3, 3))
        B = rng.normal(size=(3, 3)) + rng.normal(size=3) * rng.uniform(0, 3)
        d, pa, pb, _ = oracle.tri_tri(A, B)
        ref = qp_distance(A, B)
        worst = max(worst, abs(d - ref))
        assert abs(d - ref) <= 1e-9 * max(1.0, ref), (k, d, ref)
        # closest points lie on their triangles and realise d
        assert _on_triangle(pa, A, 1e-9) and _on_triangle(pb, B, 1e-9)
        assert np.linalg.norm(pa - pb) == pytest.approx(d, abs=1e-9)
    assert worst < 1e-9


def test_tri_tri_symmetry_and_rigid_invariance():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(12)
    for _ in range(500):
        A = rng.normal(size=(3, 3))
        B = rng.normal(size=(3, 3)) + rng.normal(size=3)
        d1, pa1, pb1, _ = oracle.tri_tri(A, B)
        d2, pa2, pb2, _ = oracle.tri_tri(B, A)
        assert d1 == pytest.approx(d2, rel=1e-12, abs=1e-14)
        R = Rotation.random(random_state=rng).as_matrix()
        t = rng.normal(size=3) * 5
        d3, pa3, pb3, _ = oracle.tri_tri(A @ R.T + t, B @ R.T + t)
        assert d3 == pytest.approx(d1, rel=1e-11, abs=1e-13)


def test_dense_sampling_bounds():
    """Barycentric grid sampling bounds d from above, within the grid spacing."""
    rng = np.random.default_rng(13)
    n = 24
    g = [(i / n, j / n) for i in range(n + 1) for j in range(n + 1 - i)]
    W = np.array([[1 - u - v, u, v] for u, v in g])
    for _ in range(40):
        A = rng.normal(size=(3, 3))
        B = rng.normal(size=(3, 3)) + rng.normal(size=3) * 2
        d, *_ = oracle.tri_tri(A, B)
        PA, PB = W @ A, W @ B
        dm = np.sqrt(((PA[:, None, :] - PB[None, :, :]) ** 2).sum(-1)).min()
        spacing = max(np.linalg.norm(A[i] - A[j]) for i in range(3) for j in range(3)) / n + \
            max(np.linalg.norm(B[i] - B[j]) for i in range(3) for j in range(3)) / n
        assert d <= dm + 1e-12
        assert dm <= d + spacing
