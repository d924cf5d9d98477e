"""Comparison of GPU results with the oracle (shared by the GPU tests).

Contact records carry the two closest points p_a, p_b; the contact point is
their midpoint and the normal their difference (section 5, contact-point
definition). Where the closest points of a triangle pair are unique they are
compared with the oracle's element by element; where several point pairs
attain the distance (parallel edges or faces, coplanar overlap) the choice is
not unique, and the check is that p_a lies on triangle a, p_b on triangle b
and |p_b - p_a| = d.
"""

import numpy as np

import oracle


def contact_set(con):
    return {(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"])) for c in con}


def contact_keys(con):
    """(pair, tri_a, tri_b) of each record, in the order returned."""
    return list(zip(con["pair"].tolist(), con["tri_a"].tolist(), con["tri_b"].tolist()))


def assert_contact_order(con):
    """Records are ordered by (pair, tri_a, tri_b), each key once."""
    k = contact_keys(con)
    bad = [i for i in range(1, len(k)) if not k[i - 1] < k[i]]
    assert not bad, ("out of order at", bad[:5], [k[i - 1:i + 1] for i in bad[:3]])


def _edges(T):
    return [(T[k], T[(k + 1) % 3]) for k in range(3)]


def feature_points(ta, tb):
    """The 15 distance features of a triangle pair in the oracle's order (A's
    vertices against B, B's vertices against A, the 9 edge pairs), each as
    (d, p_a, p_b, near_parallel), from the oracle's primitives."""
    A, B = ta.reshape(3, 3), tb.reshape(3, 3)
    out = []
    for k in range(3):
        d, q = oracle.point_triangle(A[k], B)
        out.append((d, A[k].copy(), q, False))
    for k in range(3):
        d, q = oracle.point_triangle(B[k], A)
        out.append((d, q, B[k].copy(), False))
    for (p1, q1) in _edges(A):
        for (p2, q2) in _edges(B):
            d, c1, c2 = oracle.segment_segment(p1, q1, p2, q2)
            e1, e2 = q1 - p1, q2 - p2
            cr = np.cross(e1, e2)
            par = (cr @ cr) <= 1e-8 * (e1 @ e1) * (e2 @ e2)
            out.append((d, c1, c2, par))
    return out


def points_unique(ta, tb, d, qa, qb, tol, band):
    """True when every feature within `band` of the distance gives the same
    closest points as the oracle (within tol/10) and none of them is a
    near-parallel edge pair: the closest points are then well defined."""
    if d == 0.0:
        # an intersection: the oracle's point is the first edge crossing in
        # its fixed order; coplanar overlap (every feature at 0) is ambiguous
        return min(f[0] for f in feature_points(ta, tb)) > 0.0
    for fd, pa, pb, par in feature_points(ta, tb):
        if fd <= d + band:
            if par:
                return False
            if max(np.abs(pa - qa).max(), np.abs(pb - qb).max()) > tol / 10:
                return False
    return True


def check_points(scene, pairs, con, times=None, rtol=1e-6, rtol_pts=None, stats=None):
    """Closest points of every contact record against the oracle at the
    record's time (times[pair], default 0). Returns the number of records
    compared element by element and the number checked by invariants only."""
    rtol_pts = rtol if rtol_pts is None else rtol_pts
    halo = scene.halo[scene.mesh_of]
    cache = {}
    n_cmp = n_inv = 0
    for c in con:
        p = int(c["pair"])
        ia, ib = (int(x) for x in pairs[p])
        t = 0.0 if times is None else float(times[p])
        dl = halo[ia] + halo[ib]
        key = (ia, ib, t)
        if key not in cache:
            cache[key] = (scene.meshes[scene.mesh_of[ia]], scene.meshes[scene.mesh_of[ib]])
        (Va, Fa), (Vb, Fb) = cache[key]
        ta = oracle.world_tris(Va, Fa[[int(c["tri_a"])]], scene.state[ia], t)[0]
        tb = oracle.world_tris(Vb, Fb[[int(c["tri_b"])]], scene.state[ib], t)[0]
        d, qa, qb, _ = oracle.tri_tri(ta, tb)
        tol = rtol_pts * max(d, dl)
        scale = max(1.0, float(np.abs(ta).max()), float(np.abs(tb).max()))
        pa, pb = np.asarray(c["pa"], np.float64), np.asarray(c["pb"], np.float64)
        # invariants: each point on its own triangle, and their distance is d
        on_a, _ = oracle.point_triangle(pa, ta.reshape(3, 3))
        on_b, _ = oracle.point_triangle(pb, tb.reshape(3, 3))
        assert on_a <= tol + 1e-14 * scale and on_b <= tol + 1e-14 * scale, (c, on_a, on_b)
        assert abs(np.linalg.norm(pb - pa) - d) <= tol + 1e-14 * scale, (c, d)
        if points_unique(ta, tb, d, qa, qb, tol, 1e-9 * scale):
            n_cmp += 1
            err = max(np.abs(pa - qa).max(), np.abs(pb - qb).max())
            assert err <= 10 * tol + 1e-14 * scale, ("closest points", c, qa, qb, err)
        else:
            n_inv += 1
    if stats is not None:
        stats["compared"] = stats.get("compared", 0) + n_cmp
        stats["invariants_only"] = stats.get("invariants_only", 0) + n_inv
    return n_cmp, n_inv


def check_static(scene, pairs, pr, con, ref, rcon, rtol, dense=True, rtol_pts=None, max_points=4000,
                 times=None):
    """Pair minima, argmins, closest points and contact sets against the oracle.
    Tolerance form: |x - x_ref| <= rtol * max(|x_ref|, delta). Contact records'
    closest points are checked with check_points (all records, or a seeded
    sample of max_points of them)."""
    rtol_pts = rtol if rtol_pts is None else rtol_pts
    n = pairs.shape[0]
    assert pr.shape[0] == n
    halo = scene.halo[scene.mesh_of]
    delta = halo[pairs[:, 0]] + halo[pairs[:, 1]]
    # contact flags and sets: exact
    assert np.array_equal(pr["contact"], ref["contact"]), (pr["contact"], ref["contact"])
    got, exp = contact_set(con), contact_set(rcon)
    assert got == exp, ("missing", sorted(exp - got)[:10], "extra", sorted(got - exp)[:10])
    # and in the order the interface states: by (pair, tri_a, tri_b)
    assert contact_keys(con) == sorted(exp)
    # contact records: distance against the oracle's record, points by check_points
    rmap = {(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"])): c for c in rcon}
    for c in con:
        r = rmap[(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"]))]
        dl = delta[c["pair"]]
        assert abs(c["d"] - r["d"]) <= rtol * max(r["d"], dl), (c, r)
        if "t" in con.dtype.names:
            tp = 0.0 if times is None else float(times[int(c["pair"])])
            assert c["t"] == tp, (c, tp)
    sel = con
    if con.shape[0] > max_points:
        rng = np.random.default_rng(len(con))
        sel = con[np.sort(rng.choice(con.shape[0], size=max_points, replace=False))]
    check_points(scene, pairs, sel, times=times, rtol=rtol, rtol_pts=rtol_pts)
    # pair minima
    for p in range(n):
        if not dense and not ref["contact"][p]:
            assert not np.isfinite(pr["dmin"][p]) and pr["tri_a"][p] == -1
            continue
        dr = ref["d"][p]
        assert abs(pr["dmin"][p] - dr) <= rtol * max(dr, delta[p]), (p, pr["dmin"][p], dr)
        # the reported argmin attains the minimum (ties may pick another pair),
        # and its closest points are checked like a contact record's
        rec = np.zeros(1, dtype=[("pair", "<i4"), ("tri_a", "<i4"), ("tri_b", "<i4"),
                                 ("pa", "<f8", 3), ("pb", "<f8", 3)])
        rec["pair"], rec["tri_a"], rec["tri_b"] = p, pr["tri_a"][p], pr["tri_b"][p]
        rec["pa"], rec["pb"] = pr["pa"][p], pr["pb"][p]
        ia, ib = pairs[p]
        Va, Fa = scene.meshes[scene.mesh_of[ia]]
        Vb, Fb = scene.meshes[scene.mesh_of[ib]]
        tp = 0.0 if times is None else float(times[p])
        ta = oracle.world_tris(Va, Fa[[pr["tri_a"][p]]], scene.state[ia], tp)
        tb = oracle.world_tris(Vb, Fb[[pr["tri_b"][p]]], scene.state[ib], tp)
        d, qa, qb, _ = oracle.tri_tri(ta[0], tb[0])
        assert abs(d - dr) <= rtol * max(dr, delta[p])
        check_points(scene, pairs, rec, times=times, rtol=rtol, rtol_pts=rtol_pts)
        if (pr["tri_a"][p], pr["tri_b"][p]) == (ref["tri_a"][p], ref["tri_b"][p]):
            tol = rtol_pts * max(dr, delta[p]) * 10
            scale = max(1.0, float(np.abs(ta).max()), float(np.abs(tb).max()))
            if points_unique(ta[0], tb[0], d, qa, qb, tol / 10, 1e-9 * scale):
                assert np.abs(pr["pa"][p] - ref["pa"][p]).max() <= tol, (pr["pa"][p], ref["pa"][p])
                assert np.abs(pr["pb"][p] - ref["pb"][p]).max() <= tol
