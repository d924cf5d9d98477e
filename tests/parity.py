"""Comparison of GPU results with the oracle (shared by the GPU tests)."""

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


def check_static(scene, pairs, pr, con, ref, rcon, rtol, dense=True, rtol_pts=None):
    """Pair minima, argmins, closest points and contact sets against the oracle.
    Tolerance form: |x - x_ref| <= rtol * max(|x_ref|, delta)."""
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
    # contact records
    rmap = {(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"])): c for c in rcon}
    for c in con:
        r = rmap[(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"]))]
        dl = delta[c["pair"]]
        assert abs(c["d"] - r["d"]) <= rtol * max(r["d"], dl), (c, r)
        # closest points: checked by invariants (unique only off parallel features)
        assert abs(np.linalg.norm(c["pb"] - c["pa"]) - c["d"]) <= rtol_pts * dl
    # pair minima
    for p in range(n):
        if not dense and not ref["contact"][p]:
            assert not np.isfinite(pr["dmin"][p]) and pr["tri_a"][p] == -1
            continue
        dr = ref["d"][p]
        assert abs(pr["dmin"][p] - dr) <= rtol * max(dr, delta[p]), (p, pr["dmin"][p], dr)
        # the reported argmin attains the minimum (ties may pick another pair)
        ia, ib = pairs[p]
        ma, mb = scene.mesh_of[ia], scene.mesh_of[ib]
        Va, Fa = scene.meshes[ma]
        Vb, Fb = scene.meshes[mb]
        ta = oracle.world_tris(Va, Fa[[pr["tri_a"][p]]], scene.state[ia])
        tb = oracle.world_tris(Vb, Fb[[pr["tri_b"][p]]], scene.state[ib])
        d, qa, qb, _ = oracle.tri_tri(ta[0], tb[0])
        assert abs(d - dr) <= rtol * max(dr, delta[p])
        assert abs(np.linalg.norm(pr["pb"][p] - pr["pa"][p]) - dr) <= rtol_pts * max(dr, delta[p])
        if (pr["tri_a"][p], pr["tri_b"][p]) == (ref["tri_a"][p], ref["tri_b"][p]):
            tol = rtol_pts * max(dr, delta[p]) * 10
            assert np.abs(pr["pa"][p] - ref["pa"][p]).max() <= tol, (pr["pa"][p], ref["pa"][p])
            assert np.abs(pr["pb"][p] - ref["pb"][p]).max() <= tol
