"""Pins of the oracle's contact fusion (section 5: contact points close in
space fused into one, centred within parallel triangles)."""

import numpy as np

import oracle
import synth


def _fan(k=6, r=0.5):
    ang = np.arange(k) * 2 * np.pi / k
    V = np.concatenate([[[0, 0, 0]], np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(k)], 1)])
    F = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
    return V, F


def _scene(VA, FA, VB, FB, xb, eps):
    st = np.zeros((2, 13))
    st[:, 3] = 1.0
    st[1, :3] = xb
    return synth.Scene(meshes=[(VA, FA), (VB, FB)], halo=np.array([eps, eps]), mesh_of=np.array([0, 1], np.int32),
                       state=st, pairs=np.array([[0, 1]], np.int32))


def test_vertex_over_a_fan_fuses_into_one():
    """A spike's tip above the shared vertex of a fan of 6 triangles: one
    contact per fan triangle, all at the shared vertex; fused into one
    record at the midpoint (0, 0, h/2) with d = h and 6 members."""
    V, F = _fan()
    tip = np.array([[0, 0, 0], [-0.2, 0.1, 0.5], [0.2, 0.1, 0.5]])
    h, eps = 0.006, 0.005
    sc = _scene(V, F, tip, np.array([[0, 1, 2]], np.int32), [0, 0, h], eps)
    _, con = oracle.static_pairs(sc)
    assert con.shape[0] == 6
    f = oracle.fuse_contacts(con, np.array([2 * eps]))
    assert f.shape[0] == 1 and f["pad"][0] == 6 and (f["tri_a"][0], f["tri_b"][0]) == (0, 0)
    mid = 0.5 * (f["pa"][0] + f["pb"][0])
    assert np.allclose(mid, [0, 0, h / 2], atol=1e-15) and abs(f["d"][0] - h) <= 1e-15
    assert abs(np.linalg.norm(f["pb"][0] - f["pa"][0]) - h) <= 1e-15


def test_far_apart_contacts_stay_apart():
    """Two spikes touching a plane 1 apart: two groups, in record order."""
    V, F = _fan(r=3.0)
    tips = np.array([[0, 0, 0], [-0.2, 0.1, 0.5], [0.2, 0.1, 0.5],
                     [1, 0.3, 0], [0.8, 0.4, 0.5], [1.2, 0.4, 0.5]])
    sc = _scene(V, F, tips, np.array([[0, 1, 2], [3, 4, 5]], np.int32), [0.05, 0.07, 0.004], 0.005)
    _, con = oracle.static_pairs(sc)
    f = oracle.fuse_contacts(con, np.array([0.01]))
    assert f.shape[0] == 2 and f["pad"].sum() == con.shape[0]
    mids = 0.5 * (f["pa"] + f["pb"])
    assert np.linalg.norm(mids[0] - mids[1]) > 0.9


def test_invariants_on_a_packing_sample():
    """Members are conserved, groups come in record order with their seed's
    triangles, every fused contact point lies within delta of its seed's,
    and each group's distance is one of its pair's contact distances."""
    sc = synth.cfg1_scene(run=5)
    _, con = oracle.static_pairs(sc)
    delta = np.full(sc.pairs.shape[0], 0.02)
    f = oracle.fuse_contacts(con, delta)
    assert f["pad"].sum() == con.shape[0] and f.shape[0] < con.shape[0]
    keys = list(zip(f["pair"], f["tri_a"], f["tri_b"]))
    assert keys == sorted(keys)
    rmap = {(int(c["pair"]), int(c["tri_a"]), int(c["tri_b"])): c for c in con}
    for g in f:
        seed = rmap[(int(g["pair"]), int(g["tri_a"]), int(g["tri_b"]))]
        ms = 0.5 * (seed["pa"] + seed["pb"])
        mg = 0.5 * (g["pa"] + g["pb"])
        assert np.linalg.norm(mg - ms) <= 0.02 + 1e-12
        assert g["d"] in con["d"][con["pair"] == g["pair"]]
        assert g["d"] <= seed["d"]
