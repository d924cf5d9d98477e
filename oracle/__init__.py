"""FP64 CPU oracle (ctypes wrapper around mcd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library. It shares no code with
the GPU path. See mcd_oracle.c for what each routine computes and which part
of the paper it follows.

Parity unpinned: closest points when several feature pairs tie (parallel
edges or faces; only invariants are checked there) and graze leaves of the
time-stamp search (counted, not compared).
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcd_oracle.c")
_LIB = os.path.join(_HERE, "libmcd_oracle.so")

CONTACT_DT = np.dtype([("pair", "<i4"), ("tri_a", "<i4"), ("tri_b", "<i4"), ("pad", "<i4"),
                       ("d", "<f8"), ("pa", "<f8", 3), ("pb", "<f8", 3)])
PAIR_DT = np.dtype([("d", "<f8"), ("pa", "<f8", 3), ("pb", "<f8", 3), ("toi", "<f8"),
                    ("tri_a", "<i4"), ("tri_b", "<i4"), ("contact", "<i4"), ("status", "<i4")])

STATUS_NONE, STATUS_AT_START, STATUS_COLLIDES = 0, 1, 2


def build(force=False):
    """Compile the oracle with gcc (plain C, -O2, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_tri_tri.restype = ctypes.c_double
        L.orc_tri_tri.argtypes = [P, P, P, P, P]
        L.orc_point_triangle.restype = ctypes.c_double
        L.orc_point_triangle.argtypes = [P, P, P]
        L.orc_segment_segment.restype = ctypes.c_double
        L.orc_segment_segment.argtypes = [P, P, P, P, P, P]
        L.orc_segment_triangle.restype = ctypes.c_int
        L.orc_segment_triangle.argtypes = [P, P, P, P]
        L.orc_pose.restype = None
        L.orc_pose.argtypes = [P, ctypes.c_double, P, P]
        L.orc_world_tris.restype = None
        L.orc_world_tris.argtypes = [P, P, ctypes.c_int, P, ctypes.c_double, P]
        L.orc_tri_pair_toi.restype = ctypes.c_double
        L.orc_tri_pair_toi.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_double, P, P]
        L.orc_static_pairs.restype = ctypes.c_int64
        L.orc_static_pairs.argtypes = [P, P, P, P, P, P, P, P, ctypes.c_int32, P,
                                       ctypes.c_double, P, P, ctypes.c_int64]
        L.orc_narrow_tri_pair.restype = ctypes.c_double
        L.orc_narrow_tri_pair.argtypes = [P, P, P, ctypes.c_double]
        L.orc_narrow_pairs.restype = ctypes.c_int64
        L.orc_narrow_pairs.argtypes = [P, P, P, P, P, P, P, P, ctypes.c_int32, P, ctypes.c_double, P, P,
                                       ctypes.c_int64, P]
        L.orc_fuse_contacts.restype = ctypes.c_int64
        L.orc_fuse_contacts.argtypes = [P, ctypes.c_int64, P, P]
        L.orc_broad_phase.restype = ctypes.c_int64
        L.orc_broad_phase.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_double, P, ctypes.c_int64, P, P]
        L.orc_toi_pairs.restype = ctypes.c_int64
        L.orc_toi_pairs.argtypes = [P, P, P, P, P, P, P, P, P, ctypes.c_int32, P,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_double, P, P,
                                    ctypes.c_int64, P]
        L.orc_mass_properties.restype = ctypes.c_int
        L.orc_mass_properties.argtypes = [P, P, ctypes.c_int32, P, P, P]
        L.orc_impulses.restype = ctypes.c_int32
        L.orc_impulses.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n
    return a


def tri_tri(A, B):
    """Distance of two triangles (3x3 vertex rows). Returns (d, pa, pb, feature)."""
    A, B = _f64(A, 9), _f64(B, 9)
    pa, pb = np.zeros(3), np.zeros(3)
    f = ctypes.c_int(-1)
    d = lib().orc_tri_tri(_p(A), _p(B), _p(pa), _p(pb), ctypes.byref(f))
    return d, pa, pb, f.value


def point_triangle(p, T):
    p, T = _f64(p, 3), _f64(T, 9)
    q = np.zeros(3)
    return lib().orc_point_triangle(_p(p), _p(T), _p(q)), q


def segment_segment(p1, q1, p2, q2):
    a = [_f64(x, 3) for x in (p1, q1, p2, q2)]
    c1, c2 = np.zeros(3), np.zeros(3)
    d = lib().orc_segment_segment(_p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), _p(c1), _p(c2))
    return d, c1, c2


def segment_triangle(p, q, T):
    p, q, T = _f64(p, 3), _f64(q, 3), _f64(T, 9)
    x = np.zeros(3)
    hit = lib().orc_segment_triangle(_p(p), _p(q), _p(T), _p(x))
    return bool(hit), x


def pose(state, t):
    """World rotation matrix (3x3) and position of a particle at time t."""
    s = _f64(state, 13)
    R, x = np.zeros(9), np.zeros(3)
    lib().orc_pose(_p(s), float(t), _p(R), _p(x))
    return R.reshape(3, 3), x


def world_tris(V, F, state, t=0.0):
    V, F = _f64(V), np.ascontiguousarray(F, dtype=np.int32)
    s = _f64(state, 13)
    out = np.zeros((F.shape[0], 9))
    lib().orc_world_tris(_p(V), _p(F), F.shape[0], _p(s), float(t), _p(out))
    return out


class _Flat:
    """Scene flattened into the arrays the C routines read."""

    def __init__(self, scene):
        Vs = [np.asarray(m[0], np.float64) for m in scene.meshes]
        Fs = [np.asarray(m[1], np.int32) for m in scene.meshes]
        self.V = np.ascontiguousarray(np.concatenate(Vs), dtype=np.float64)
        self.F = np.ascontiguousarray(np.concatenate(Fs), dtype=np.int32)
        self.voff = np.concatenate([[0], np.cumsum([v.shape[0] for v in Vs])[:-1]]).astype(np.int64)
        self.toff = np.concatenate([[0], np.cumsum([f.shape[0] for f in Fs])[:-1]]).astype(np.int64)
        self.tcount = np.array([f.shape[0] for f in Fs], dtype=np.int32)
        self.halo = np.ascontiguousarray(scene.halo, dtype=np.float64)
        self.radius = np.array([np.sqrt((v * v).sum(axis=1)).max() for v in Vs], dtype=np.float64)
        self.mesh_of = np.ascontiguousarray(scene.mesh_of, dtype=np.int32)
        self.state = np.ascontiguousarray(scene.state, dtype=np.float64)


def static_pairs(scene, pairs=None, t=0.0, cap=None):
    """Static query at time t over all triangle pairs of each particle pair.
    Returns (pair results (PAIR_DT), contacts (CONTACT_DT) in (pair, i, j) order)."""
    fl = _Flat(scene)
    pairs = np.ascontiguousarray(scene.pairs if pairs is None else pairs, dtype=np.int32)
    n = pairs.shape[0]
    out = np.zeros(max(n, 1), dtype=PAIR_DT)
    cap = 1 << 16 if cap is None else cap
    while True:
        con = np.zeros(max(cap, 1), dtype=CONTACT_DT)
        tot = lib().orc_static_pairs(_p(fl.V), _p(fl.F), _p(fl.voff), _p(fl.toff), _p(fl.tcount),
                                     _p(fl.halo), _p(fl.mesh_of), _p(fl.state), n, _p(pairs),
                                     float(t), _p(out), _p(con), cap)
        if tot <= cap:
            return out[:n], con[:tot]
        cap = int(tot)


def toi_pairs(scene, dt, S=64, tol_rel=1e-6, pairs=None, cap=None):
    """Earliest collision time stamp per particle pair over [0, dt].
    Returns (pair results, contacts at each pair's time stamp, diag dict)."""
    fl = _Flat(scene)
    pairs = np.ascontiguousarray(scene.pairs if pairs is None else pairs, dtype=np.int32)
    n = pairs.shape[0]
    out = np.zeros(max(n, 1), dtype=PAIR_DT)
    diag = np.zeros(2, dtype=np.int64)
    cap = 1 << 16 if cap is None else cap
    while True:
        con = np.zeros(max(cap, 1), dtype=CONTACT_DT)
        tot = lib().orc_toi_pairs(_p(fl.V), _p(fl.F), _p(fl.voff), _p(fl.toff), _p(fl.tcount),
                                  _p(fl.halo), _p(fl.radius), _p(fl.mesh_of), _p(fl.state), n,
                                  _p(pairs), float(dt), int(S), float(tol_rel), _p(out), _p(con),
                                  cap, _p(diag))
        if tot <= cap:
            return out[:n], con[:tot], dict(evals=int(diag[0]), grazes=int(diag[1]))
        cap = int(tot)


def tri_pair_toi(A, B, sa, sb, delta, L, dt, S=64, tol_rel=1e-6):
    """Time stamp of one body-frame triangle pair on two trajectories."""
    A, B = _f64(A, 9), _f64(B, 9)
    sa, sb = _f64(sa, 13), _f64(sb, 13)
    ev, gr = ctypes.c_int64(0), ctypes.c_int64(0)
    t = lib().orc_tri_pair_toi(_p(A), _p(B), _p(sa), _p(sb), float(delta), float(L), float(dt),
                               int(S), float(tol_rel) * float(dt), ctypes.byref(ev), ctypes.byref(gr))
    return t, dict(evals=ev.value, grazes=gr.value)


def broad_phase(x, v, r, dt=0.0):
    """Candidate pairs (positions a < b, ordered) and cluster labels (the
    smallest position of each particle's subgraph) of spheres of radius r
    moving from x with velocity v over [0, dt]: section 3's checks 1 and 2,
    then min-labelling. Returns (pairs int32 (m, 2), labels int32 (n,),
    sweeps)."""
    x, v, r = _f64(x), _f64(v), _f64(r)
    n = r.shape[0]
    cap = 1 << 16
    while True:
        out = np.zeros((max(cap, 1), 2), dtype=np.int32)
        lab = np.zeros(max(n, 1), dtype=np.int32)
        sw = ctypes.c_int32(0)
        m = lib().orc_broad_phase(int(n), _p(x), _p(v), _p(r), float(dt), _p(out), cap, _p(lab),
                                  ctypes.byref(sw))
        if m <= cap:
            return out[:m], lab[:n], sw.value
        cap = int(m)


def narrow_tri_pair(A, B, w_rel, delta):
    """One narrowing round for a triangle pair (world-frame start positions,
    B's displacement relative to A over the span): the earliest contact as a
    fraction of the span, or 2.0 when there is none."""
    A, B, w = _f64(A, 9), _f64(B, 9), _f64(w_rel, 3)
    return lib().orc_narrow_tri_pair(_p(A), _p(B), _p(w), float(delta))


def narrow_pairs(scene, dt, pairs=None, cap=None):
    """The paper's narrowing time stamp per particle pair (translation only).
    Returns (pair results, contacts at each pair's time, rounds per pair)."""
    fl = _Flat(scene)
    pairs = np.ascontiguousarray(scene.pairs if pairs is None else pairs, dtype=np.int32)
    n = pairs.shape[0]
    out = np.zeros(max(n, 1), dtype=PAIR_DT)
    rounds = np.zeros(max(n, 1), dtype=np.int32)
    cap = 1 << 16 if cap is None else cap
    while True:
        con = np.zeros(max(cap, 1), dtype=CONTACT_DT)
        tot = lib().orc_narrow_pairs(_p(fl.V), _p(fl.F), _p(fl.voff), _p(fl.toff), _p(fl.tcount),
                                     _p(fl.halo), _p(fl.mesh_of), _p(fl.state), n, _p(pairs), float(dt),
                                     _p(out), _p(con), cap, _p(rounds))
        if tot <= cap:
            return out[:n], con[:tot], rounds[:n]
        cap = int(tot)


def fuse_contacts(contacts, delta):
    """Fused contact records (section 5): contacts sorted by (pair, tri_a,
    tri_b) as the static and time-stamp queries return them; delta: the
    threshold of each pair. The `pad` field of a fused record counts its
    members."""
    c = np.ascontiguousarray(contacts, dtype=CONTACT_DT)
    d = _f64(delta)
    out = np.zeros(max(c.shape[0], 1), dtype=CONTACT_DT)
    m = lib().orc_fuse_contacts(_p(c), c.shape[0], _p(d), _p(out))
    return out[:m]


class _ImpulseOpts(ctypes.Structure):
    _fields_ = [("restitution", ctypes.c_double), ("friction", ctypes.c_double), ("relax", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("pad", ctypes.c_int32)]


def mass_properties(V, F):
    """Unit-density mass, centre of mass and inertia tensor about it (3x3) of
    a closed triangle mesh (section 6 needs the masses; divergence theorem)."""
    V = _f64(V)
    F = np.ascontiguousarray(F, dtype=np.int32)
    m = np.zeros(1)
    c = np.zeros(3)
    I = np.zeros(9)
    if lib().orc_mass_properties(_p(V), _p(F), F.shape[0], _p(m), _p(c), _p(I)) != 0:
        raise ValueError("mesh encloses no volume")
    return float(m[0]), c, I.reshape(3, 3)


def impulses(mass, com, inertia, states, ab, pa, pb, restitution=0.0, friction=0.0, relax=1.0, tol=1e-4,
             max_iter=100):
    """Impulses at a cluster's contact points and the particles' new
    velocities (section 6, Picard iteration over coloured contacts).
    mass (np,), com (np, 3) body frame, inertia (np, 3, 3) about the centre
    of mass in the body frame, states (np, 13); ab (nc, 2) local particle
    indices of each contact, pa/pb (nc, 3) its closest points (world).
    Returns (impulse (nc, 4): normal, tangential xyz; vel (np, 6): v, w;
    the most sweeps any cluster ran; colour of each contact). Clusters, the
    connected components of the contact graph, iterate independently."""
    mass = _f64(mass)
    np_ = mass.shape[0]
    com, inertia, states = _f64(com, 3 * np_), _f64(inertia, 9 * np_), _f64(states, 13 * np_)
    ab = np.ascontiguousarray(ab, dtype=np.int32).reshape(-1, 2)
    nc = ab.shape[0]
    pa, pb = _f64(pa, 3 * nc), _f64(pb, 3 * nc)
    o = _ImpulseOpts(restitution, friction, relax, tol, max_iter, 0)
    imp = np.zeros((max(nc, 1), 4))
    vel = np.zeros((max(np_, 1), 6))
    col = np.zeros(max(nc, 1), dtype=np.int32)
    it = lib().orc_impulses(np_, _p(mass), _p(com), _p(inertia), _p(states), nc, _p(ab), _p(pa), _p(pb),
                            ctypes.byref(o), _p(imp), _p(vel), _p(col))
    return imp[:nc], vel[:np_], int(it), col[:nc]
