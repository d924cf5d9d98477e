"""ctypes binding of include/mcd.h (argument marshalling only).

Every computation runs in libmcd.so on the GPU. The names follow the C calls:
Context.mesh_load -> mcd_mesh_load, Context.query_pairs -> mcd_query_pairs, ...
"""

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_LIB_PATH = os.path.join(_HERE, "libmcd.so")
_HEADER = os.path.join(_ROOT, "include", "mcd.h")

Q_FP64, Q_MIXED, Q_DENSE, Q_TIMING, Q_CLOSEST, Q_CONTACTS, Q_VALIDATE, Q_NARROW, Q_FUSE = (1, 2, 4, 8, 16, 32, 64,
                                                                                     128, 256)
Q_DEVICE_OUT = 512
CFG_NO_GRAPHS, CFG_NO_TUNE = 1, 2
NONE, AT_START, COLLIDES = 0, 1, 2
_STATUS = {0: "MCD_OK", -1: "MCD_E_INVALID", -2: "MCD_E_OOM", -3: "MCD_E_NOT_FOUND",
           -4: "MCD_E_BUSY", -5: "MCD_E_TIMEOUT", -6: "MCD_E_HIP"}

PAIR_RESULT_DT = np.dtype([("dmin", "<f8"), ("pa", "<f8", 3), ("pb", "<f8", 3), ("toi", "<f8"),
                           ("tri_a", "<i4"), ("tri_b", "<i4"), ("contact", "<i4"),
                           ("status", "<i4")])
CONTACT_DT = np.dtype([("pair", "<i4"), ("tri_a", "<i4"), ("tri_b", "<i4"), ("merged", "<i4"),
                       ("d", "<f8"), ("pa", "<f8", 3), ("pb", "<f8", 3), ("t", "<f8")])
STATS_DT = np.dtype([("tile_pairs_total", "<i8"), ("tile_pairs_kept", "<i8"),
                     ("tri_pairs_covered", "<i8"), ("tri_pairs_evaluated", "<i8"),
                     ("fp64_rechecks", "<i8"), ("refine_items", "<i8"), ("candidates", "<i8"),
                     ("fp64_evals", "<i8"), ("grazes", "<i8"), ("fp32_samples", "<i8"), ("retries", "<i8"),
                     ("gpu_ms", "<f8"), ("main_ms", "<f8"), ("latency_ms", "<f8"),
                     ("batch_queries", "<i4"), ("batch_pairs", "<i4"), ("tri_pairs_tiled", "<i8"),
                     ("sphere_tests", "<i8"), ("cull_ms", "<f8"), ("near_ms", "<f8"), ("sort_ms", "<f8"),
                     ("endgame_ms", "<f8"), ("submit_ms", "<f8"), ("near_pairs", "<i8"),
                     ("banded", "<i8"), ("validated", "<i8"), ("margin_ratio", "<f8"),
                     ("margin_ratio_np", "<f8"), ("cull_tests", "<i8"), ("graph_captures", "<i8"),
                     ("tune_pending", "<i4"), ("pad", "<i4")])


class MCDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, code), msg))
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("margin_c", ctypes.c_double), ("contact_cap", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


class _ImpulseOpts(ctypes.Structure):
    _fields_ = [("restitution", ctypes.c_double), ("friction", ctypes.c_double), ("relax", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _QOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("flags", ctypes.c_uint32), ("samples", ctypes.c_int32),
                ("tol_rel", ctypes.c_double)]


def lib_path():
    return _LIB_PATH


_lib = None


def load_library():
    """Load libmcd.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("libmcd.so is not built: run __graft_entry__.build() "
                           "(or python paper_2309_15417_amd/build.py)")
    L = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                           ctypes.c_double)
    sig = {
        "mcd_abi_version": (I32, []),
        "mcd_create": (I32, [P, P, P]),
        "mcd_destroy": (None, [P]),
        "mcd_last_error": (ctypes.c_char_p, [P]),
        "mcd_mesh_load": (I32, [P, P, I32, P, I32, D, P]),
        "mcd_mesh_unload": (I32, [P, I32]),
        "mcd_particles_set": (I32, [P, I32, P, P, P]),
        "mcd_query_pairs": (I32, [P, I32, P, P, P]),
        "mcd_query_pairs_dev": (I32, [P, I32, P, P, P, P]),
        "mcd_query_cluster": (I32, [P, I32, P, P, P, P]),
        "mcd_poll": (I32, [P, U64, P]),
        "mcd_wait": (I32, [P, U64, I64]),
        "mcd_result_sizes": (I32, [P, U64, P, P]),
        "mcd_fetch": (I32, [P, U64, P, I32, P, I64, P]),
        "mcd_result_view": (I32, [P, U64, P, P, P]),
        "mcd_fetch_dev": (I32, [P, U64, P, I32, P, I64, P]),
        "mcd_cluster_time": (I32, [P, U64, P]),
        "mcd_query_stats": (I32, [P, U64, P]),
        "mcd_release": (I32, [P, U64]),
        "mcd_broad_phase": (I32, [P, I32, P, D, P, P, P, I64, P]),
        "mcd_impulses": (I32, [P, I32, P, P, P, P, P, P, P, P]),
        "mcd_query_pairs_noalloc": (I32, [P, I32, P, P, P, P, I64, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


_quick = None
# Calls that return without blocking once a ticket is complete; through this
# handle they keep the GIL (no hand-over to a thread spinning on the clock).
_QUICK = ("mcd_poll", "mcd_result_sizes", "mcd_result_view", "mcd_query_stats", "mcd_release")


def _quick_library():
    global _quick
    if _quick is None:
        L = load_library()
        Q = ctypes.PyDLL(_LIB_PATH)
        for name in _QUICK:
            f, g = getattr(Q, name), getattr(L, name)
            f.restype, f.argtypes = g.restype, g.argtypes
        _quick = Q
    return _quick


def header_symbols():
    """Function names declared in include/mcd.h."""
    txt = open(_HEADER).read()
    return sorted(set(re.findall(r"\b(mcd_[a-z_]+)\s*\(", txt)))


def exported_symbols():
    L = ctypes.CDLL(_LIB_PATH)
    return [s for s in header_symbols() if hasattr(L, s)]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """One library context on the current HIP device (see mcd_create)."""

    def __init__(self, mem_budget=0, streams=0, margin_c=0.0, contact_cap=0, stream=None, flags=0,
                 tune_cache=None):
        self._L = load_library()
        self._Q = _quick_library()
        cfg = _Config(mem_budget, streams, margin_c, contact_cap, flags,
                      tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        st = self._L.mcd_create(ctypes.byref(cfg), ctypes.c_void_p(stream or 0), ctypes.byref(h))
        if st != 0:
            raise MCDError(st, self._L.mcd_last_error(None).decode())
        self._h = h
        self._scene_pids = None

    def close(self):
        if getattr(self, "_h", None):
            self._L.mcd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != 0:
            raise MCDError(st, self._L.mcd_last_error(self._h).decode())

    # -- stores
    def mesh_load(self, V, F, eps):
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        mid = ctypes.c_int32(-1)
        self._check(self._L.mcd_mesh_load(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0],
                                          float(eps), ctypes.byref(mid)))
        return mid.value

    def mesh_unload(self, mesh_id):
        self._check(self._L.mcd_mesh_unload(self._h, int(mesh_id)))

    def particles_set(self, pid, mesh_id, states):
        pid = np.ascontiguousarray(pid, dtype=np.int32)
        mesh_id = np.ascontiguousarray(mesh_id, dtype=np.int32)
        states = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 13)
        self._check(self._L.mcd_particles_set(self._h, pid.shape[0], _ptr(pid), _ptr(mesh_id),
                                              _ptr(states)))

    def load_scene(self, scene):
        """Load a synthetic scene's meshes and particles (particle id = index)."""
        ids = [self.mesh_load(V, F, scene.halo[k]) for k, (V, F) in enumerate(scene.meshes)]
        ids = np.asarray(ids, dtype=np.int32)
        n = scene.n_particles
        self.particles_set(np.arange(n, dtype=np.int32), ids[scene.mesh_of], scene.state)
        return ids

    # -- queries
    def query_pairs(self, pairs, dt=0.0, flags=0, samples=0, tol_rel=0.0):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        o = _QOpts(float(dt), int(flags), int(samples), float(tol_rel))
        t = ctypes.c_uint64(0)
        self._check(self._L.mcd_query_pairs(self._h, pairs.shape[0], _ptr(pairs), ctypes.byref(o),
                                            ctypes.byref(t)))
        return t.value

    def query_pairs_dev(self, d_pairs_ptr, n, dt=0.0, flags=0, samples=0, tol_rel=0.0, stream=None):
        o = _QOpts(float(dt), int(flags), int(samples), float(tol_rel))
        t = ctypes.c_uint64(0)
        self._check(self._L.mcd_query_pairs_dev(self._h, int(n), ctypes.c_void_p(d_pairs_ptr),
                                                ctypes.byref(o), ctypes.c_void_p(stream or 0),
                                                ctypes.byref(t)))
        return t.value

    def query_pairs_noalloc(self, d_pairs_ptr, n, d_results_ptr, d_contacts_ptr, cap_contacts, stream=None):
        """mcd_query_pairs_noalloc: device pointers in, device records out;
        returns the contact count."""
        m = ctypes.c_int64(0)
        self._check(self._L.mcd_query_pairs_noalloc(self._h, int(n), ctypes.c_void_p(d_pairs_ptr),
                                                    ctypes.c_void_p(stream or 0), ctypes.c_void_p(d_results_ptr),
                                                    ctypes.c_void_p(d_contacts_ptr), int(cap_contacts),
                                                    ctypes.byref(m)))
        return m.value

    def query_cluster(self, pids, states=None, dt=0.0, flags=0, samples=0, tol_rel=0.0):
        pids = np.ascontiguousarray(pids, dtype=np.int32)
        sp = None
        if states is not None:
            states = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 13)
            sp = _ptr(states)
        o = _QOpts(float(dt), int(flags), int(samples), float(tol_rel))
        t = ctypes.c_uint64(0)
        self._check(self._L.mcd_query_cluster(self._h, pids.shape[0], _ptr(pids), sp,
                                              ctypes.byref(o), ctypes.byref(t)))
        return t.value

    def broad_phase(self, pids, dt=0.0, clusters=True, pairs=True):
        """Candidate pairs (particle ids) and clusters of a particle set
        (mcd_broad_phase). Returns (cluster per particle or None, cluster
        count, pairs (m, 2) or None)."""
        pids = np.ascontiguousarray(pids, dtype=np.int32)
        n = pids.shape[0]
        lab = np.zeros(max(n, 1), np.int32) if clusters else None
        k = ctypes.c_int32(0)
        m = ctypes.c_int64(0)
        self._check(self._L.mcd_broad_phase(self._h, n, _ptr(pids), float(dt),
                                            _ptr(lab) if clusters else None, ctypes.byref(k),
                                            None, 0, ctypes.byref(m)))
        out = None
        if pairs:
            out = np.zeros((max(m.value, 1), 2), np.int32)
            self._check(self._L.mcd_broad_phase(self._h, n, _ptr(pids), float(dt), None, None,
                                                _ptr(out), out.shape[0], ctypes.byref(m)))
            out = out[:m.value]
        return (lab[:n] if clusters else None), k.value, out

    def poll(self, ticket):
        d = ctypes.c_int32(0)
        self._check(self._L.mcd_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket, timeout_ns=-1):
        self._check(self._L.mcd_wait(self._h, ctypes.c_uint64(ticket), int(timeout_ns)))

    def _complete(self, ticket):
        """Block (without the GIL) until the ticket is complete."""
        d = ctypes.c_int32(0)
        self._check(self._Q.mcd_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        if not d.value:
            self.wait(ticket)

    def result_sizes(self, ticket):
        self._complete(ticket)
        n, c = ctypes.c_int32(0), ctypes.c_int64(0)
        self._check(self._Q.mcd_result_sizes(self._h, ctypes.c_uint64(ticket), ctypes.byref(n),
                                             ctypes.byref(c)))
        return n.value, c.value

    def fetch(self, ticket, with_pairs=False, out=None, contacts=True):
        """Returns (pair results, contacts[, pair particle ids]). `out` may be a
        dict of arrays from an earlier fetch; they are reused when large
        enough (the returned arrays are views of them). contacts=False skips
        the records (required for Q_DEVICE_OUT tickets; None is returned)."""
        self.wait(ticket)
        n, nc = self.result_sizes(ticket)
        out = {} if out is None else out
        if not contacts:
            pr = np.empty(max(n, 1), dtype=PAIR_RESULT_DT)
            pp = np.empty((max(n, 1), 2), dtype=np.int32)
            self._check(self._L.mcd_fetch(self._h, ctypes.c_uint64(ticket), _ptr(pr), pr.shape[0],
                                          None, 0, _ptr(pp)))
            return (pr[:n], None, pp[:n]) if with_pairs else (pr[:n], None)

        def buf(name, shape, dtype):
            a = out.get(name)
            if a is None or a.shape[0] < shape[0]:
                a = np.empty((int(shape[0] * 1.25) + 1,) + shape[1:], dtype=dtype)
                out[name] = a
            return a

        pr = buf("pr", (max(n, 1),), PAIR_RESULT_DT)
        con = buf("con", (max(nc, 1),), CONTACT_DT)
        pp = buf("pp", (max(n, 1), 2), np.int32)
        self._check(self._L.mcd_fetch(self._h, ctypes.c_uint64(ticket), _ptr(pr), pr.shape[0],
                                      _ptr(con), con.shape[0], _ptr(pp)))
        if with_pairs:
            return pr[:n], con[:nc], pp[:n]
        return pr[:n], con[:nc]

    def view(self, ticket, with_pairs=False):
        """mcd_result_view: (pair results, contacts[, pair ids]) as arrays over
        the library's own host memory, without a copy. They are valid until
        release(ticket) or close(); contacts is None when the records are not
        on the host."""
        n, nc = self.result_sizes(ticket)
        p_pr, p_con, p_pp = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        self._check(self._Q.mcd_result_view(self._h, ctypes.c_uint64(ticket), ctypes.byref(p_pr),
                                            ctypes.byref(p_con), ctypes.byref(p_pp)))

        def arr(ptr, count, dtype, shape):
            if not ptr.value or count == 0:
                return np.empty(shape, dtype=dtype)
            buf = (ctypes.c_char * (count * np.dtype(dtype).itemsize)).from_address(ptr.value)
            return np.frombuffer(buf, dtype=dtype).reshape(shape)

        pr = arr(p_pr, n, PAIR_RESULT_DT, (n,))
        con = None if (nc > 0 and not p_con.value) else arr(p_con, nc, CONTACT_DT, (nc,))
        if with_pairs:
            return pr, con, arr(p_pp, 2 * n, np.int32, (n, 2))
        return pr, con

    def fetch_dev(self, ticket, d_pr_ptr, cap_pairs, d_con_ptr, cap_contacts, stream=None):
        """mcd_fetch_dev: a Q_DEVICE_OUT ticket's results copied into device
        memory (pointers, e.g. torch tensors' data_ptr()) on `stream`."""
        self._check(self._L.mcd_fetch_dev(self._h, ctypes.c_uint64(ticket), ctypes.c_void_p(d_pr_ptr or 0),
                                          int(cap_pairs), ctypes.c_void_p(d_con_ptr or 0), int(cap_contacts),
                                          ctypes.c_void_p(stream or 0)))

    def impulses(self, pid_pairs, contacts, restitution=0.0, friction=0.0, relax=1.0, tol=1e-4, max_iter=100):
        """mcd_impulses: the particle interaction solve over contact records
        (their pa and pb) joining the particles pid_pairs[k]. Returns
        (impulse (n, 4): normal, tangential xyz on b; particle ids;
        new velocities (np, 6): v, w; sweeps run)."""
        pp = np.ascontiguousarray(pid_pairs, dtype=np.int32).reshape(-1, 2)
        con = np.ascontiguousarray(contacts, dtype=CONTACT_DT)
        n = pp.shape[0]
        if con.shape[0] != n:
            raise ValueError("one contact record per particle pair")
        o = _ImpulseOpts(float(restitution), float(friction), float(relax), float(tol), int(max_iter), 0)
        imp = np.zeros((max(n, 1), 4))
        pids = np.zeros(max(2 * n, 1), dtype=np.int32)
        vel = np.zeros((max(2 * n, 1), 6))
        k, sw = ctypes.c_int32(0), ctypes.c_int32(0)
        self._check(self._L.mcd_impulses(self._h, n, _ptr(pp), _ptr(con), ctypes.byref(o), _ptr(imp),
                                         ctypes.byref(k), _ptr(pids), _ptr(vel), ctypes.byref(sw)))
        return imp[:n], pids[:k.value], vel[:k.value], sw.value

    def cluster_time(self, ticket):
        t = ctypes.c_double(0)
        self._check(self._L.mcd_cluster_time(self._h, ctypes.c_uint64(ticket), ctypes.byref(t)))
        return t.value

    def stats(self, ticket, raw=False):
        """mcd_query_stats as a dict, or (raw=True) as the STATS_DT record."""
        self._complete(ticket)
        s = np.zeros(1, dtype=STATS_DT)
        self._check(self._Q.mcd_query_stats(self._h, ctypes.c_uint64(ticket), _ptr(s)))
        if raw:
            return s[0]
        return {k: s[k][0].item() for k in STATS_DT.names}

    def release(self, ticket):
        self._check(self._Q.mcd_release(self._h, ctypes.c_uint64(ticket)))
