"""Closed triangle meshes in the body frame (rotation centre at the origin)."""

import math

import numpy as np


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return v, f


def icosphere(subdiv, radius=1.0):
    """Icosahedron refined `subdiv` times by edge midpoints, projected on the
    sphere. Returns (V, F) with V float64 (10*4^s+2, 3), F int32 (20*4^s, 3),
    faces wound counter-clockwise seen from outside."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(int(subdiv)):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = np.add(verts[a], verts[b]) * 0.5
                m /= np.linalg.norm(m)
                verts.append(tuple(m))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int32)
    V = np.array(verts, dtype=np.float64) * radius
    return V, np.ascontiguousarray(f, dtype=np.int32)


def uv_sphere_size(T):
    """(m segments, k interior latitude rings) for a UV sphere of about T
    triangles: k = max(2, round(sqrt(T/4))), m = max(3, round(T/(2k))), so the
    mesh has exactly 2*m*k triangles."""
    k = max(2, int(round(math.sqrt(T / 4.0))))
    m = max(3, int(round(T / (2.0 * k))))
    return m, k


def uv_sphere(T, radius=1.0):
    """Closed UV sphere: two triangle-fan caps and k-1 quad bands between k
    interior latitude rings of m vertices each; 2*m*k triangles, all vertices
    on the sphere of the given radius."""
    m, k = uv_sphere_size(T)
    V = [(0.0, 0.0, radius)]
    for i in range(1, k + 1):
        th = math.pi * i / (k + 1)
        for j in range(m):
            ph = 2.0 * math.pi * j / m
            V.append((radius * math.sin(th) * math.cos(ph),
                      radius * math.sin(th) * math.sin(ph),
                      radius * math.cos(th)))
    V.append((0.0, 0.0, -radius))
    south = len(V) - 1

    def ring(i, j):
        return 1 + (i - 1) * m + (j % m)

    F = []
    for j in range(m):
        F.append((0, ring(1, j), ring(1, j + 1)))
    for i in range(1, k):
        for j in range(m):
            a, b = ring(i, j), ring(i, j + 1)
            c, d = ring(i + 1, j), ring(i + 1, j + 1)
            F.append((a, c, d))
            F.append((a, d, b))
    for j in range(m):
        F.append((south, ring(k, j + 1), ring(k, j)))
    return np.array(V, dtype=np.float64), np.array(F, dtype=np.int32)


def perturb_radial(V, rng, amp=0.1):
    """Scale each vertex's distance from the centre by 1 + U[-amp, amp]."""
    s = 1.0 + rng.uniform(-amp, amp, size=(V.shape[0], 1))
    return V * s


def mesh_radius(V):
    """Largest vertex distance from the body-frame origin."""
    return float(np.sqrt((V * V).sum(axis=1)).max())
