"""Seeded scenes: particles (mesh id + rigid state), halos and candidate pairs.

State layout per particle (13 float64): x[3] centre of rotation in the world
frame, q[4] unit quaternion (w, x, y, z) taking body to world, v[3] linear
velocity, w[3] angular velocity (world frame). Seeds follow
``config index * 1000 + run``.
"""

import dataclasses
import functools
import math

import numpy as np
from scipy.spatial import cKDTree

from .meshes import icosphere, uv_sphere, perturb_radial, mesh_radius


@dataclasses.dataclass
class Scene:
    meshes: list            # [(V float64 (nv,3), F int32 (nt,3))] body frame
    halo: np.ndarray        # float64 per mesh: halo width eps
    mesh_of: np.ndarray     # int32 per particle
    state: np.ndarray       # float64 (n, 13)
    pairs: np.ndarray       # int32 (npairs, 2) candidate particle pairs
    dt: float = 0.0         # step length (0 for static queries)
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_particles(self):
        return int(self.mesh_of.shape[0])

    def tri_counts(self):
        return np.array([m[1].shape[0] for m in self.meshes], dtype=np.int64)

    def dense_tri_pairs(self, pairs=None):
        """Number of triangle pairs spanned by the given particle pairs."""
        p = self.pairs if pairs is None else pairs
        nt = self.tri_counts()[self.mesh_of]
        return int((nt[p[:, 0]] * nt[p[:, 1]]).sum())


def random_quaternions(n, rng):
    """Uniform random unit quaternions (Shoemake's subgroup method), (w,x,y,z)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], axis=1)
    return q


def random_unit_vectors(n, rng):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _state(x, q, v=None, w=None):
    n = x.shape[0]
    s = np.zeros((n, 13), dtype=np.float64)
    s[:, 0:3] = x
    s[:, 3:7] = q
    if v is not None:
        s[:, 7:10] = v
    if w is not None:
        s[:, 10:13] = w
    return s


def relax_packing(n, radius, phi, rng, max_iter=20000):
    """Centres of n equal spheres in a cube at volume fraction phi: uniform
    random start, then repeated pairwise push-apart of overlapping spheres
    (each moved by half the overlap plus a small excess, walls clamp) until no
    two spheres overlap. Returns (centres (n,3), cube side)."""
    side = (n * 4.0 / 3.0 * math.pi * radius ** 3 / phi) ** (1.0 / 3.0)
    x = rng.uniform(radius, side - radius, size=(n, 3))
    d0 = 2.0 * radius
    for _ in range(max_iter):
        tree = cKDTree(x)
        pr = tree.query_pairs(d0, output_type="ndarray")
        if pr.shape[0] == 0:
            break
        a, b = pr[:, 0], pr[:, 1]
        dv = x[b] - x[a]
        dist = np.linalg.norm(dv, axis=1)
        dist = np.maximum(dist, 1e-12)
        push = (d0 - dist) * 0.5 * 1.02 + 1e-9
        u = dv / dist[:, None]
        dx = np.zeros_like(x)
        np.add.at(dx, a, -u * push[:, None])
        np.add.at(dx, b, u * push[:, None])
        x = np.clip(x + dx, radius, side - radius)
    else:
        raise RuntimeError("relax_packing did not converge")
    return x, side


def rsa_packing(n, radius, phi, rng, max_attempts=None):
    """Random sequential addition of n equal spheres in a cube at volume
    fraction phi (valid below the RSA jamming limit, about 0.38)."""
    side = (n * 4.0 / 3.0 * math.pi * radius ** 3 / phi) ** (1.0 / 3.0)
    cell = 2.0 * radius
    nc = max(1, int(side // cell))
    cell = side / nc
    grid = {}
    pts = np.zeros((n, 3))
    k = 0
    attempts = 0
    max_attempts = max_attempts or 2000 * n
    d2 = (2.0 * radius) ** 2
    while k < n:
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError("rsa_packing: too many attempts")
        p = rng.uniform(radius, side - radius, size=3)
        c = tuple(np.minimum((p // cell).astype(int), nc - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                        q = pts[j]
                        if (p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2 + (p[2] - q[2]) ** 2 < d2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[k] = p
            grid.setdefault(c, []).append(k)
            k += 1
    return pts, side


def sphere_pairs(x, R, delta, v=None, dt=0.0):
    """Candidate particle pairs from bounding spheres (centre x, radius R about
    the rotation centre, so rotation never changes them): static,
    |x_a - x_b| <= R_a + R_b + delta; moving (v, dt given), the centres move on
    straight lines and the pair is kept when their closest approach over
    [0, dt] satisfies the same bound. Returns int32 (m, 2) with a < b, sorted."""
    R = np.asarray(R, dtype=np.float64)
    reach = 2.0 * R.max() + delta
    if v is not None and dt > 0:
        reach += 2.0 * np.linalg.norm(v, axis=1).max() * dt
    tree = cKDTree(x)
    pr = tree.query_pairs(reach, output_type="ndarray")
    if pr.shape[0] == 0:
        return np.zeros((0, 2), dtype=np.int32)
    a, b = pr[:, 0], pr[:, 1]
    lim = R[a] + R[b] + delta
    dx = x[b] - x[a]
    if v is not None and dt > 0:
        dv = v[b] - v[a]
        vv = (dv * dv).sum(axis=1)
        t = np.where(vv > 0, -(dx * dv).sum(axis=1) / np.where(vv > 0, vv, 1.0), 0.0)
        t = np.clip(t, 0.0, dt)
        dx = dx + dv * t[:, None]
    keep = np.sqrt((dx * dx).sum(axis=1)) <= lim
    out = np.stack([a[keep], b[keep]], axis=1).astype(np.int32)
    out.sort(axis=1)
    order = np.lexsort((out[:, 1], out[:, 0]))
    return np.ascontiguousarray(out[order])


@functools.lru_cache(maxsize=None)
def _ico(s):
    return icosphere(s)


@functools.lru_cache(maxsize=None)
def _uv(T):
    return uv_sphere(T)


def cfg1_scene(run=0, n_pairs=16, subdiv=2, eps=0.01, gap_max=0.02):
    """16 pairs of icospheres (subdivision 2, 320 triangles, radius 1), each
    particle uniformly rotated; B's centre at A's + (2 + g) u with u uniform
    on the sphere and g ~ U[0, gap_max]. Pairs sit 10 apart on the x axis."""
    rng = np.random.default_rng(1 * 1000 + run)
    V, F = _ico(subdiv)
    n = 2 * n_pairs
    q = random_quaternions(n, rng)
    u = random_unit_vectors(n_pairs, rng)
    g = rng.uniform(0.0, gap_max, size=n_pairs)
    x = np.zeros((n, 3))
    x[0::2, 0] = 10.0 * np.arange(n_pairs)
    x[1::2] = x[0::2] + (2.0 + g)[:, None] * u
    pairs = np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], axis=1).astype(np.int32)
    return Scene(meshes=[(V, F)], halo=np.array([eps]), mesh_of=np.zeros(n, np.int32),
                 state=_state(x, q), pairs=pairs,
                 info=dict(name="cfg1", gaps=g, eps=eps))


def _perturbed_particles(rng, subdivs, amp=0.1):
    meshes = []
    for s in subdivs:
        V, F = _ico(int(s))
        meshes.append((perturb_radial(V, rng, amp), F))
    return meshes


def cfg2_scene(run=0, n=2000, phi=0.55, eps=0.005, pack_r=1.0, subdivs=(1, 2, 3, 4)):
    """Static packing: n perturbed icospheres (subdivision uniform over
    `subdivs`, vertex radii scaled by 1+U[-0.1,0.1]), centres from a relaxation
    packing of spheres of radius pack_r at volume fraction phi. The default
    pack_r = 1 packs on the nominal radius (phi is the solid fraction):
    neighbours touch through their bumps and interpenetrate by up to 0.2.
    pack_r = 1.1 packs on the largest possible vertex radius, so no two
    bounding spheres overlap and no particles interpenetrate; neighbours
    then come within the halo only where both meshes have a vertex at the
    very top of the perturbation range, which at eps = 0.005 leaves no
    triangle pair in contact. Candidate pairs from a uniform-grid test on the
    meshes' bounding spheres with delta = 2 eps."""
    rng = np.random.default_rng(2 * 1000 + run)
    s = rng.choice(np.asarray(subdivs), size=n)
    meshes = _perturbed_particles(rng, s)
    x, side = relax_packing(n, pack_r, phi, rng)
    q = random_quaternions(n, rng)
    R = np.array([mesh_radius(m[0]) for m in meshes])
    pairs = sphere_pairs(x, R, 2 * eps)
    return Scene(meshes=meshes, halo=np.full(n, eps), mesh_of=np.arange(n, dtype=np.int32),
                 state=_state(x, q), pairs=pairs,
                 info=dict(name="cfg2", side=side, subdiv=s, eps=eps, pack_r=pack_r))


def cfg3_scene(run=0, n_pairs=4096, tmin=20, tmax=5120, eps=0.005):
    """Uneven pair queries: per pair two UV spheres (radius 1) whose triangle
    counts are log-uniform in [tmin, tmax], uniformly rotated, centres
    2 + g apart with g ~ U[0, 2 eps]; meshes of equal size are shared."""
    rng = np.random.default_rng(3 * 1000 + run)
    T = np.exp(rng.uniform(math.log(tmin), math.log(tmax), size=2 * n_pairs))
    meshes, ids, mesh_of = [], {}, np.zeros(2 * n_pairs, np.int32)
    for i, t in enumerate(T):
        V, F = _uv(int(round(t)))
        key = F.shape[0]
        if key not in ids:
            ids[key] = len(meshes)
            meshes.append((V, F))
        mesh_of[i] = ids[key]
    n = 2 * n_pairs
    q = random_quaternions(n, rng)
    u = random_unit_vectors(n_pairs, rng)
    g = rng.uniform(0.0, 2 * eps, size=n_pairs)
    x = np.zeros((n, 3))
    x[0::2, 0] = 10.0 * (np.arange(n_pairs) % 64)
    x[0::2, 1] = 10.0 * (np.arange(n_pairs) // 64)
    x[1::2] = x[0::2] + (2.0 + g)[:, None] * u
    pairs = np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], axis=1).astype(np.int32)
    return Scene(meshes=meshes, halo=np.full(len(meshes), eps), mesh_of=mesh_of,
                 state=_state(x, q), pairs=pairs, info=dict(name="cfg3", gaps=g, eps=eps))


def cfg4_scene(run=0, n=10000, phi=0.30, eps=0.005, bound_r=1.1, subdivs=(2, 3),
               v_sigma=1.0, w_sigma=5.0, target=0.05, dt=None, proxy_r=1.045):
    """Moving particles: n perturbed icospheres (subdivision 2 or 3) placed by
    random sequential addition at fraction phi on bounding radius 1.1,
    v ~ N(0, v_sigma^2) per component, w ~ N(0, w_sigma^2) rad/s. Unless dt is
    given, dt is bisected so that about `target` of the swept-sphere candidate
    pairs would bring spheres of radius proxy_r into contact. proxy_r = 1.045
    (between the nominal radius 1 and the bounding radius 1.1) makes the
    fraction of candidate pairs whose meshes collide about 5% for the default
    parameters (the spinning bumps reach beyond the nominal sphere)."""
    rng = np.random.default_rng(4 * 1000 + run)
    s = rng.choice(np.asarray(subdivs), size=n)
    meshes = _perturbed_particles(rng, s)
    x, side = rsa_packing(n, bound_r, phi, rng)
    q = random_quaternions(n, rng)
    v = rng.normal(0.0, v_sigma, size=(n, 3))
    w = rng.normal(0.0, w_sigma, size=(n, 3))
    R = np.array([mesh_radius(m[0]) for m in meshes])
    delta = 2 * eps

    def proxy_fraction(t):
        pr = sphere_pairs(x, R, delta, v=v, dt=t)
        if pr.shape[0] == 0:
            return 0.0, pr
        a, b = pr[:, 0], pr[:, 1]
        dx, dv = x[b] - x[a], v[b] - v[a]
        vv = (dv * dv).sum(axis=1)
        tc = np.clip(np.where(vv > 0, -(dx * dv).sum(axis=1) / np.where(vv > 0, vv, 1), 0), 0, t)
        dmin = np.linalg.norm(dx + dv * tc[:, None], axis=1)
        d0 = np.linalg.norm(dx, axis=1)
        hit = (d0 > 2.0 * proxy_r + delta) & (dmin <= 2.0 * proxy_r + delta)
        return float(hit.mean()), pr

    if dt is None:
        lo, hi = 1e-5, 1.0
        for _ in range(40):
            mid = math.sqrt(lo * hi)
            f, _ = proxy_fraction(mid)
            if f < target:
                lo = mid
            else:
                hi = mid
        dt = hi
    frac, pairs = proxy_fraction(dt)
    return Scene(meshes=meshes, halo=np.full(n, eps), mesh_of=np.arange(n, dtype=np.int32),
                 state=_state(x, q, v, w), pairs=pairs, dt=float(dt),
                 info=dict(name="cfg4", side=side, subdiv=s, eps=eps, proxy_fraction=frac))


def cfg5_scene(run=0, n=100000, phi=0.55, eps=0.005, pack_r=1.0, subdivs=(1, 2, 3),
               mesh_pool=4096, block=2000):
    """Serving population: n resident perturbed icospheres (subdivision 1-3,
    80-1,280 triangles). Centres: a relaxation packing of `block` spheres of
    the nominal radius at solid fraction phi in a cube (as in cfg2_scene),
    repeated on a grid of cubes
    until n particles are placed (a packing of 100,000 directly takes minutes
    to relax). Each particle draws its mesh from `mesh_pool` distinct perturbed
    meshes and gets its own uniform rotation."""
    rng = np.random.default_rng(5 * 1000 + run)
    npool = int(mesh_pool)
    s = rng.choice(np.asarray(subdivs), size=npool)
    meshes = _perturbed_particles(rng, s)
    xb, side = relax_packing(block, pack_r, phi, rng)
    nblk = -(-n // block)
    g = int(math.ceil(nblk ** (1.0 / 3.0)))
    cells = [(i, j, k) for i in range(g) for j in range(g) for k in range(g)][:nblk]
    x = np.concatenate([xb + side * np.array(c, dtype=np.float64) for c in cells])[:n]
    mesh_of = rng.integers(0, npool, size=n).astype(np.int32)
    q = random_quaternions(n, rng)
    return Scene(meshes=meshes, halo=np.full(npool, eps), mesh_of=mesh_of,
                 state=_state(x, q), pairs=np.zeros((0, 2), np.int32),
                 info=dict(name="cfg5", side=side * g, eps=eps, block=block))


def cluster_sizes(n_queries, rng, alpha=1.5, nmin=1, nmax=2000):
    """Discrete power law P(n) ~ n^-alpha on [nmin, nmax]."""
    k = np.arange(nmin, nmax + 1)
    p = k.astype(np.float64) ** (-alpha)
    p /= p.sum()
    return rng.choice(k, size=n_queries, p=p)


def cluster_members(x, seeds, sizes):
    """Each cluster = its seed particle and the size-1 nearest others."""
    tree = cKDTree(x)
    out = []
    for s, m in zip(seeds, sizes):
        _, idx = tree.query(x[s], k=int(m))
        out.append(np.atleast_1d(idx).astype(np.int32))
    return out


def pair_test_scene(meshA, meshB, stateA, stateB, epsA, epsB=None):
    """One particle pair from explicit meshes and states (tests)."""
    epsB = epsA if epsB is None else epsB
    st = np.stack([np.asarray(stateA, np.float64), np.asarray(stateB, np.float64)])
    if st.shape[1] == 7:
        st = np.concatenate([st, np.zeros((2, 6))], axis=1)
    return Scene(meshes=[meshA, meshB], halo=np.array([epsA, epsB]),
                 mesh_of=np.array([0, 1], np.int32), state=st,
                 pairs=np.array([[0, 1]], np.int32))
