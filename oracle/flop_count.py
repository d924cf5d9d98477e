"""Floating-point operation count of one triangle-pair evaluation in the
oracle's own formulation (the unit C_full that the benchmark's roofline
figures use).

The oracle's distance routines (closest point on a triangle, segment-segment
closest points, segment-triangle intersection and the triangle-triangle
distance that combines them) are taken verbatim from mcd_oracle.c and
compiled as C++ with `double` replaced by a number type that counts its
additions, multiplications, divisions and square roots; comparisons and
selects are not counted, and the oracle is built without contraction, so an
FMA never occurs (it would count 2). The count depends on the geometry
(Voronoi regions, clamping, early exit on intersection), so it is averaged
over every triangle pair of a seeded sample of candidate particle pairs of
the 2,000-particle static packing (the oracle's dense workload), and over
the near pairs among them (triangle spheres within the threshold) separately.

Test infrastructure, like the rest of oracle/. Run: python oracle/flop_count.py
"""

import os
import re
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

COUNTER = r'''
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <vector>
static long long n_add, n_mul, n_div, n_sqrt;
struct Flop {
    double v;
    Flop() : v(0) {}
    Flop(double x) : v(x) {}
};
static inline Flop operator+(Flop a, Flop b) { ++n_add; return Flop(a.v + b.v); }
static inline Flop operator-(Flop a, Flop b) { ++n_add; return Flop(a.v - b.v); }
static inline Flop operator*(Flop a, Flop b) { ++n_mul; return Flop(a.v * b.v); }
static inline Flop operator/(Flop a, Flop b) { ++n_div; return Flop(a.v / b.v); }
static inline Flop operator-(Flop a) { return Flop(-a.v); }
static inline bool operator<(Flop a, Flop b) { return a.v < b.v; }
static inline bool operator>(Flop a, Flop b) { return a.v > b.v; }
static inline bool operator<=(Flop a, Flop b) { return a.v <= b.v; }
static inline bool operator>=(Flop a, Flop b) { return a.v >= b.v; }
static inline Flop sqrt(Flop a) { ++n_sqrt; return Flop(std::sqrt(a.v)); }
static inline Flop fabs(Flop a) { return Flop(std::fabs(a.v)); }
#define double Flop
#define ORC_ABI 1
'''

MAIN = r'''
#undef double
int main(int argc, char** argv)
{
    FILE* f = std::fopen(argv[1], "rb");
    long long n = 0;
    if (std::fread(&n, sizeof n, 1, f) != 1) return 1;
    std::vector<double> buf((size_t)n * 18);
    if (std::fread(buf.data(), sizeof(double), buf.size(), f) != buf.size()) return 1;
    std::fclose(f);
    std::vector<Flop> A(9), B(9), pa(3), pb(3);
    long long hits = 0;
    for (long long k = 0; k < n; ++k) {
        for (int i = 0; i < 9; ++i) { A[i] = Flop(buf[18 * k + i]); B[i] = Flop(buf[18 * k + 9 + i]); }
        int feat = -1;
        Flop d = orc_tri_tri(A.data(), B.data(), pa.data(), pb.data(), &feat);
        hits += (d.v == 0.0);
    }
    std::printf("%lld %lld %lld %lld %lld %lld\n", n, n_add, n_mul, n_div, n_sqrt, hits);
    return 0;
}
'''


def oracle_distance_source():
    """The oracle's distance routines, verbatim: from the 3-vector type to
    the end of the triangle-triangle distance."""
    src = open(os.path.join(HERE, "mcd_oracle.c")).read()
    a = src.index("typedef struct { double x, y, z; } v3;")
    b = src.index("/* Exposed primitives")
    return src[a:b]


def build(tmp):
    cpp = os.path.join(tmp, "flop_count.cpp")
    with open(cpp, "w") as f:
        f.write(COUNTER + oracle_distance_source() + MAIN)
    exe = os.path.join(tmp, "flop_count")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-w", "-o", exe, cpp])
    return exe


def count(exe, tris, tmp):
    path = os.path.join(tmp, "pairs.bin")
    with open(path, "wb") as f:
        np.array([tris.shape[0]], np.int64).tofile(f)
        np.ascontiguousarray(tris, np.float64).tofile(f)
    out = subprocess.check_output([exe, path], text=True).split()
    n, add, mul, div, sq, hits = (int(x) for x in out)
    return dict(pairs=n, add=add / n, mul=mul / n, div=div / n, sqrt=sq / n,
                flops=(add + mul + div + sq) / n, intersecting=hits / n)


def sample_triangle_pairs(n_pairs=24, max_tri_pairs=400000, seed=2000):
    """Every triangle pair (world frame) of n_pairs seeded candidate pairs of
    the static packing, subsampled to max_tri_pairs; and the near pairs among
    all of them (triangle bounding spheres within the threshold)."""
    sys.path.insert(0, ROOT)
    import oracle
    import synth
    sc = synth.cfg2_scene(run=0)
    rng = np.random.default_rng(seed)
    idx = rng.choice(sc.pairs.shape[0], size=n_pairs, replace=False)
    allp, near = [], []
    for p in idx:
        ia, ib = sc.pairs[p]
        Va, Fa = sc.meshes[sc.mesh_of[ia]]
        Vb, Fb = sc.meshes[sc.mesh_of[ib]]
        ta = oracle.world_tris(Va, Fa, sc.state[ia]).reshape(-1, 3, 3)
        tb = oracle.world_tris(Vb, Fb, sc.state[ib]).reshape(-1, 3, 3)
        ca, cb = ta.mean(1), tb.mean(1)
        ra = np.linalg.norm(ta - ca[:, None], axis=2).max(1)
        rb = np.linalg.norm(tb - cb[:, None], axis=2).max(1)
        i, j = np.meshgrid(np.arange(len(ta)), np.arange(len(tb)), indexing="ij")
        i, j = i.ravel(), j.ravel()
        k = rng.choice(i.size, size=min(i.size, max_tri_pairs // n_pairs), replace=False)
        allp.append(np.concatenate([ta[i[k]].reshape(-1, 9), tb[j[k]].reshape(-1, 9)], 1))
        gap = np.linalg.norm(ca[:, None] - cb[None], axis=2) - ra[:, None] - rb[None]
        ni, nj = np.nonzero(gap <= 2 * 0.005)
        near.append(np.concatenate([ta[ni].reshape(-1, 9), tb[nj].reshape(-1, 9)], 1))
    return np.concatenate(allp), np.concatenate(near)


def main():
    allp, near = sample_triangle_pairs()
    with tempfile.TemporaryDirectory() as tmp:
        exe = build(tmp)
        a = count(exe, allp, tmp)
        b = count(exe, near, tmp)
    for name, r in (("all triangle pairs of the sampled candidate pairs", a), ("near triangle pairs", b)):
        print("%s: %d pairs, %.1f flops per evaluation (add %.1f, mul %.1f, div %.1f, sqrt %.1f), "
              "%.3f intersecting" % (name, r["pairs"], r["flops"], r["add"], r["mul"], r["div"], r["sqrt"],
                                     r["intersecting"]))
    return a, b


if __name__ == "__main__":
    main()
