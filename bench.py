#!/usr/bin/env python
"""Throughput of the narrow-phase contact query on one MI355X.

Headline workload (one step): every candidate pair of a static packing of
2,000 perturbed icospheres (subdivision 1-4, 80-5,120 triangles, radius 1
with vertex radii scaled by 1+U[-0.1, 0.1]) at packing fraction 0.55 on the
nominal radius 1 (neighbours touch through their bumps and interpenetrate by
up to 0.2), halo eps = 0.005 (contact threshold 0.01), submitted as one pair
query through the C ABI: tile cull, near list, FP32 triangle-pair filter,
FP64 re-decision of the candidates, exact minima of the pairs in contact,
contact records sorted on the device. Meshes and particle states are
resident in HBM before the timed region. A step's time is device time (one
replayed HIP graph plus the contact sort); the host staging of the pair
sources and the download of the records are reported under pcie_inclusive.

`value` = contacts per second of device time. The same line carries the
packing on the bounding radius 1.1 (static_bounding_radius: no particles
interpenetrate, and no triangle pair comes within the halo, so it measures
the cull alone), the collision time stamps of the 10,000-particle moving
packing (toi) and the serving loop on 100,000 resident particles (serve),
each with its own step time, roofline and latency percentiles; and the
oracle on the host's cores (cpu_baseline). Warm-up runs at least --warmup
steps and continues until the autotuner has chosen the launch shape of the
query's size class, so no timed step runs a trial shape.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work units. C_FULL: floating-point operations of one full
# triangle-pair distance evaluation in the oracle's formulation (6
# segment-triangle intersection tests, 6 point-triangle and 9 segment-segment
# distances), counted by compiling the oracle's routines with a counting
# number type (oracle/flop_count.py: 1,331.9 on average over every triangle
# pair of 24 sampled candidate pairs of the static packing, 1,436.9 over its
# near pairs; additions, multiplications, divisions and square roots, no
# contraction). FLOPS_PER_CULL: one bounding-sphere test (centre difference,
# squared length, radii), about 12 flops.
C_FULL = 1332
FLOPS_PER_CULL = 12
# FP32 floating-point operations of one triangle-pair evaluation in the
# filter's formulation (FMA counted as 2, reciprocal as 1; comparisons,
# min/max and selects not counted): 6 vertex-face tests of 22 (plane height 6,
# inside test 15, square 1), 18 for the two triangles' edge vectors, 9
# edge-edge distances of 51 each.
FLOPS_PER_EVAL = 6 * 22 + 18 + 9 * 51
# Triangle bounding-sphere test that lets a wave skip a B triangle: centre
# difference 3, squared length 5, reach 2, square 1.
FLOPS_PER_SPHERE = 11
# Plane-separation test of a near triangle pair (in the near-list kernel):
# B's vertices moved into A's frame (54), B's plane moved (normal 15, offset
# 6), six vertex heights (36).
FLOPS_PER_PLANE = 54 + 15 + 6 + 36
# One FP32 sample of the time-stamp scan in the method's units: B's triangle
# moved to the sample time (3 vertices x 18), then a full evaluation.
FLOPS_PER_SAMPLE = 54 + C_FULL
# One bounding-sphere gap at a sample time in the time-stamp sphere walks:
# centre moved by the sample transform (9 FMA, 3 adds), difference 3, squared
# length 5, square root 1, minus the two radii and the margin 3.
FLOPS_PER_GAP = 18 + 3 + 3 + 5 + 1 + 3
# One FP64 distance evaluation of the end-game at a time t: both poses at t
# (quaternion update 28 each, rotation matrix 24 each), relative transform
# (27 FMA + 9 FMA + 3), B's triangle moved (54), a full evaluation.
FLOPS_PER_FP64_EVAL = 2 * (28 + 24) + 2 * 36 + 3 + 54 + C_FULL
# Vector ALU peaks of the MI355X (256 CUs, 2.4 GHz). FP32: the published
# 157.3 TFLOP/s (4 SIMDs x 32 lanes x 2 flops per CU and cycle). The build
# has no packed-FP32 instructions, yet plain wave64 FP32 code reaches this
# rate: the dense evaluation kernel issues 586 vector instructions per 64
# triangle-pair evaluations and runs 1.09e11 evaluations/s, i.e. one
# instruction per 2.5 cycles per SIMD, which a 4-cycle (16-lane) issue could
# not sustain. FP64: 78.6 TFLOP/s (half the FP32 rate).
PEAK_FP32_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12
PEAK_FP64_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def peak_of(kernel):
    """Vector peak for a kernel's arithmetic type (FP64 kernels: the plain
    FP64 evaluation and the end-game)."""
    return PEAK_FP64_TFLOPS if ("64" in kernel or "endgame" in kernel) else PEAK_FP32_TFLOPS


def cpu_baseline(sc, target_evals=1.2e8, max_pairs=64):
    """The oracle on a seeded sample of the packing's candidate pairs (every
    triangle pair of each sampled particle pair evaluated: the oracle has no
    culling). Reported in contacts/s, with its evaluation rate beside it."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(2000)
    order = rng.permutation(sc.pairs.shape[0])
    nt = sc.tri_counts()[sc.mesh_of]
    pick, tot = [], 0
    for k in order:
        a, b = sc.pairs[k]
        pick.append(k)
        tot += int(nt[a]) * int(nt[b])
        if tot >= target_evals or len(pick) >= max_pairs:
            break
    sub = sc.pairs[np.array(sorted(pick))]
    oracle.lib()
    t0 = time.perf_counter()
    _, con = oracle.static_pairs(sc, pairs=sub)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    out = {"value": con.shape[0] / dt, "unit": "contacts/s", "cores": cores, "kind": "oracle",
           "evals_per_s": tot / dt, "cpu_model": cpu_model(),
           "sample": "%d seeded candidate pairs of the same packing (%d contacts), all %d triangle "
                     "pairs each evaluated (the oracle has no culling), %.1f s"
                     % (len(pick), con.shape[0], tot, dt)}
    # one thread, on the first pairs of the same sample (the oracle's
    # OpenMP team set to one thread for the call)
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return out
    one, tot1 = [], 0
    for k in sorted(pick):
        a, b = sc.pairs[k]
        one.append(k)
        tot1 += int(nt[a]) * int(nt[b])
        if tot1 >= target_evals / 12:
            break
    gomp.omp_set_num_threads(1)
    try:
        t0 = time.perf_counter()
        _, con1 = oracle.static_pairs(sc, pairs=sc.pairs[np.array(one)])
        dt1 = time.perf_counter() - t0
    finally:
        gomp.omp_set_num_threads(cores)
    out["single_thread"] = {"evals_per_s": tot1 / dt1, "contacts_per_s": con1.shape[0] / dt1,
                            "sample": "the first %d pairs of that sample (%d triangle pairs), %.1f s"
                                      % (len(one), tot1, dt1)}
    return out


def cpu_model():
    """The host CPU's model name (Linux), for the oracle's timings."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


PROFILE_SOURCES = ("mcd_kernels.hip", "mcd_toi.hip", "mcd_geom.h", "mcd_dev.h", "mcd_internal.h")


def kernel_source_hash():
    """sha256 over the device sources; a stored counter reading is used only
    while the kernels it was taken on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2309_15417_amd", "csrc")
    for f in PROFILE_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_of(kernel, workload):
    """HBM bytes per launch of a kernel, from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE summary in profiles/<kernel>_<workload>.md (scaled by the copy
    calibration recorded there), or None when there is no summary or the
    device sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def warm(run_step, warmup, max_extra=96):
    """At least `warmup` untimed steps, then more until the autotuner has
    chosen the launch shape of the query's size class (stats tune_pending =
    0), so that no timed step runs one of its trial shapes. Returns the
    number of warm-up steps run."""
    k, st = 0, None
    while k < warmup or (st is not None and st["tune_pending"] > 0 and k < warmup + max_extra):
        st = run_step()
        k += 1
    if st is not None and st["tune_pending"] > 0:
        raise RuntimeError("the autotuner did not settle within %d warm-up steps" % k)
    return k


def run_static(args, sc, label, fp64_leg=True, per_kernel=True):
    """The static contact query over every candidate pair of a packing:
    mixed path timed (graph replay), the same steps kernel by kernel for
    per-kernel times, and the plain FP64 path for comparison."""
    import torch
    import paper_2309_15417_amd as mcd
    stream = torch.cuda.current_stream().cuda_stream
    ctx = mcd.Context(stream=stream)
    ctx.load_scene(sc)
    pairs = sc.pairs
    outbuf = {}

    def step(flags):
        t = ctx.query_pairs(pairs, flags=flags)
        pr, con = ctx.fetch(t, out=outbuf)
        st = ctx.stats(t)
        ctx.release(t)
        return pr, con, st

    def timed(flags, steps, warmup):
        nwarm = warm(lambda: step(flags)[2], warmup)
        torch.cuda.synchronize()
        lat, stats, ncon = [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            pr, con, st = step(flags)
            lat.append(time.perf_counter() - s0)
            stats.append(st)
            ncon.append(con.shape[0])
        torch.cuda.synchronize()
        assert all(x["tune_pending"] == 0 for x in stats)
        return time.perf_counter() - t0, lat, stats, ncon, nwarm

    print("[bench] %s: mixed path, >= %d warmup + %d timed steps" % (label, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    wall, lat, stats, ncon, nwarm = timed(mcd.Q_MIXED, args.steps, args.warmup)
    kstats = stats
    if per_kernel:
        print("[bench] %s: the same steps kernel by kernel with events" % label, file=sys.stderr, flush=True)
        _, _, kstats, _, _ = timed(mcd.Q_MIXED | mcd.Q_TIMING, args.steps, 1)
    out = static_line(args, sc, pairs, wall, lat, stats, ncon, kstats)
    out["warmup_steps_run"] = nwarm
    if fp64_leg and not args.no_fp64:
        print("[bench] %s: plain FP64 path for comparison" % label, file=sys.stderr, flush=True)
        k64 = max(3, args.steps // 4)
        wall64, lat64, st64, nc64, nw64 = timed(mcd.Q_FP64, k64, args.warmup)
        _, _, k64s, _, _ = timed(mcd.Q_FP64 | mcd.Q_TIMING, k64, 1)
        f64 = static_line(args, sc, pairs, wall64, lat64, st64, nc64, k64s, fp64=True)
        out["fp64_plain"] = {"ms_per_step": f64["ms_per_step"], "value": f64["value"],
                             "warmup_steps_run": nw64,
                             "host_ms_per_step": f64["pcie_inclusive"]["ms_per_step"],
                             "kernels": f64["kernels"],
                             "speedup_mixed_vs_fp64": f64["ms_per_step"] / out["ms_per_step"]}
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=16,
                    help="untimed steps (at least; more run until the autotuner has settled)")
    ap.add_argument("--run", type=int, default=0, help="scene seed run index")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-host-paths", action="store_true", help="static: skip the end-to-end host API legs")
    ap.add_argument("--no-sub", action="store_true",
                    help="static: leave out the static_bounding_radius, toi and serve sub-objects")
    ap.add_argument("--queries", type=int, default=10000, help="serve: measured queries per phase")
    ap.add_argument("--streams", type=int, default=2, help="serve: concurrent batch slots")
    ap.add_argument("--workload", default="static", choices=["static", "dense", "batch", "toi", "serve", "copy"],
                    help="static: contact query on the 2,000-particle packing (default); "
                         "dense: the same pairs with every triangle pair evaluated (exact minimum per pair); "
                         "batch: 4,096 uneven single-pair queries batched by the scheduler; "
                         "toi: collision time stamps on the 10,000-particle moving packing; "
                         "serve: Poisson stream of cluster queries on 100,000 resident particles; "
                         "copy: one 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the contact query runs on a single MI355X "
              "(multi-GPU sharding is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth

    torch.cuda.set_device(0)
    if args.workload == "toi":
        print(json.dumps(bench_toi(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "dense":
        return bench_dense(args)
    if args.workload == "copy":
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_read": src.numel() * 4,
                          "bytes_written": dst.numel() * 4}), flush=True)
        return
    print("[bench] generating the 2,000-particle packing", file=sys.stderr, flush=True)
    sc = synth.cfg2_scene(run=args.run)
    out = run_static(args, sc, "static packing")
    if not args.no_host_paths:
        out["host_paths"] = host_paths(args, sc)
        print("[bench] static packing: cull levels per mesh size", file=sys.stderr, flush=True)
        out["cull_levels"] = cull_levels(sc)
        print("[bench] static packing: particle interaction over the fused contacts", file=sys.stderr, flush=True)
        out["interaction"] = interaction(sc)
    if not args.no_sub:
        print("[bench] generating the 2,000-particle packing on the bounding radius 1.1", file=sys.stderr,
              flush=True)
        sc1 = synth.cfg2_scene(run=args.run, pack_r=1.1)
        r1 = run_static(args, sc1, "static packing, bounding radius", fp64_leg=False, per_kernel=True)
        out["static_bounding_radius"] = {k: r1[k] for k in ("value", "unit", "ms_per_step", "contacts_per_step",
                                                            "evals_per_step", "config", "roofline", "kernels",
                                                            "query_latency_ms", "pcie_inclusive",
                                                            "warmup_steps_run")}
        sub = argparse.Namespace(**vars(args))
        sub.no_cpu_baseline = True
        sub.no_fp64 = True
        out["toi"] = bench_toi(sub)
        out["serve"] = bench_serve(sub)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out), flush=True)


def host_paths(args, sc):
    """The static query end to end through the host API, per step: the pair
    list in, the contact records out where the caller reads them.
    - fetch_copy: host pair list, records copied into the caller's array
      (the pcie_inclusive figure of the line);
    - view: host pair list, records read in place in the library's pinned
      memory (mcd_result_view, no host copy);
    - pipelined_view: the same with two stream slots and two queries in
      flight, so one query's readback overlaps the next one's kernels;
    - device_out: host pair list, records left on the device and copied into
      caller device memory (MCD_Q_DEVICE_OUT, mcd_fetch_dev);
    - device_list_out: device pair list in, device records out (no PCIe
      transfer of pairs or records)."""
    import collections
    import numpy as np
    import torch
    import paper_2309_15417_amd as mcd
    out = {}
    pairs = sc.pairs
    dpairs = torch.from_numpy(pairs.copy()).cuda()
    cur = torch.cuda.current_stream()
    nc_max = [1]
    bufs = {}

    def dev_bufs(n, nc):
        if "pr" not in bufs or bufs["pr"].shape[0] < n or bufs["con"].shape[0] < nc:
            bufs["pr"] = torch.empty((int(n * 1.25) + 1, mcd.PAIR_RESULT_DT.itemsize), dtype=torch.uint8,
                                     device="cuda")
            bufs["con"] = torch.empty((int(nc * 1.25) + 1, mcd.CONTACT_DT.itemsize), dtype=torch.uint8,
                                      device="cuda")
        return bufs["pr"], bufs["con"]

    def finish_host(ctx, t, copy, outbuf):
        if copy:
            pr, con = ctx.fetch(t, out=outbuf)
        else:
            pr, con = ctx.view(t)
        ncon = con.shape[0]
        st = ctx.stats(t)
        ctx.release(t)
        return st, ncon

    def finish_dev(ctx, t):
        n, nc = ctx.result_sizes(t)
        bpr, bcon = dev_bufs(n, nc)
        ctx.fetch_dev(t, bpr.data_ptr(), bpr.shape[0], bcon.data_ptr(), bcon.shape[0], stream=cur.cuda_stream)
        cur.synchronize()
        st = ctx.stats(t)
        ctx.release(t)
        return st, nc

    variants = [
        ("fetch_copy", 1, 1, lambda c: c.query_pairs(pairs, flags=mcd.Q_MIXED), "copy"),
        ("view", 1, 1, lambda c: c.query_pairs(pairs, flags=mcd.Q_MIXED), "view"),
        ("pipelined_view", 2, 2, lambda c: c.query_pairs(pairs, flags=mcd.Q_MIXED), "view"),
        ("device_out", 1, 1, lambda c: c.query_pairs(pairs, flags=mcd.Q_MIXED | mcd.Q_DEVICE_OUT), "dev"),
        ("device_list_out", 1, 1,
         lambda c: c.query_pairs_dev(dpairs.data_ptr(), pairs.shape[0], flags=mcd.Q_MIXED | mcd.Q_DEVICE_OUT,
                                     stream=cur.cuda_stream), "dev"),
    ]
    for name, slots, depth, submit, how in variants:
        print("[bench] static packing, host path: %s" % name, file=sys.stderr, flush=True)
        with mcd.Context(stream=cur.cuda_stream, streams=slots) as ctx:
            ctx.load_scene(sc)
            outbuf = {}

            def done(t):
                if how == "dev":
                    return finish_dev(ctx, t)
                return finish_host(ctx, t, how == "copy", outbuf)

            warm(lambda: done(submit(ctx))[0], args.warmup)
            torch.cuda.synchronize()
            inflight = collections.deque()
            ncon = []
            t0 = time.perf_counter()
            for k in range(args.steps + depth - 1):
                if k < args.steps:
                    inflight.append(submit(ctx))
                if len(inflight) == depth or k >= args.steps:
                    st, nc = done(inflight.popleft())
                    ncon.append(nc)
            while inflight:
                st, nc = done(inflight.popleft())
                ncon.append(nc)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            out[name] = {"ms_per_step": ms, "contacts_per_s": float(np.mean(ncon)) / (ms * 1e-3),
                         "slots": slots, "in_flight": depth}
    return out


def cull_levels(sc):
    """The cull's two bounding levels per mesh-size class of the static
    packing: for the candidate pairs whose larger mesh has the class's
    triangle count, the tile pairs a flat cull tests (every tile pair) against
    the sphere tests of the group level plus the tile tests of the kept group
    pairs, and what the later stages see."""
    import numpy as np
    import torch
    import paper_2309_15417_amd as mcd
    nt = sc.tri_counts()[sc.mesh_of]
    big = np.maximum(nt[sc.pairs[:, 0]], nt[sc.pairs[:, 1]])
    small = np.minimum(nt[sc.pairs[:, 0]], nt[sc.pairs[:, 1]])
    out = {}
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.load_scene(sc)
        classes = [("largest mesh %d triangles" % c, big == c) for c in np.unique(big)]
        classes.append(("both meshes 5120 triangles", (big == 5120) & (small == 5120)))
        for name, sel in classes:
            sub = sc.pairs[sel]
            if sub.shape[0] == 0:
                continue
            t = ctx.query_pairs(sub, flags=mcd.Q_MIXED)
            _, con = ctx.fetch(t)
            st = ctx.stats(t)
            ctx.release(t)
            out[name] = {"pairs": int(sub.shape[0]), "flat_tile_tests": int(st["tile_pairs_total"]),
                         "group_and_tile_tests": int(st["cull_tests"]),
                         "tests_ratio": st["cull_tests"] / max(1, st["tile_pairs_total"]),
                         "tile_pairs_kept": int(st["tile_pairs_kept"]),
                         "triangle_sphere_tests": int(st["sphere_tests"]),
                         "full_evaluations": int(st["tri_pairs_evaluated"]), "contacts": int(con.shape[0])}
    return out


def disjoint_clusters(sc, rng):
    """Clusters of the static packing that share no particle: in a seeded
    order, each unused particle with its unused neighbours (by candidate
    pair) forms one; the candidate pairs inside the clusters are returned."""
    import numpy as np
    n = sc.n_particles
    nbr = [[] for _ in range(n)]
    for a, b in sc.pairs:
        nbr[a].append(b)
        nbr[b].append(a)
    owner = np.full(n, -1)
    k = 0
    for s in rng.permutation(n):
        if owner[s] >= 0:
            continue
        owner[s] = k
        for b in nbr[s]:
            if owner[b] < 0:
                owner[b] = k
        k += 1
    keep = owner[sc.pairs[:, 0]] == owner[sc.pairs[:, 1]]
    return sc.pairs[keep], k


def interaction(sc, reps=3):
    """Particle interaction (section 6) on cluster-sized problems: the static
    packing split into clusters that share no particle (a particle with its
    neighbours), particles with seeded random velocities, the contact query
    over the pairs inside the clusters with MCD_Q_FUSE, then mcd_impulses
    (frictionless, e = 0, tol 1e-4) timed end to end: host colouring and
    clustering, upload, one device workgroup per cluster, download."""
    import numpy as np
    import torch
    import paper_2309_15417_amd as mcd
    rng = np.random.default_rng(12)
    states = sc.state.copy()
    states[:, 7:10] = rng.normal(size=(sc.n_particles, 3))
    states[:, 10:13] = rng.normal(scale=0.5, size=(sc.n_particles, 3))
    pairs, nclusters = disjoint_clusters(sc, rng)
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ids = ctx.load_scene(sc)
        ctx.particles_set(np.arange(sc.n_particles, dtype=np.int32), ids[sc.mesh_of], states)
        t = ctx.query_pairs(pairs, flags=mcd.Q_MIXED | mcd.Q_FUSE)
        _, con, pp = ctx.fetch(t, with_pairs=True)
        con, pid_pairs = con.copy(), pp[con["pair"]].copy()
        ctx.release(t)
        ctx.impulses(pid_pairs, con, max_iter=10000)          # warm-up
        ms, sw = [], 0
        for _ in range(reps):
            t0 = time.perf_counter()
            imp, pids, vel, sw = ctx.impulses(pid_pairs, con, max_iter=10000)
            ms.append((time.perf_counter() - t0) * 1e3)
    m = float(np.median(ms))
    return {"clusters": int(nclusters), "pairs": int(pairs.shape[0]), "contacts": int(con.shape[0]),
            "particles": int(pids.shape[0]), "sweeps_max": int(sw), "ms": m,
            "contact_updates_per_s": con.shape[0] * sw / (m * 1e-3),
            "active_contacts": int((imp[:, 0] > 0).sum())}


def static_line(args, sc, pairs, wall, lat, stats, ncon, kstats, fp64=False):
    """JSON line of a static run. A step's time is its device time: the
    kernels from the tile cull to the sorted contact records in HBM (one
    replayed HIP graph plus the sort), with the pair-record upload and the
    result download excluded (both are reported under pcie_inclusive).
    Per-kernel times come from the same steps launched kernel by kernel with
    HIP events between the kernels on the query's stream (kstats)."""
    import numpy as np
    st = stats[0]
    mean = lambda k: float(np.mean([s[k] for s in kstats]))
    ms = float(np.mean([s["gpu_ms"] for s in stats]))
    host_ms = wall / len(stats) * 1e3
    con = float(np.mean(ncon))
    evals, tests = st["tri_pairs_evaluated"], st["sphere_tests"]
    # algorithmic work in the units of the method: a bounding-sphere test
    # (tile pairs in the cull, triangle spheres in the near-list stage) and a
    # full triangle-pair evaluation (C_FULL, counted on the oracle's
    # formulation); the plane-separation test of the near-list stage is a
    # filter of this implementation and is not counted
    kern = {
        "k_cull": (mean("cull_ms"), st["cull_tests"] * FLOPS_PER_CULL),
        "k_near": (mean("near_ms"), tests * FLOPS_PER_CULL),
        "k_eval64" if fp64 else "k_eval32": (mean("main_ms"), evals * C_FULL),
    }
    kernels = {}
    for k, (kms, flops) in kern.items():
        a = flops / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
        kernels[k] = {"ms": kms, "achieved_tflops": a, "frac": a / peak_of(k), "peak": peak_of(k)}
    dom = max(kern, key=lambda k: kern[k][0])
    return {
        "metric": "tri-pair distance evals/s + contacts/s at eps; p99 cluster-query latency",
        "value": con / (ms * 1e-3),
        "unit": "contacts/s",
        "n_gpus": 1,
        "steps": len(stats),
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "static packing: 2000 perturbed icospheres (80-5120 tris), "
                               "phi=0.55 on radius %.1f%s, eps=0.005, all %d candidate pairs per step, "
                               "FP32 filter + FP64 re-decision"
                               % (sc.info["pack_r"],
                                  " (bounding radius: no interpenetration)" if sc.info["pack_r"] > 1.05
                                  else " (nominal radius: neighbours interpenetrate by up to 0.2)",
                                  pairs.shape[0]),
                   "particles": int(sc.n_particles), "candidate_pairs": int(pairs.shape[0]),
                   "triangles": int(sc.tri_counts().sum()), "eps": 0.005, "pack_radius": sc.info["pack_r"]},
        "contacts_per_step": int(ncon[0]),
        "evals_per_s": evals / (ms * 1e-3),
        "evals_per_step": int(evals),
        "sphere_tests_per_step": int(tests),
        "cull_tests_per_step": int(st["cull_tests"]),
        "near_pairs_per_step": int(st["near_pairs"]),
        "tiled_tri_pairs_per_step": int(st["tri_pairs_tiled"]),
        "covered_tri_pairs_per_s": st["tri_pairs_covered"] / (ms * 1e-3),
        "query_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                             "p99": float(np.percentile(lat, 99) * 1e3)},
        "pcie_inclusive": {"ms_per_step": host_ms, "contacts_per_s": con / (host_ms * 1e-3)},
        "stats": {k: st[k] for k in ("tile_pairs_total", "tile_pairs_kept", "fp64_rechecks",
                                     "refine_items", "retries")},
        "kernel_by_kernel_ms_per_step": mean("gpu_ms"),
        "kernels": kernels,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": kernels[dom]["achieved_tflops"],
                     "peak": peak_of(dom), "unit": "TFLOP/s", "frac": kernels[dom]["frac"],
                     "traffic": traffic_of(dom, "static_packing"),
                     "kernel_ms": kern[dom][0]},
    }


def bench_dense(args):
    """Dense query on the static packing: every triangle pair of every
    candidate pair evaluated by the FP32 filter (k_dist32, lane = A triangle,
    B's tile in LDS), the items that can hold a pair's minimum re-run in FP64,
    contacts re-decided in FP64. This measures the raw triangle-pair
    evaluation rate against the vector ALU roofline; `value` = evaluations per
    second of device time."""
    import numpy as np
    import torch
    import synth
    import paper_2309_15417_amd as mcd
    print("[bench] generating the 2,000-particle packing", file=sys.stderr, flush=True)
    sc = synth.cfg2_scene(run=args.run)
    ctx = mcd.Context(stream=torch.cuda.current_stream().cuda_stream)
    ctx.load_scene(sc)
    pairs = sc.pairs
    outbuf = {}
    flags = mcd.Q_MIXED | mcd.Q_DENSE
    steps, warmup = min(args.steps, 3), min(args.warmup, 1)

    def run(f, k):
        stats, ncon = [], []
        for _ in range(k):
            t = ctx.query_pairs(pairs, flags=f)
            _, con = ctx.fetch(t, out=outbuf)
            stats.append(ctx.stats(t))
            ncon.append(con.shape[0])
            ctx.release(t)
        return stats, ncon

    print("[bench] dense: %d warmup + %d timed steps" % (warmup, steps), file=sys.stderr, flush=True)
    run(flags, warmup)
    torch.cuda.synchronize()
    stats, ncon = run(flags, steps)
    print("[bench] dense: kernel by kernel with events", file=sys.stderr, flush=True)
    kstats, _ = run(flags | mcd.Q_TIMING, 1)
    st = stats[0]
    ms = float(np.mean([x["gpu_ms"] for x in stats]))
    evals = st["tri_pairs_evaluated"]
    kms = float(kstats[0]["main_ms"])
    ach = evals * C_FULL / (kms * 1e-3) / 1e12
    ach_k = evals * FLOPS_PER_EVAL / (kms * 1e-3) / 1e12
    out = {
        "metric": "tri-pair distance evals/s + contacts/s at eps; p99 cluster-query latency",
        "value": evals / (ms * 1e-3),
        "unit": "tri-pair evals/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "dense static packing: 2000 perturbed icospheres (80-5120 tris), phi=0.55, "
                               "eps=0.005, every triangle pair of all %d candidate pairs, FP32 filter + FP64 "
                               "refinement of the minima and re-decision of the contacts" % pairs.shape[0],
                   "particles": int(sc.n_particles), "candidate_pairs": int(pairs.shape[0]), "eps": 0.005},
        "evals_per_step": int(evals),
        "contacts_per_step": int(ncon[0]),
        "contacts_per_s": ncon[0] / (ms * 1e-3),
        "refine_items": int(st["refine_items"]),
        "kernels": {"k_dist32": {"ms": kms, "achieved_tflops": ach, "frac": ach / PEAK_FP32_TFLOPS,
                                 "peak": PEAK_FP32_TFLOPS,
                                 "achieved_tflops_kernel_formulation": ach_k,
                                 "frac_kernel_formulation": ach_k / PEAK_FP32_TFLOPS}},
        "roofline": {"bound": "alu", "kernel": "k_dist32", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
                     "traffic": traffic_of("k_dist32", "dense_packing"), "kernel_ms": kms},
    }
    ctx.close()
    if not args.no_cpu_baseline:
        # the oracle evaluates every triangle pair too: the same sample as the
        # static line, reported in evaluations/s
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        cb = cpu_baseline(sc)
        out["cpu_baseline"] = {"value": cb["evals_per_s"], "unit": "tri-pair evals/s", "cores": cb["cores"],
                               "kind": "oracle", "contacts_per_s": cb["value"], "sample": cb["sample"]}
    print(json.dumps(out), flush=True)


def toi_cpu_baseline(sc, max_pairs=12):
    import numpy as np
    import oracle
    rng = np.random.default_rng(4000)
    idx = np.sort(rng.choice(sc.pairs.shape[0], size=min(max_pairs, sc.pairs.shape[0]), replace=False))
    oracle.lib()
    t0 = time.perf_counter()
    _, _, diag = oracle.toi_pairs(sc, sc.dt, pairs=sc.pairs[idx])
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    return {"value": len(idx) / dt, "unit": "pair time stamps/s", "cores": cores, "kind": "oracle",
            "evals_per_s": diag["evals"] / dt,
            "sample": "%d seeded candidate pairs of the same moving packing, every triangle pair "
                      "scanned (%d FP64 distance evaluations), %.1f s" % (len(idx), diag["evals"], dt)}


def bench_toi(args):
    import numpy as np
    import torch
    import synth
    import paper_2309_15417_amd as mcd
    print("[bench] generating the 10,000-particle moving packing", file=sys.stderr, flush=True)
    sc = synth.cfg4_scene(run=args.run)
    ctx = mcd.Context(stream=torch.cuda.current_stream().cuda_stream)
    ctx.load_scene(sc)
    pairs = sc.pairs

    def step(flags):
        t = ctx.query_pairs(pairs, dt=sc.dt, flags=flags, samples=64, tol_rel=1e-6)
        pr, con = ctx.fetch(t)
        st = ctx.stats(t)
        ctx.release(t)
        return pr, con, st

    def timed(flags, steps, warmup):
        warm(lambda: step(flags)[2], warmup)
        torch.cuda.synchronize()
        lat, stats, res = [], [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            res = step(flags)
            lat.append(time.perf_counter() - s0)
            stats.append(res[2])
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, stats, res

    print("[bench] time stamps: %d warmup + %d timed steps" % (args.warmup, args.steps),
          file=sys.stderr, flush=True)
    wall, lat, stats, (pr, con, _) = timed(mcd.Q_MIXED, args.steps, args.warmup)
    host_ms = wall / args.steps * 1e3
    ms = float(np.mean([s["gpu_ms"] for s in stats]))
    st = stats[0]
    # per-stage times: the same steps launched kernel by kernel with events
    print("[bench] time stamps: kernel by kernel with events", file=sys.stderr, flush=True)
    _, _, kstats, _ = timed(mcd.Q_MIXED | mcd.Q_TIMING, max(3, args.steps // 2), 1)
    mean = lambda k: float(np.mean([s[k] for s in kstats]))
    samples = st["fp32_samples"]
    evals = samples + st["fp64_evals"]
    kern = {"k_toi_cull": (mean("cull_ms"), 0),
            "k_toi_near+k_toi_swalk": (mean("near_ms"), st["sphere_tests"] * FLOPS_PER_GAP),
            "k_toi_walk": (mean("main_ms"), samples * FLOPS_PER_SAMPLE),
            "k_toi_endgame": (mean("endgame_ms"), st["fp64_evals"] * FLOPS_PER_FP64_EVAL)}
    kernels = {}
    for k, (kms, flops) in kern.items():
        a = flops / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
        kernels[k] = {"ms": kms, "achieved_tflops": a, "frac": a / peak_of(k), "peak": peak_of(k)}
    dom = max(kern, key=lambda k: kern[k][0])
    out = {
        "metric": "tri-pair distance evals/s + contacts/s at eps; p99 cluster-query latency",
        "value": evals / (ms * 1e-3),
        "unit": "tri-pair evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "time stamps: 10000 moving perturbed icospheres (320/1280 tris), "
                               "v~N(0,1), w~N(0,5), dt=%.4g, S=64, tol=1e-6 dt, all %d candidate "
                               "pairs per step" % (sc.dt, pairs.shape[0]),
                   "particles": int(sc.n_particles), "candidate_pairs": int(pairs.shape[0]),
                   "dt": sc.dt},
        "pairs_per_s": pairs.shape[0] / (ms * 1e-3),
        "colliding_pairs": int((pr["status"] == 2).sum()),
        "at_start_pairs": int((pr["status"] == 1).sum()),
        "collide_fraction": float((pr["status"] == 2).mean()),
        "contacts_per_s": con.shape[0] / (ms * 1e-3),
        "query_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                             "p99": float(np.percentile(lat, 99) * 1e3)},
        "pcie_inclusive": {"ms_per_step": host_ms, "pairs_per_s": pairs.shape[0] / (host_ms * 1e-3)},
        "kernel_by_kernel_ms_per_step": mean("gpu_ms"),
        "stats": {k: st[k] for k in ("tile_pairs_total", "tile_pairs_kept", "tri_pairs_evaluated",
                                     "sphere_tests", "fp32_samples", "candidates", "fp64_evals",
                                     "grazes")},
        "kernels": kernels,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": kernels[dom]["achieved_tflops"],
                     "peak": peak_of(dom), "unit": "TFLOP/s", "frac": kernels[dom]["frac"],
                     "traffic": traffic_of(dom.split("+")[0], "moving_packing"),
                     "kernel_ms": kern[dom][0]},
    }
    if not args.no_fp64:
        print("[bench] FP64 end-game on every candidate (plain FP64 scan)", file=sys.stderr, flush=True)
        w64, l64, s64, _ = timed(mcd.Q_FP64, 2, 1)
        ms64 = float(np.mean([s["gpu_ms"] for s in s64]))
        out["fp64_plain"] = {"ms_per_step": ms64, "host_ms_per_step": w64 / 2 * 1e3,
                             "speedup_mixed_vs_fp64": ms64 / ms}
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = toi_cpu_baseline(sc)
    ctx.close()
    return out


def bench_batch(args):
    """4,096 particle-pair queries of UV spheres with 20-5,120 triangles
    (log-uniform), gaps U[0, 2 eps], eps = 0.005, each submitted as its own
    query: the scheduler concatenates pending compatible queries into batches,
    each batch one replayed graph of persistent kernels (autotuned launch
    shapes). Compared with the same queries served one at a time (one graph
    launch each, serialised) and with all pairs as one query."""
    import numpy as np
    import synth
    import paper_2309_15417_amd as mcd
    print("[bench] generating 4,096 uneven pairs", file=sys.stderr, flush=True)
    sc = synth.cfg3_scene(run=args.run)
    pairs = sc.pairs
    nq = pairs.shape[0]

    def batched(ctx):
        t0 = time.perf_counter()
        tickets = [ctx.query_pairs(pairs[i:i + 1]) for i in range(nq)]
        ncon, dev, bq = 0, 0.0, []
        for t in tickets:
            ctx.wait(t)
        wall = time.perf_counter() - t0
        for t in tickets:
            _, c = ctx.result_sizes(t)
            st = ctx.stats(t)
            ncon += c
            dev += st["gpu_ms"] / max(1, st["batch_queries"])
            bq.append(st["batch_queries"])
            ctx.release(t)
        return wall, ncon, dev, bq

    out = {"metric": "tri-pair distance evals/s + contacts/s at eps; p99 cluster-query latency",
           "unit": "contacts/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "4096 single-pair queries, UV spheres of 20-5120 triangles "
                                  "(log-uniform), gap U[0, 0.01], eps=0.005, batched by the "
                                  "scheduler on %d streams" % args.streams,
                      "queries": nq, "streams": args.streams,
                      "tri_pairs": int(sc.dense_tri_pairs())}}
    with mcd.Context(streams=args.streams) as ctx:
        ctx.load_scene(sc)
        print("[bench] warm-up (autotuner)", file=sys.stderr, flush=True)
        for _ in range(max(args.warmup, 3)):
            batched(ctx)
        walls, devs, ncon, bqs = [], [], 0, []
        for _ in range(args.steps):
            w, ncon, d, bq = batched(ctx)
            walls.append(w)
            devs.append(d)
            bqs += bq
        wall, dev = float(np.mean(walls)), float(np.mean(devs))
        # all pairs as one query
        t = ctx.query_pairs(pairs)
        ctx.wait(t)
        ctx.release(t)
        t0 = time.perf_counter()
        t = ctx.query_pairs(pairs)
        ctx.wait(t)
        one_wall = time.perf_counter() - t0
        one = ctx.stats(t)
        ctx.release(t)
    out.update({"value": ncon / (dev * 1e-3), "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": dev, "contacts_per_step": ncon,
                "queries_per_s": nq / wall, "wall_ms_per_step": wall * 1e3,
                "mean_batch_queries": float(np.mean(bqs)),
                "one_query": {"ms_per_step": one["gpu_ms"], "wall_ms": one_wall * 1e3}})
    with mcd.Context(streams=1) as ctx:
        ctx.load_scene(sc)
        print("[bench] one query at a time", file=sys.stderr, flush=True)
        for i in range(64):
            t = ctx.query_pairs(pairs[i:i + 1])
            ctx.wait(t)
            ctx.release(t)
        t0 = time.perf_counter()
        dev1 = 0.0
        for i in range(nq):
            t = ctx.query_pairs(pairs[i:i + 1])
            ctx.wait(t)
            dev1 += ctx.stats(t)["gpu_ms"]
            ctx.release(t)
        w1 = time.perf_counter() - t0
    out["per_query_serial"] = {"queries_per_s": nq / w1, "wall_ms_per_step": w1 * 1e3,
                               "device_ms_per_step": dev1,
                               "batching_speedup_wall": w1 / wall}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Cluster queries (seed particle + its nearest neighbours, sizes ~ n^-1.5
    on [1, 2000]) against 100,000 resident particles: saturated throughput
    with continuous batching, latency under Poisson arrivals at 0.5/0.8/0.95
    of that rate, and the same stream served one query at a time."""
    import numpy as np
    import synth
    import paper_2309_15417_amd as mcd
    print("[bench] generating 100,000 resident particles", file=sys.stderr, flush=True)
    sc = synth.cfg5_scene(run=args.run)
    rng = np.random.default_rng(5000 + args.run)
    nwq, nq = 1000, args.queries
    sizes = synth.cluster_sizes(nwq + 4 * nq, rng)
    seeds = rng.integers(0, sc.n_particles, size=sizes.size)
    members = synth.cluster_members(sc.state[:, :3], seeds, sizes)

    batch_q, sub_ms = [], []

    work = {}
    caps = []

    def reset():
        batch_q.clear()
        sub_ms.clear()
        work.clear()
        caps.clear()

    def consume(ctx, t, acc):
        """Wait for a ticket, read its results in place (mcd_result_view) and
        its statistics, release it."""
        ctx.wait(t)
        n, c = ctx.result_sizes(t)
        ctx.view(t)
        st = ctx.stats(t)
        acc["lat"].append(st["latency_ms"])
        batch_q.append(st["batch_queries"])
        sub_ms.append(st["submit_ms"])
        acc["pairs"] += n
        acc["con"] += c
        # a batch's counters and device time are shared by its queries
        caps.append(st["graph_captures"])
        share = 1.0 / max(1, st["batch_queries"])
        for k in ("gpu_ms", "tri_pairs_evaluated", "sphere_tests", "tile_pairs_total"):
            work[k] = work.get(k, 0.0) + st[k] * share
        ctx.release(t)

    def drain(ctx, tickets):
        reset()
        acc = {"lat": [], "pairs": 0, "con": 0}
        for t in tickets:
            consume(ctx, t, acc)
        return np.array(acc["lat"]), acc["pairs"], acc["con"]

    submit_s = [0.0]

    def saturated(ctx, qs):
        """Every query submitted at once; the phase ends when the last result
        is ready: the latest submission time plus library latency over the
        queries (the results are read and released afterwards, untimed)."""
        ts = np.empty(len(qs))
        tickets = [None] * len(qs)
        t0 = time.perf_counter()
        for i, m in enumerate(qs):
            ts[i] = time.perf_counter() - t0
            tickets[i] = ctx.query_cluster(m)
        submit_s[0] = time.perf_counter() - t0
        lat, npairs, ncon = drain(ctx, tickets)
        wall = float(np.max(ts + lat * 1e-3))
        return wall, lat, npairs, ncon

    def poisson(ctx, qs, rate):
        """Queries submitted at Poisson arrival times by a thread that does
        nothing else; their results are read and released once the last has
        been submitted (a query's latency is the library's, from submission
        to completion). The phase ends when the last result is ready: the
        latest submission time plus library latency over the queries."""
        gaps = rng.exponential(1.0 / rate, size=len(qs))
        arrivals = np.cumsum(gaps)
        tickets = [None] * len(qs)
        ts = np.empty(len(qs))
        t0 = time.perf_counter()
        for i, m in enumerate(qs):
            # spin until the arrival time (sleep overshoots by tens of microseconds)
            now = time.perf_counter() - t0
            while now < arrivals[i]:
                now = time.perf_counter() - t0
            ts[i] = now
            tickets[i] = ctx.query_cluster(m)
        t_sub = time.perf_counter() - t0
        late = float(np.max(ts - arrivals))
        lat, npairs, ncon = drain(ctx, tickets)
        w = float(np.max(ts + lat * 1e-3))
        return w, t_sub, late, lat, npairs, ncon

    out = {"metric": "tri-pair distance evals/s + contacts/s at eps; p99 cluster-query latency",
           "unit": "cluster queries/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "serving: 100000 resident perturbed icospheres (80-1280 tris, "
                                  "4096 distinct meshes), cluster queries of n ~ n^-1.5 on "
                                  "[1, 2000] particles (seed + nearest), static contact query "
                                  "per cluster, %d queries per phase" % nq,
                      "particles": sc.n_particles, "mean_cluster": float(sizes.mean()),
                      "streams": args.streams}}
    with mcd.Context(streams=args.streams) as ctx:
        print("[bench] loading %d meshes" % len(sc.meshes), file=sys.stderr, flush=True)
        ctx.load_scene(sc)
        print("[bench] warm-up", file=sys.stderr, flush=True)
        saturated(ctx, members[:nwq])
        print("[bench] saturated continuous batching", file=sys.stderr, flush=True)
        wall, lat, npairs, ncon = saturated(ctx, members[nwq:nwq + nq])
        qps = nq / wall
        flops = (work["tri_pairs_evaluated"] * C_FULL + (work["sphere_tests"] + work["tile_pairs_total"])
                 * FLOPS_PER_CULL)
        dev_ms = work["gpu_ms"]
        ach = flops / (dev_ms * 1e-3) / 1e12 if dev_ms > 0 else 0.0
        out["roofline"] = {"bound": "alu", "kernel": "whole contact-query chain (device time of the batches)",
                           "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / PEAK_FP32_TFLOPS, "traffic": None,
                           "device_ms_per_query": dev_ms / nq}
        out.update({"value": qps, "steps": nq, "warmup": nwq, "ms_per_step": wall / nq * 1e3,
                    "pairs_per_s": npairs / wall, "contacts_per_s": ncon / wall,
                    "saturated": {"queries_per_s": qps, "wall_s": wall, "submit_s": submit_s[0],
                                  "library_submit_ms_mean": float(np.mean(sub_ms)),
                                  "mean_batch_queries": float(np.mean(batch_q)),
                                  "latency_ms_p50": float(np.percentile(lat, 50)),
                                  "latency_ms_p99": float(np.percentile(lat, 99))}})
        # Poisson batches are smaller than saturated ones and fall in other
        # size classes: their launch shapes are tuned, their chains captured
        # and the pinned record buffers of a phase pooled in untimed runs of
        # the phases' size at each rate first
        print("[bench] warm-up at the Poisson rates", file=sys.stderr, flush=True)
        for frac in (0.5, 0.8, 0.95):
            poisson(ctx, members[:nq], frac * qps)
        out["poisson"] = {}
        for k, frac in enumerate((0.5, 0.8, 0.95)):
            print("[bench] Poisson at %.2f of saturated rate" % frac, file=sys.stderr, flush=True)
            qs = members[nwq + (k + 1) * nq: nwq + (k + 2) * nq]
            w, t_sub, late, l, npr, nc = poisson(ctx, qs, frac * qps)
            # arrivals: the queries were submitted at their Poisson times
            # (late = the largest delay of a submission behind its time);
            # the phase ends when the last result is on the host
            out["poisson"]["%.2f" % frac] = {"rate_qps": frac * qps, "arrival_qps": len(qs) / t_sub,
                                             "max_submit_delay_ms": late * 1e3,
                                             "completion_qps": len(qs) / w, "drain_ms": (w - t_sub) * 1e3,
                                             "latency_ms_p50": float(np.percentile(l, 50)),
                                             "latency_ms_p99": float(np.percentile(l, 99)),
                                             "graph_captures_in_phase": int(max(caps) - min(caps)),
                                             "contacts_per_s": nc / w}
        out["query_latency_ms"] = {"p50": out["poisson"]["0.80"]["latency_ms_p50"],
                                   "p99": out["poisson"]["0.80"]["latency_ms_p99"]}
    with mcd.Context(streams=1) as ctx:
        ctx.load_scene(sc)
        print("[bench] one query at a time", file=sys.stderr, flush=True)
        qs = members[nwq:nwq + nq]
        for m in members[:200]:
            t = ctx.query_cluster(m)
            ctx.wait(t)
            ctx.release(t)
        t0 = time.perf_counter()
        lat = []
        for m in qs:
            t = ctx.query_cluster(m)
            ctx.wait(t)
            lat.append(ctx.stats(t)["latency_ms"])
            ctx.release(t)
        w = time.perf_counter() - t0
        out["per_query_serial"] = {"queries_per_s": nq / w,
                                   "latency_ms_p50": float(np.percentile(lat, 50)),
                                   "latency_ms_p99": float(np.percentile(lat, 99)),
                                   "batching_speedup": qps / (nq / w)}
    return out


if __name__ == "__main__":
    main()
