"""The work unit of the roofline figures: the instrumented flop count of one
triangle-pair evaluation in the oracle's formulation (oracle/flop_count.py)
agrees with the constant the benchmark uses."""

import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(path, name):
    spec = importlib.util.spec_from_file_location(name, path)
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_c_full_matches_instrumented_count():
    fc = _load(os.path.join(ROOT, "oracle", "flop_count.py"), "flop_count")
    bench = _load(os.path.join(ROOT, "bench.py"), "bench_module")
    allp, near = fc.sample_triangle_pairs(n_pairs=6, max_tri_pairs=60000)
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        exe = fc.build(tmp)
        a = fc.count(exe, allp, tmp)
    assert abs(a["flops"] - bench.C_FULL) <= 0.03 * bench.C_FULL, a
    # a full evaluation of triangles that do not intersect runs 6
    # intersection tests (4 edge lengths and a normal length each) and the
    # final square root; intersecting ones stop at the first crossing edge
    assert 30.0 < a["sqrt"] <= 31.0
