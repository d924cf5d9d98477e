"""Query flags of the interface (GPU, through the C ABI): what CLOSEST and
CONTACTS select, the FP32 margin validation of MCD_Q_VALIDATE, and the
guard-band count of the FP64 re-decision.

The FP32 filter is conservative when its distance is never off by more than
its margin mu (plus the near-parallel correction where that applies): then
every triangle pair within the threshold in FP64 is a candidate. A
validating query re-evaluates in FP64 every triangle pair the filter
evaluates and reports the largest |d32 - d64| / margin; it must stay below
1/8 over about 1e8 evaluations of the static packing (on the nominal radius,
where neighbours interpenetrate) in random orientations
(pairs with a near-parallel edge pair are measured against their widened
bound mu + c and reported separately).
"""

import numpy as np
import pytest

import oracle
import synth
from parity import check_static

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _q(ctx, pairs, **kw):
    t = ctx.query_pairs(pairs, **kw)
    pr, con = ctx.fetch(t)
    st = ctx.stats(t)
    ctx.release(t)
    return pr.copy(), con.copy(), st


def test_closest_and_contacts_flags(mcd):
    sc = synth.cfg1_scene(run=4)
    ref, rcon = oracle.static_pairs(sc)
    with mcd.Context() as ctx:
        ctx.load_scene(sc)
        for base in (mcd.Q_MIXED, mcd.Q_FP64, mcd.Q_MIXED | mcd.Q_DENSE):
            _say("flags", base)
            pr, con, _ = _q(ctx, sc.pairs, flags=base)
            both, conb, _ = _q(ctx, sc.pairs, flags=base | mcd.Q_CLOSEST | mcd.Q_CONTACTS)
            assert pr.tobytes() == both.tobytes() and con.tobytes() == conb.tobytes()
            check_static(sc, sc.pairs, pr, con, ref, rcon, 1e-6, dense=bool(base & mcd.Q_DENSE))
            assert np.all(con["t"] == 0.0)
            # closest points only: no contact records, pair results unchanged
            pc, cc, _ = _q(ctx, sc.pairs, flags=base | mcd.Q_CLOSEST)
            assert cc.shape[0] == 0 and pc.tobytes() == pr.tobytes()
            # contact records only: the same records, pair results carry the flag
            pk, ck, _ = _q(ctx, sc.pairs, flags=base | mcd.Q_CONTACTS)
            assert ck.tobytes() == con.tobytes()
            assert np.array_equal(pk["contact"], pr["contact"])
            assert np.all(np.isinf(pk["dmin"])) and np.all(pk["tri_a"] == -1)
        # time stamps: the same selection
        mv = synth.cfg4_scene(run=3, n=200, subdivs=(1,), proxy_r=1.0)
        ctx.load_scene(mv)
        _say("flags, time stamps")
        pr, con, _ = _q(ctx, mv.pairs, dt=mv.dt)
        assert (pr["status"] == mcd.COLLIDES).any() and con.shape[0] > 0
        assert np.array_equal(con["t"], pr["toi"][con["pair"]])
        pc, cc, _ = _q(ctx, mv.pairs, dt=mv.dt, flags=mcd.Q_CLOSEST)
        assert cc.shape[0] == 0 and pc.tobytes() == pr.tobytes()
        pk, ck, _ = _q(ctx, mv.pairs, dt=mv.dt, flags=mcd.Q_CONTACTS)
        assert ck.tobytes() == con.tobytes()
        assert np.array_equal(pk["toi"], pr["toi"]) and np.array_equal(pk["status"], pr["status"])
        assert np.all(np.isinf(pk["dmin"]))
        # VALIDATE applies to static MIXED contact-set queries only
        for bad in (dict(flags=mcd.Q_FP64 | mcd.Q_VALIDATE), dict(flags=mcd.Q_MIXED | mcd.Q_DENSE | mcd.Q_VALIDATE),
                    dict(flags=mcd.Q_VALIDATE, dt=0.1), dict(flags=1 << 12)):
            with pytest.raises(mcd.MCDError):
                ctx.query_pairs(mv.pairs, **bad)


def test_fp32_margin_validation(mcd):
    """Every FP32 evaluation of the static packing, in 100 sets of random
    particle orientations (about 1e8 evaluations), compared with FP64: the
    largest |d32 - d64| stays below 1/8 of the margin. A validating query's
    results equal the plain query's, and no re-decided pair falls in the
    1e-9 * delta guard band of the threshold."""
    # the packing on the nominal radius: its neighbours interpenetrate, so
    # each query evaluates about a million near triangle pairs
    sc = synth.cfg2_scene(run=0, pack_r=1.0)
    rng = np.random.default_rng(8080)
    total, worst, worst_np, banded = 0, 0.0, 0.0, 0
    with mcd.Context() as ctx:
        ids = ctx.load_scene(sc)
        pid = np.arange(sc.n_particles, dtype=np.int32)
        for it in range(100):
            if it:
                st = sc.state.copy()
                st[:, 3:7] = synth.random_quaternions(sc.n_particles, rng)
                ctx.particles_set(pid, ids[sc.mesh_of], st)
            pv, cv, sv = _q(ctx, sc.pairs, flags=mcd.Q_MIXED | mcd.Q_VALIDATE)
            if it == 0:
                pr, con, s0 = _q(ctx, sc.pairs, flags=mcd.Q_MIXED)
                assert pv.tobytes() == pr.tobytes() and cv.tobytes() == con.tobytes()
                assert s0["validated"] == 0 and s0["margin_ratio"] == 0.0 and s0["margin_ratio_np"] == 0.0
            assert sv["validated"] > 0.5 * sv["tri_pairs_evaluated"]
            total += sv["validated"]
            worst = max(worst, sv["margin_ratio"])
            worst_np = max(worst_np, sv["margin_ratio_np"])
            banded += sv["banded"]
            if it % 10 == 0:
                _say("validation", it, total, worst, worst_np)
    _say("validated", total, "largest |d32 - d64| / mu", worst, "near-parallel / (mu + c)", worst_np,
         "banded", banded)
    assert total >= 1e8
    assert worst <= 0.125
    # near-parallel edge pairs: the widened bound still holds with room
    assert worst_np <= 0.5
    assert banded == 0
