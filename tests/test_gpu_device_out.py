"""Results without a host copy: MCD_Q_DEVICE_OUT queries whose records stay in
device memory and are copied into caller device buffers (mcd_fetch_dev), and
zero-copy views of host records (mcd_result_view). Each must equal the
ordinary query's mcd_fetch output bit for bit, on the static packing."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcd():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_15417_amd as m
    return m


@pytest.fixture(scope="module")
def scene():
    return synth.cfg2_scene(run=0)


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _host(ctx, pairs, flags):
    t = ctx.query_pairs(pairs, flags=flags)
    pr, con = ctx.fetch(t)
    ctx.release(t)
    return pr.copy(), con.copy()


def _device(mcd, ctx, t):
    """A DEVICE_OUT ticket's results through mcd_fetch_dev into torch buffers."""
    import torch
    n, nc = ctx.result_sizes(t)
    res = torch.zeros((max(n, 1), mcd.PAIR_RESULT_DT.itemsize), dtype=torch.uint8, device="cuda")
    con = torch.zeros((max(nc, 1), mcd.CONTACT_DT.itemsize), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    ctx.fetch_dev(t, res.data_ptr(), res.shape[0], con.data_ptr(), con.shape[0], stream=s.cuda_stream)
    s.synchronize()
    pr = res.cpu().numpy().view(mcd.PAIR_RESULT_DT).reshape(-1)[:n]
    cr = con.cpu().numpy().view(mcd.CONTACT_DT).reshape(-1)[:nc]
    return pr, cr


def _same(a, b):
    assert a.shape == b.shape
    assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("extra", [0, 256], ids=["plain", "fused"])
def test_device_out_equals_host_records(mcd, scene, extra):
    import torch
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.load_scene(scene)
        pairs = scene.pairs
        _say("device out, host pair list", pairs.shape[0], "flags", extra)
        ref_pr, ref_con = _host(ctx, pairs, mcd.Q_MIXED | extra)
        assert ref_con.shape[0] > 0
        t = ctx.query_pairs(pairs, flags=mcd.Q_MIXED | mcd.Q_DEVICE_OUT | extra)
        pr, con = _device(mcd, ctx, t)
        _same(pr, ref_pr)
        _same(con, ref_con)
        # host pair results are still there; the records are not
        hpr, hcon = ctx.fetch(t, contacts=False)
        assert hcon is None
        _same(hpr, ref_pr)
        with pytest.raises(mcd.MCDError):
            ctx.fetch(t)
        vpr, vcon = ctx.view(t)
        assert vcon is None
        _same(vpr, ref_pr)
        ctx.release(t)
        # device pair list in, device records out; then a smaller query
        # reusing the pooled buffer
        for k, sub in enumerate((pairs, pairs[::5].copy())):
            _say("device out, device pair list", k, sub.shape[0])
            rpr, rcon = _host(ctx, sub, mcd.Q_MIXED | extra)
            d = torch.from_numpy(sub.copy()).cuda()
            torch.cuda.synchronize()
            t = ctx.query_pairs_dev(d.data_ptr(), sub.shape[0], flags=mcd.Q_MIXED | mcd.Q_DEVICE_OUT | extra)
            pr, con = _device(mcd, ctx, t)
            ctx.release(t)
            _same(pr, rpr)
            _same(con, rcon)


def test_view_equals_fetch(mcd, scene):
    import torch
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.load_scene(scene)
        _say("result view", scene.pairs.shape[0])
        t = ctx.query_pairs(scene.pairs)
        pr, con, pp = ctx.fetch(t, with_pairs=True)
        vpr, vcon, vpp = ctx.view(t, with_pairs=True)
        _same(vpr, pr)
        _same(vcon, con)
        _same(vpp, pp)
        ctx.release(t)


def test_device_out_errors(mcd, scene):
    import torch
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.load_scene(scene)
        pairs = scene.pairs[:64].copy()
        _say("device out errors")
        for flags, dt in ((mcd.Q_DEVICE_OUT, 0.01), (mcd.Q_DEVICE_OUT | mcd.Q_CONTACTS, 0.0),
                          (mcd.Q_DEVICE_OUT | mcd.Q_CLOSEST, 0.0)):
            with pytest.raises(mcd.MCDError):
                ctx.query_pairs(pairs, dt=dt, flags=flags)
        t = ctx.query_pairs(pairs)                      # host records: no device copy to fetch
        buf = torch.zeros((pairs.shape[0], mcd.PAIR_RESULT_DT.itemsize), dtype=torch.uint8, device="cuda")
        with pytest.raises(mcd.MCDError):
            ctx.fetch_dev(t, buf.data_ptr(), buf.shape[0], 0, 0)
        ctx.release(t)
        t = ctx.query_pairs(pairs, flags=mcd.Q_DEVICE_OUT)
        with pytest.raises(mcd.MCDError):               # capacity below the pair count
            ctx.fetch_dev(t, buf.data_ptr(), pairs.shape[0] - 1, 0, 0)
        ctx.fetch_dev(t, buf.data_ptr(), buf.shape[0], 0, 0, stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        ctx.release(t)
        ref, _ = _host(ctx, pairs, mcd.Q_MIXED)
        _same(buf.cpu().numpy().view(mcd.PAIR_RESULT_DT).reshape(-1), ref)


def test_batched_queries_view_and_fetch(mcd, scene):
    """Queries submitted together run as one batch and share the batch's
    contact records; each query's view (re-based in place) and fetch
    (re-based while copied), in either order, equal the query run alone."""
    import torch
    chunks = np.array_split(scene.pairs[:3000], 12)
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream, streams=1) as ctx:
        ctx.load_scene(scene)
        _say("batched queries", len(chunks))
        alone = [_host(ctx, c, mcd.Q_MIXED) for c in chunks]
        tickets = [ctx.query_pairs(c) for c in chunks]
        batched = 0
        for k, t in enumerate(tickets):
            ctx.wait(t)
            batched += ctx.stats(t)["batch_queries"] > 1
            if k % 2:
                vpr, vcon = ctx.view(t)
                vcon = vcon.copy()
                pr, con = ctx.fetch(t)
            else:
                pr, con = ctx.fetch(t)
                vpr, vcon = ctx.view(t)
                vcon = vcon.copy()
            ctx.release(t)
            _same(pr, alone[k][0])
            _same(con, alone[k][1])
            _same(vcon, alone[k][1])
            assert con.shape[0] == 0 or con["pair"].max() < chunks[k].shape[0]
        assert batched > 0
