"""The allocation-free entry point (mcd_query_pairs_noalloc) against the
device-list query it varies (mcd_query_pairs_dev), through the C ABI: two
calls in a row, the second with a smaller input, each bit-identical to the
allocating query on the same pairs; results written into caller-owned
device memory."""

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


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _noalloc(mcd, ctx, pairs, cap):
    import torch
    d = torch.from_numpy(pairs.copy()).cuda()
    res = torch.zeros((pairs.shape[0], mcd.PAIR_RESULT_DT.itemsize), dtype=torch.uint8, device="cuda")
    con = torch.zeros((max(cap, 1), mcd.CONTACT_DT.itemsize), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    n = ctx.query_pairs_noalloc(d.data_ptr(), pairs.shape[0], res.data_ptr(), con.data_ptr(), cap,
                                stream=torch.cuda.current_stream().cuda_stream)
    pr = res.cpu().numpy().view(mcd.PAIR_RESULT_DT).reshape(-1)
    cr = con.cpu().numpy().view(mcd.CONTACT_DT).reshape(-1)[:n]
    return pr, cr


def _reference(mcd, ctx, pairs):
    import torch
    d = torch.from_numpy(pairs.copy()).cuda()
    torch.cuda.synchronize()
    t = ctx.query_pairs_dev(d.data_ptr(), pairs.shape[0], flags=mcd.Q_MIXED)
    pr, con = ctx.fetch(t)
    ctx.release(t)
    return pr.copy(), con.copy()


def test_noalloc_equals_device_list_query(mcd):
    import torch
    sc = synth.cfg2_scene(run=0)                 # the static packing, 4,400 pairs
    small = sc.pairs[::7].copy()                 # then a smaller input
    with mcd.Context(stream=torch.cuda.current_stream().cuda_stream) as ctx:
        ctx.load_scene(sc)
        for k, pairs in enumerate((sc.pairs, small)):
            _say("no-alloc call", k, pairs.shape[0])
            ref_pr, ref_con = _reference(mcd, ctx, pairs)
            assert ref_con.shape[0] > 0
            pr, con = _noalloc(mcd, ctx, pairs, ref_con.shape[0] + 16)
            assert pr.tobytes() == ref_pr.tobytes()
            assert con.tobytes() == ref_con.tobytes()
        # a contact buffer too small: the count comes back with the error
        with pytest.raises(mcd.MCDError):
            _noalloc(mcd, ctx, small, 1)
        # after the error the array still serves a correct query
        pr, con = _noalloc(mcd, ctx, small, ref_con.shape[0] + 16)
        assert pr.tobytes() == ref_pr.tobytes() and con.tobytes() == ref_con.tobytes()
