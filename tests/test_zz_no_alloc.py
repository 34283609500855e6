"""The allocation-free matrix forward (dgal_iou_matrix_noalloc) through the C
ABI, against dgal_iou_matrix on the same inputs: two calls in a row on the
library's shared static scratch, the second with a smaller input, then a
block over the scratch's tile limit, refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import IOU_TOL, dev_t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available()
    return d


def _say(msg):
    print(msg, flush=True)


def _both(dg, a, b, a_off, self_pairs, a_z=None):
    """IoU of the same call through dgal_iou_matrix (with a work list) and
    through dgal_iou_matrix_noalloc (the library's scratch); returns both."""
    dev = a.device
    pa, _ = dg.polys(a, None, a_z)
    pb, _ = dg.polys(b, None, a_z if self_pairs else None)
    seg = dg.segments(a.shape[0], b.shape[0], a_off, None, self_pairs=self_pairs)
    d_a, d_b, d_o, nseg, total, tiles, _ = seg
    ptr = lambda t: None if t is None else t.data_ptr()
    stream = torch.cuda.current_stream().cuda_stream
    ctx = dg.context(dev)
    ref = torch.full((total,), -7.0, device=dev)
    saved = dg.SavedPairs(max(1 << 16, total // 16), a.shape[1] + b.shape[1], tiles, dev)
    st = dg.lib.dgal_iou_matrix(ctx, pa, pb, ptr(d_a), ptr(d_b), ptr(d_o), nseg, int(self_pairs),
                                ref.data_ptr(), total, ctypes.byref(saved.struct()), stream)
    assert st == dg.DGAL_OK, st
    got = torch.full((total,), -7.0, device=dev)
    st = dg.lib.dgal_iou_matrix_noalloc(ctx, pa, pb, ptr(d_a), ptr(d_b), ptr(d_o), nseg,
                                        int(self_pairs), got.data_ptr(), total, stream)
    assert st == dg.DGAL_OK, st
    torch.cuda.synchronize()
    dg.check_errors(dev)
    return got, ref, int(saved.count.item())


def test_noalloc_matches_matrix_call_twice(dg):
    # first call: 12 ragged scenes of 3D boxes, per-scene self pairs
    d = synth.c5_scenes(scenes=12, nmin=50, nmax=1200, seed=77)
    xy, lo, hi, off = d["a_xy"], d["a_zlo"], d["a_zhi"], d["off"]
    _say(f"case: no-alloc scenes {len(xy)} boxes, {int(d['out_off'][-1])} pairs")
    a = dev_t(xy)
    got, ref, surv = _both(dg, a, a, off, True, (dev_t(lo), dev_t(hi)))
    assert surv > 1000
    assert torch.equal(got, ref)
    # the first scene against the oracle as well
    n0 = int(off[1])
    r0, _ = oracle.iou_matrix(xy[:n0], a_z=(lo[:n0], hi[:n0]),
                              a_off=np.array([0, n0], np.int64), self_pairs=True)
    assert np.abs(got[:n0 * n0].cpu().numpy() - r0).max() <= IOU_TOL
    # second call, smaller: one 2D block of two crowded sets
    d2 = synth.c2_matrix(n=300, m=257, seed=3)
    c = d2["a_xy"].astype(np.float64).mean(1, keepdims=True)
    a2 = (d2["a_xy"] - c + 0.1 * c).astype(np.float32)
    c = d2["b_xy"].astype(np.float64).mean(1, keepdims=True)
    b2 = (d2["b_xy"] - c + 0.1 * c).astype(np.float32)
    _say("case: no-alloc block 300 x 257 after the scenes")
    got2, ref2, surv2 = _both(dg, dev_t(a2), dev_t(b2), None, False)
    assert 0 < surv2 < surv
    assert torch.equal(got2, ref2)
    r2, _ = oracle.iou_matrix(a2, b2)
    assert np.abs(got2.cpu().numpy() - r2).max() <= IOU_TOL


def test_noalloc_refuses_a_block_over_the_tile_limit(dg):
    """One block of 8 x 65537 rows against 256 columns needs 65,537 tiles:
    refused on the host (DGAL_ECAPACITY), the output left untouched (it is
    allocated whole, so that nothing could write outside it)."""
    rows = 8 * (65536 + 1)
    a = torch.zeros((rows, 4, 2), device="cuda")
    b = torch.zeros((256, 4, 2), device="cuda")
    out = torch.full((rows * 256,), -7.0, device="cuda")
    pa, _ = dg.polys(a)
    pb, _ = dg.polys(b)
    st = dg.lib.dgal_iou_matrix_noalloc(dg.context(a.device), pa, pb, None, None, None, 0, 0,
                                        out.data_ptr(), rows * 256,
                                        torch.cuda.current_stream().cuda_stream)
    assert st == dg.DGAL_ECAPACITY, st
    torch.cuda.synchronize()
    assert torch.all(out == -7.0)
    dg.check_errors(a.device)
