"""The plain per-op GPU form used as the benchmark's "vs plain" denominator
computes the same IoU and gradients as the oracle (so the speedup compares
like with like)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import GRAD_TOL, IOU_TOL, grad_rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wl", ["c3", "c4"])
def test_plain_form_matches_oracle(wl):
    from bench_plain import iou_pairs_plain
    d = synth.get(wl, n=30000, seed=17)
    a = torch.from_numpy(d["a_xy"]).cuda().requires_grad_(True)
    b = torch.from_numpy(d["b_xy"]).cuda().requires_grad_(True)
    anv = None if "a_nv" not in d else torch.from_numpy(d["a_nv"]).cuda()
    bnv = None if "b_nv" not in d else torch.from_numpy(d["b_nv"]).cuda()
    iou = iou_pairs_plain(a, b, anv, bnv)
    iou.backward(torch.from_numpy(d["grad"]).cuda())
    ref, nx, xf, _ = oracle.iou_pairs(d["a_xy"], d["b_xy"], d.get("a_nv"), d.get("b_nv"), threads=8)
    marg = oracle.pair_margins(d["a_xy"], d["b_xy"], d.get("a_nv"), d.get("b_nv"), threads=8)
    # the plain form is fp32 throughout (no fp64 rebuild): sliver intersections,
    # whose fp32 gradient carries ~u F / sqrt(I), stay out of its gradient bar
    keep = oracle.filtered_mask(marg) & (marg[:, 4] >= oracle.FILTER_SLIVER)
    assert np.abs(iou.detach().cpu().numpy() - ref).max() <= IOU_TOL
    ga, gb, _, _ = oracle.iou_pairs_grad(d["a_xy"], d["b_xy"], d["grad"], nx, xf, d.get("a_nv"),
                                         d.get("b_nv"), threads=8)
    n = len(ref)
    err = grad_rel_err(np.concatenate([a.grad.cpu().numpy().reshape(n, -1),
                                       b.grad.cpu().numpy().reshape(n, -1)], 1),
                       np.concatenate([ga.reshape(n, -1), gb.reshape(n, -1)], 1))
    assert err[keep].max() <= GRAD_TOL


def test_plain_scenes_match_oracle():
    """The plain form of the per-scene 3D self-pair matrix (the scenes
    benchmark's "vs plain" denominator) against the oracle: IoU on every
    pair, and per-box gradients scaled by the sum of each box's pair terms."""
    from bench_plain import iou3d_scenes_plain
    d = synth.c5_scenes(scenes=3, nmin=60, nmax=150, seed=18)
    xy, lo, hi, off = d["a_xy"], d["a_zlo"], d["a_zhi"], d["off"]
    c = xy.astype(np.float64).mean(1, keepdims=True)
    xy = (xy - c + 0.1 * c).astype(np.float32)  # crowd the boxes so that many pairs overlap
    t = [torch.from_numpy(v).cuda().requires_grad_(True) for v in (xy, lo, hi)]
    iou = iou3d_scenes_plain(t[0], t[1], t[2], off)
    g = np.random.default_rng(19).uniform(-1, 1, iou.shape[0]).astype(np.float32)
    iou.backward(torch.from_numpy(g).cuda())
    ref, _ = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.abs(iou.detach().cpu().numpy() - ref).max() <= IOU_TOL
    assert np.count_nonzero(ref) > 3 * len(xy)
    ga, _, gz, _ = oracle.iou_matrix_grad(g, xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    got = np.concatenate([t[0].grad.cpu().numpy().reshape(len(xy), -1),
                          t[1].grad.cpu().numpy()[:, None], t[2].grad.cpu().numpy()[:, None]], 1)
    want = np.concatenate([ga.reshape(len(xy), -1), gz], 1)
    # continuous random boxes: no ties, so either evaluation order of a pair
    # has the same structure; bar relative to each box's gradient magnitude
    err = np.linalg.norm(got - want, axis=1) / np.maximum(np.linalg.norm(want, axis=1), 1e-3)
    assert err.max() <= 10 * GRAD_TOL, err.max()
