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
    keep = oracle.filtered_mask(oracle.pair_margins(d["a_xy"], d["b_xy"], d.get("a_nv"),
                                                    d.get("b_nv"), threads=8))
    assert np.abs(iou.detach().cpu().numpy() - ref).max() <= IOU_TOL
    ga, gb, _, _ = oracle.iou_pairs_grad(d["a_xy"], d["b_xy"], d["grad"], nx, xf, d.get("a_nv"),
                                         d.get("b_nv"), threads=8)
    n = len(ref)
    err = grad_rel_err(np.concatenate([a.grad.cpu().numpy().reshape(n, -1),
                                       b.grad.cpu().numpy().reshape(n, -1)], 1),
                       np.concatenate([ga.reshape(n, -1), gb.reshape(n, -1)], 1))
    assert err[keep].max() <= GRAD_TOL
