"""GPU parity of the fused box front end (box parameters -> corners in-kernel
-> IoU, and the backward down to the parameters) against the FP64 oracle,
which forms the corners from the same fp32 parameters in fp64."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import GRAD_TOL, IOU_TOL, dev_t, grad_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


def _say(msg):
    print(msg, flush=True)


def _corners(box):
    """Corners of the boxes in fp64, rounded to fp32 (for the filter only)."""
    b = np.asarray(box, np.float64)
    return synth.boxes_to_quads(b[:, 0], b[:, 1], b[:, 2], b[:, 3], b[:, 4])


def _check_boxes(dg, a, b, grad):
    n = len(a)
    ta, tb = dev_t(a), dev_t(b)
    iou, nx, xf = dg.iou_boxes(ta, tb)
    dg.check_errors()
    ga, gb = dg.iou_boxes_backward(ta, tb, dev_t(grad), nx, xf)
    iou, nx, xf = iou.cpu().numpy(), nx.cpu().numpy(), xf.cpu().numpy()
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    r_iou, r_nx, r_xf, bad = oracle.iou_boxes(a, b, threads=8)
    assert bad == 0
    # the GPU's fp32 corners differ from the oracle's fp64 ones by a few ulp;
    # the non-degenerate filter (margins far above that) is taken on the
    # corners rounded to fp32
    keep = oracle.filtered_mask(oracle.pair_margins(_corners(a), _corners(b), threads=8))
    assert keep.mean() > 0.5
    assert np.array_equal(nx[keep], r_nx[keep])
    assert np.array_equal(xf[keep], r_xf[keep])
    d = np.abs(iou.astype(np.float64) - r_iou)
    assert d.max() <= IOU_TOL, d.max()
    r_ga, r_gb = oracle.iou_boxes_grad(a, b, grad, r_nx, r_xf, threads=8)
    err = grad_rel_err(np.concatenate([ga, gb], 1), np.concatenate([r_ga, r_gb], 1))
    assert err[keep].max() <= GRAD_TOL, err[keep].max()
    return {"n": n, "filtered": float(keep.mean()), "max_iou_err": float(d.max()),
            "max_grad_err": float(err[keep].max())}


def test_boxes_2d(dg):
    n = 65536 + 17
    _say(f"case: boxes 2D {n} pairs")
    d = synth.c3_boxes(n=n, seed=111)
    _say(str(_check_boxes(dg, d["a_box"], d["b_box"], d["grad"])))


def test_boxes_full_size(dg):
    """The benchmark's box workload: 1,048,576 box-parameter pairs, every pair
    against the oracle."""
    d = synth.c3_boxes()
    _say(f"case: boxes 2D full {len(d['a_box'])} pairs")
    _say(str(_check_boxes(dg, d["a_box"], d["b_box"], d["grad"])))


def test_boxes_3d(dg):
    n = 32768 + 5
    _say(f"case: boxes 3D {n} pairs")
    d = synth.c3_boxes(n=n, seed=112, three_d=True)
    _say(str(_check_boxes(dg, d["a_box"], d["b_box"], d["grad"])))


def test_boxes_match_corner_path(dg):
    """The fused path and the vertex path on the GPU's own inputs agree."""
    d = synth.c3_boxes(n=4096, seed=113)
    iou_b, _, _ = dg.iou_boxes(dev_t(d["a_box"]), dev_t(d["b_box"]))
    iou_v, _, _ = dg.iou_pairs(dev_t(_corners(d["a_box"])), dev_t(_corners(d["b_box"])))
    assert (iou_b - iou_v).abs().max().item() <= IOU_TOL


def test_boxes_axis_aligned_contacts(dg):
    """Axis-aligned boxes (yaw 0) on integer centres with integer sizes: the
    fp32 and fp64 corners are the same exact values, shared and collinear
    edges and corner touches are common, and the count and flag sequence
    equal the oracle's on every pair."""
    rng = np.random.default_rng(115)
    n = 20000

    def boxes():
        return np.stack([rng.integers(-3, 4, n), rng.integers(-3, 4, n),
                         rng.integers(1, 4, n), rng.integers(1, 4, n), np.zeros(n)],
                        1).astype(np.float32)

    a, b = boxes(), boxes()
    _say("case: axis-aligned integer boxes 20000")
    iou, nx, xf = dg.iou_boxes(dev_t(a), dev_t(b))
    dg.check_errors()
    iou, nx, xf = iou.cpu().numpy(), nx.cpu().numpy(), xf.cpu().numpy()
    r_iou, r_nx, r_xf, bad = oracle.iou_boxes(a, b, threads=8)
    assert bad == 0
    assert np.abs(iou - r_iou).max() <= IOU_TOL
    assert np.array_equal(nx, r_nx)
    assert np.array_equal(xf, r_xf)
    assert (nx > 0).mean() > 0.15  # a fifth of the pairs overlap


def test_boxes_autograd_and_edges(dg):
    d = synth.c3_boxes(n=1000, seed=114)
    a = dev_t(d["a_box"]).requires_grad_(True)
    b = dev_t(d["b_box"]).requires_grad_(True)
    g = dev_t(d["grad"])
    iou = dg.IoUBoxes.apply(a, b)
    (iou * g).sum().backward()
    r_iou, r_nx, r_xf, _ = oracle.iou_boxes(d["a_box"], d["b_box"])
    r_ga, r_gb = oracle.iou_boxes_grad(d["a_box"], d["b_box"], d["grad"], r_nx, r_xf)
    keep = oracle.filtered_mask(oracle.pair_margins(_corners(d["a_box"]), _corners(d["b_box"])))
    err = grad_rel_err(np.concatenate([a.grad.cpu().numpy(), b.grad.cpu().numpy()], 1),
                       np.concatenate([r_ga, r_gb], 1))
    assert err[keep].max() <= GRAD_TOL
    # empty batch; identical boxes give 1
    z = torch.zeros((0, 5), device="cuda")
    assert dg.iou_boxes(z, z)[0].shape == (0,)
    same = dev_t(d["a_box"][:64])
    assert (dg.iou_boxes(same, same)[0] - 1).abs().max().item() <= IOU_TOL
