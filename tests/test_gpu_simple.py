"""GPU parity of the simple-polygon (non-convex) IoU path through the C ABI
against the FP64 simple-polygon oracle: IoU to 1e-5 on every pair, the saved
crossing / entering masks and vertex-0 inclusion bit-exact on every pair
(contacts resolved by the tie rule on both sides), gradients to 1e-3
relative on pairs in general position."""
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


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _check(dg, a, b, a_nv=None, b_nv=None, grad=None, min_keep=0.9):
    n = len(a)
    ta, tb, tan, tbn = dev_t(a), dev_t(b), dev_t(a_nv), dev_t(b_nv)
    iou, xm, sm, ins = dg.iou_simple_pairs(ta, tb, tan, tbn)
    if grad is None:
        grad = np.random.default_rng(0).uniform(-1, 1, n).astype(np.float32)
    ga, gb = dg.iou_simple_backward(ta, tb, dev_t(grad), xm, sm, ins, tan, tbn)
    dg.check_errors()
    iou, ins = iou.cpu().numpy(), ins.cpu().numpy()
    xm, sm = _u64(xm), _u64(sm)
    r_iou, r_xm, r_sm, r_ins, bad = oracle.simple_iou_pairs(a, b, a_nv, b_nv, threads=16)
    assert bad == 0
    d = np.abs(iou.astype(np.float64) - r_iou)
    assert d.max() <= IOU_TOL, (d.max(), int(d.argmax()))
    keep = oracle.simple_filtered_mask(oracle.simple_margins(a, b, a_nv, b_nv, threads=16))
    assert keep.mean() >= min_keep
    assert np.array_equal(xm[keep], r_xm[keep])
    assert np.array_equal(sm[keep], r_sm[keep])
    assert np.array_equal(ins[keep], r_ins[keep])
    # every pair: the masks are functions of exact, tie-ruled signs alone
    assert np.array_equal(xm, r_xm), np.nonzero(xm != r_xm)[0][:5]
    assert np.array_equal(sm, r_sm), np.nonzero(sm != r_sm)[0][:5]
    assert np.array_equal(ins, r_ins), np.nonzero(np.any(ins != r_ins, axis=-1) if ins.ndim > 1 else ins != r_ins)[0][:5]
    r_ga, r_gb = oracle.simple_iou_pairs_grad(a, b, grad, a_nv, b_nv, threads=16)
    g = np.concatenate([ga.cpu().numpy().reshape(n, -1), gb.cpu().numpy().reshape(n, -1)], 1)
    r = np.concatenate([r_ga.reshape(n, -1), r_gb.reshape(n, -1)], 1)
    err = grad_rel_err(g, r)
    assert err[keep].max() <= GRAD_TOL, (err[keep].max(), int(np.flatnonzero(keep)[err[keep].argmax()]))
    return {"n": n, "filtered": float(keep.mean()), "max_iou_err": float(d.max()),
            "max_grad_err": float(err[keep].max())}


def test_simple_polygons_ragged(dg):
    n = 65536 + 77
    _say(f"case: simple 3..8-gon pairs {n}")
    d = synth.c4_simple(n=n, seed=301)
    _say(str(_check(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], d["grad"])))


def test_simple_full_size(dg):
    d = synth.c4_simple()
    _say(f"case: simple full {len(d['a_xy'])} pairs")
    _say(str(_check(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], d["grad"])))


def test_simple_quads(dg):
    """Four-slot kernels: non-convex quadrilaterals, fixed count."""
    rng = np.random.default_rng(302)
    n = 30000
    ca = rng.uniform(-1, 1, (n, 2))
    a, _ = synth.random_simple(rng, n, ca, kmin=4, kmax=4)
    b, _ = synth.random_simple(rng, n, ca + rng.normal(0, 0.5, (n, 2)), kmin=4, kmax=4)
    _say(f"case: simple quads {n}")
    _say(str(_check(dg, a, b)))


def test_convex_inputs_match_convex_path(dg):
    """On convex polygons the two paths compute the same IoU and gradient."""
    for d in (synth.c3_pairs(n=20000, seed=303), synth.c4_polygons(n=20000, seed=304)):
        a, b, an, bn, g = d["a_xy"], d["b_xy"], d.get("a_nv"), d.get("b_nv"), d["grad"]
        _say(f"case: convex inputs {len(a)}")
        _check(dg, a, b, an, bn, g)
        ta, tb, tan, tbn = dev_t(a), dev_t(b), dev_t(an), dev_t(bn)
        i1, xm, sm, ins = dg.iou_simple_pairs(ta, tb, tan, tbn)
        i2, nx, xf = dg.iou_pairs(ta, tb, tan, tbn)
        assert (i1 - i2).abs().max().item() <= 2 * IOU_TOL


def test_rectilinear_contacts(dg):
    """Integer rectilinear shapes (exact in fp32) touch along edges and at
    vertices; the tie rule resolves every contact as a motion of b, and the
    area is continuous in that motion, so the IoU is the exact one and the
    saved state is the oracle's (which applies the same rule)."""
    rng = np.random.default_rng(305)
    shapes = []
    for _ in range(4000):
        w, h = int(rng.integers(3, 8)), int(rng.integers(3, 8))
        if rng.integers(0, 2):
            a_, b_ = int(rng.integers(1, w)), int(rng.integers(1, h))
            v = [(0, 0), (w, 0), (w, b_), (a_, b_), (a_, h), (0, h)]
        else:
            v = [(0, 0), (w, 0), (w, h), (0, h)]
        v = np.array(v + [v[0]] * (8 - len(v)), np.float32)
        shapes.append((v + rng.integers(-4, 5, 2).astype(np.float32), len(set(map(tuple, v)))))
    a = np.stack([s[0] for s in shapes[:2000]])
    b = np.stack([s[0] for s in shapes[2000:]])
    an = np.array([s[1] for s in shapes[:2000]], np.uint8)
    bn = np.array([s[1] for s in shapes[2000:]], np.uint8)
    _say("case: rectilinear contacts 2000")
    iou, xm, sm, ins = dg.iou_simple_pairs(dev_t(a), dev_t(b), dev_t(an), dev_t(bn))
    ref, r_xm, r_sm, r_ins, _ = oracle.simple_iou_pairs(a, b, an, bn)
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    # the contacts are exact, so the tie-ruled masks are the oracle's too
    assert np.array_equal(_u64(xm), r_xm) and np.array_equal(_u64(sm), r_sm)
    assert np.array_equal(ins.cpu().numpy(), r_ins)


def test_snapped_simple_polygons(dg):
    """Random simple 3..8-gons snapped to a grid of 1/4: collinear edges,
    vertices on edges and shared vertices everywhere; IoU on every pair and
    the tie-ruled masks bit-exact on every pair."""
    rng = np.random.default_rng(1900)
    n = 20000
    c = rng.uniform(-1, 1, (n, 2))
    a, an = synth.random_simple(rng, n, c, kmin=3, kmax=8)
    b, bn = synth.random_simple(rng, n, c + rng.normal(0, 0.4, (n, 2)), kmin=3, kmax=8)
    a = np.round(a * 4).astype(np.float32)
    b = np.round(b * 4).astype(np.float32)
    keep = (oracle.simple_status(a, an) == 0) & (oracle.simple_status(b, bn) == 0)
    a, b, an, bn = a[keep], b[keep], an[keep], bn[keep]
    _say(f"case: snapped simple polygons {len(a)}")
    iou, xm, sm, ins = dg.iou_simple_pairs(dev_t(a), dev_t(b), dev_t(an), dev_t(bn))
    dg.check_errors()
    ref, r_xm, r_sm, r_ins, bad = oracle.simple_iou_pairs(a, b, an, bn, threads=16)
    assert bad == 0
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    assert np.array_equal(_u64(xm), r_xm) and np.array_equal(_u64(sm), r_sm)
    assert np.array_equal(ins.cpu().numpy(), r_ins)


def test_identical_disjoint_empty(dg):
    d = synth.c4_simple(n=4096, seed=306)
    a, an = dev_t(d["a_xy"]), dev_t(d["a_nv"])
    iou, _, _, _ = dg.iou_simple_pairs(a, a, an, an)
    assert (iou - 1).abs().max().item() <= IOU_TOL
    far = a + torch.tensor([100.0, 0.0], device=a.device)
    iou, xm, sm, ins = dg.iou_simple_pairs(a, far, an, an)
    assert iou.abs().max().item() == 0.0 and xm.abs().max().item() == 0
    g = torch.ones(len(a), device=a.device)
    ga, gb = dg.iou_simple_backward(a, far, g, xm, sm, ins, an, an)
    assert ga.abs().max().item() == 0.0 and gb.abs().max().item() == 0.0
    e = torch.zeros((0, 8, 2), device=a.device)
    iou, xm, sm, ins = dg.iou_simple_pairs(e, e)
    assert iou.numel() == 0


def test_autograd_simple(dg):
    d = synth.c4_simple(n=2048, seed=307)
    a = dev_t(d["a_xy"]).requires_grad_(True)
    b = dev_t(d["b_xy"]).requires_grad_(True)
    an, bn = dev_t(d["a_nv"]), dev_t(d["b_nv"])
    iou = dg.IoUSimplePairs.apply(a, b, an, bn)
    (iou * dev_t(d["grad"])).sum().backward()
    r_ga, r_gb = oracle.simple_iou_pairs_grad(d["a_xy"], d["b_xy"], d["grad"], d["a_nv"], d["b_nv"])
    keep = oracle.simple_filtered_mask(oracle.simple_margins(d["a_xy"], d["b_xy"], d["a_nv"],
                                                             d["b_nv"]))
    n = len(d["a_xy"])
    err = grad_rel_err(np.concatenate([a.grad.cpu().numpy().reshape(n, -1),
                                       b.grad.cpu().numpy().reshape(n, -1)], 1),
                       np.concatenate([r_ga.reshape(n, -1), r_gb.reshape(n, -1)], 1))
    assert err[keep].max() <= GRAD_TOL
