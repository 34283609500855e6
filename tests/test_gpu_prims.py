"""GPU parity of the exported geometry primitives (intersection polygon with
nx / xflags, polygon area, and their backward kernels, through the C ABI)
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import GRAD_TOL, conditioned_mask, dev_t, grad_rel_err

pytestmark = pytest.mark.gpu

# Vertex tolerance.  A crossing is P_i + t e_i with t = o_i / (o_i - o_i1);
# the fp32 orientations carry at most 8u E D absolute error (u = 2^-24, the
# certification bound), so the vertex moves along e_i by at most
# 8u E D / (|f_j| |sin|): relative to the pair's coordinate scale,
# ~ 8u (E / |f_j|) / |sin| with E / |f_j| <= 4 on these shapes.  Vertex
# codes and the final shift back by P_0 add a few ulp of the scale.
U = 2.0 ** -24


def _vertex_tol(scale, sin_min):
    return scale * (32 * U / np.maximum(sin_min, 1e-3) + 8 * U)


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


def _say(msg):
    print(msg, flush=True)


def _check_intersect(dg, a, b, a_nv=None, b_nv=None, seed=0):
    n, ka = a.shape[:2]
    kb = b.shape[1]
    cap = ka + kb
    ta, tb, tan, tbn = dev_t(a), dev_t(b), dev_t(a_nv), dev_t(b_nv)
    xy, nx, xf = dg.intersect(ta, tb, tan, tbn)
    dg.check_errors()
    xy, nx, xf = xy.cpu().numpy(), nx.cpu().numpy(), xf.cpu().numpy()
    r_xy, r_nx, r_xf, bad = oracle.intersect_pairs(a, b, a_nv, b_nv, threads=8)
    assert bad == 0
    marg = oracle.pair_margins(a, b, a_nv, b_nv, threads=8)
    keep = oracle.filtered_mask(marg)
    assert keep.mean() > 0.5
    # every pair: the same count and flag sequence (the signs that select and
    # order the vertices are exact on both sides)
    assert np.array_equal(nx, r_nx)
    assert np.array_equal(xf, r_xf)
    # slots past nx are zero on every pair
    past = np.arange(cap)[None, :] >= nx[:, None]
    assert np.all(xy[past] == 0.0)
    scale = np.maximum(1.0, np.maximum(np.abs(a).reshape(n, -1).max(1), np.abs(b).reshape(n, -1).max(1)))
    err = np.abs(xy.astype(np.float64) - r_xy).reshape(n, -1).max(1)
    tol = _vertex_tol(scale, marg[:, 1])
    assert np.all(err[keep] <= tol[keep]), (err[keep].max(), np.max(err[keep] / tol[keep]))
    # backward: random upstream gradient on the vertices
    rng = np.random.default_rng(seed)
    g = rng.uniform(-1, 1, (n, cap, 2)).astype(np.float32)
    g[past] = 0.0
    ga, gb = dg.intersect_backward(ta, tb, dev_t(g), dev_t(r_nx), dev_t(r_xf), tan, tbn)
    r_ga, r_gb = oracle.intersect_pairs_grad(a, b, g, r_nx, r_xf, a_nv, b_nv, threads=8)
    gg = np.concatenate([ga.cpu().numpy().reshape(n, -1), gb.cpu().numpy().reshape(n, -1)], 1)
    rr = np.concatenate([r_ga.reshape(n, -1), r_gb.reshape(n, -1)], 1)
    gerr = grad_rel_err(gg, rr)
    cond = conditioned_mask(marg)
    assert gerr[cond].max() <= GRAD_TOL, gerr[cond].max()
    return {"n": n, "filtered": float(keep.mean()), "max_vertex_err": float(err[keep].max()),
            "max_vertex_err_over_tol": float(np.max(err[keep] / tol[keep])),
            "max_grad_err": float(gerr[cond].max()), "max_grad_err_all": float(gerr.max())}


def test_intersect_grid_contacts(dg):
    """Integer rectangles and diamonds on a small grid (contacts on most
    pairs): count and set of codes equal the oracle's on every pair, and
    every vertex the oracle places at a code is the GPU's vertex of that code
    to a few ulp of the coordinates, in the same sequence."""
    rng = np.random.default_rng(2300)
    shapes = []
    for _ in range(20000):
        x0, y0 = rng.integers(-3, 3, 2)
        w, h = rng.integers(1, 4, 2)
        if rng.integers(0, 2):
            v = [(x0, y0), (x0 + w, y0), (x0 + w, y0 + h), (x0, y0 + h)]
        else:
            v = [(x0 + w, y0), (x0, y0 + w), (x0 - w, y0), (x0, y0 - w)]
        shapes.append(v)
    a = np.array(shapes[:10000], np.float32)
    b = np.array(shapes[10000:], np.float32)
    _say("case: intersect grid contacts 10000")
    xy, nx, xf = dg.intersect(dev_t(a), dev_t(b))
    dg.check_errors()
    xy, nx, xf = xy.cpu().numpy(), nx.cpu().numpy(), xf.cpu().numpy()
    r_xy, r_nx, r_xf, bad = oracle.intersect_pairs(a, b, threads=8)
    assert bad == 0
    assert np.array_equal(nx, r_nx)
    assert np.array_equal(xf, r_xf)
    # match vertices by code (codes are unique within a pair)
    worst = 0.0
    for i in np.flatnonzero(nx):
        m = int(nx[i])
        pos = {int(c): xy[i, k] for k, c in enumerate(xf[i, :m])}
        for k, c in enumerate(r_xf[i, :m]):
            worst = max(worst, float(np.abs(pos[int(c)] - r_xy[i, k]).max()))
    assert worst <= 8 * 2.0 ** -24 * 8, worst
    assert (nx > 0).mean() > 0.15


def test_intersect_rectangles(dg):
    _say("case: intersect c1 rectangles 1024 pairs")
    d = synth.c1_pairs()
    _say(str(_check_intersect(dg, d["a_xy"], d["b_xy"], seed=1)))


def test_intersect_rectangles_ragged_many_blocks(dg):
    n = 65536 + 333
    _say(f"case: intersect c3 rectangles {n} pairs")
    d = synth.c3_pairs(n=n, seed=91)
    _say(str(_check_intersect(dg, d["a_xy"], d["b_xy"], seed=2)))


def test_intersect_full_size(dg):
    """The benchmark's intersection workload: 1,048,576 rectangle pairs with
    its per-vertex upstream gradient, the backward fed the GPU's own nx /
    xflags as the benchmark does; every pair against the oracle."""
    d = synth.c3_intersect()
    a, b, g = d["a_xy"], d["b_xy"], d["grad_xy"]
    n = len(a)
    _say(f"case: intersect c3 full {n} pairs")
    ta, tb = dev_t(a), dev_t(b)
    xy, nx, xf = dg.intersect(ta, tb)
    ga, gb = dg.intersect_backward(ta, tb, dev_t(g), nx, xf)
    dg.check_errors()
    xy, nx, xf = xy.cpu().numpy(), nx.cpu().numpy(), xf.cpu().numpy()
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    r_xy, r_nx, r_xf, bad = oracle.intersect_pairs(a, b, threads=16)
    assert bad == 0
    marg = oracle.pair_margins(a, b, threads=16)
    keep = oracle.filtered_mask(marg)
    assert keep.mean() > 0.9
    assert np.array_equal(nx, r_nx)
    assert np.array_equal(xf, r_xf)
    assert np.all((nx == 0) | ((nx >= 3) & (nx <= 8)))
    scale = np.maximum(1.0, np.maximum(np.abs(a).reshape(n, -1).max(1),
                                       np.abs(b).reshape(n, -1).max(1)))
    err = np.abs(xy.astype(np.float64) - r_xy).reshape(n, -1).max(1)
    tol = _vertex_tol(scale, marg[:, 1])
    assert np.all(err[keep] <= tol[keep]), np.max(err[keep] / tol[keep])
    r_ga, r_gb = oracle.intersect_pairs_grad(a, b, g, r_nx, r_xf, threads=16)
    gerr = grad_rel_err(np.concatenate([ga.reshape(n, -1), gb.reshape(n, -1)], 1),
                        np.concatenate([r_ga.reshape(n, -1), r_gb.reshape(n, -1)], 1))
    cond = conditioned_mask(marg)
    assert gerr[cond].max() <= GRAD_TOL, gerr[cond].max()
    _say(str({"filtered": float(keep.mean()), "max_vertex_err_over_tol":
              float(np.max(err[keep] / tol[keep])), "max_grad_err": float(gerr[cond].max()),
              "max_grad_err_all": float(gerr.max())}))


def test_intersect_polygons(dg):
    _say("case: intersect c4 polygons 8192 pairs")
    d = synth.c4_polygons(n=8192, seed=92)
    _say(str(_check_intersect(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], seed=3)))


def test_intersect_odd_capacity(dg):
    """Triangles stored with kmax 3 against quads: capacity 7, unaligned rows."""
    _say("case: intersect kmax 3 x 4, capacity 7")
    d = synth.c4_polygons(n=4096, seed=93)
    a = np.ascontiguousarray(d["a_xy"][:, :3])
    b = synth.c1_pairs(n=4096, seed=94)["b_xy"]
    keep_tri = np.array([oracle.polygon_valid(p.astype(np.float64)) for p in a])
    a, b = a[keep_tri], b[keep_tri]
    _say(str(_check_intersect(dg, a, b, None, None, seed=4)))


def test_intersect_nested_and_empty(dg):
    outer = np.array([[[-4, -4], [4, -4], [4, 4], [-4, 4]]] * 2, np.float32)
    inner = np.array([[[-1, -0.5], [1.5, -1], [1, 1], [-0.5, 1.25]],
                      [[10, 10], [11, 10], [11, 11], [10, 11]]], np.float32)
    xy, nx, xf = dg.intersect(dev_t(outer), dev_t(inner))
    nx, xf, xy = nx.cpu().numpy(), xf.cpu().numpy(), xy.cpu().numpy()
    assert nx.tolist() == [4, 0]
    assert sorted(xf[0, :4].tolist()) == [0x10, 0x11, 0x12, 0x13] and np.all(xf[1] == 0xFF)
    assert np.all(xy[1] == 0.0)
    for r in range(4):
        assert np.array_equal(xy[0, r], inner[0, xf[0, r] & 0x0F])
    g = np.zeros((2, 8, 2), np.float32)
    g[0, :4] = np.arange(8, dtype=np.float32).reshape(4, 2) + 1
    ga, gb = dg.intersect_backward(dev_t(outer), dev_t(inner), dev_t(g), dev_t(nx), dev_t(xf))
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    assert np.all(ga == 0.0) and np.all(gb[1] == 0.0)
    for r in range(4):
        assert np.array_equal(gb[0, xf[0, r] & 0x0F], g[0, r])


def test_intersect_empty_batch(dg):
    z = torch.zeros((0, 4, 2), device="cuda")
    xy, nx, xf = dg.intersect(z, z)
    assert xy.shape == (0, 8, 2) and nx.shape == (0,)


def test_area_forward_backward(dg):
    _say("case: area c4 polygons 20000 + rectangles 1024")
    d = synth.c4_polygons(n=20000, seed=95)
    for xy, nv in ((d["a_xy"], d["a_nv"]), (synth.c1_pairs()["a_xy"], None)):
        n = len(xy)
        a = dg.area(dev_t(xy), dev_t(nv)).cpu().numpy()
        ref = oracle.areas(xy, nv)
        scale = np.abs(xy).reshape(n, -1).max(1)
        assert np.all(np.abs(a - ref) <= 16 * U * 2 * scale ** 2 * xy.shape[1]), np.abs(a - ref).max()
        g = np.random.default_rng(5).uniform(-1, 1, n).astype(np.float32)
        gx = dg.area_backward(dev_t(xy), dev_t(g), dev_t(nv)).cpu().numpy()
        rg = oracle.areas_grad(xy, g, nv)
        assert grad_rel_err(gx, rg).max() <= 1e-6


def test_autograd_area_of_intersection(dg):
    """Area(Intersect(a, b)) through torch autograd equals the intersection
    area, and its gradient is the oracle's chain (vertex gradient of the
    shoelace routed through the intersection)."""
    d = synth.c3_pairs(n=4096, seed=96)
    a = dev_t(d["a_xy"]).requires_grad_(True)
    b = dev_t(d["b_xy"]).requires_grad_(True)
    xy, nx, xf = dg.Intersect.apply(a, b)
    area = dg.Area.apply(xy, nx)
    # nx < 3 means an empty (or degenerate) intersection: its area is 0
    area.sum().backward()
    r_xy, r_nx, r_xf, _ = oracle.intersect_pairs(d["a_xy"], d["b_xy"])
    keep = oracle.filtered_mask(oracle.pair_margins(d["a_xy"], d["b_xy"]))
    ref_area = oracle.areas(r_xy.astype(np.float32), r_nx)
    got = area.detach().cpu().numpy()
    ok = keep & (r_nx >= 3)
    assert np.abs(got - ref_area)[ok].max() <= 1e-4
    gX = oracle.areas_grad(r_xy.astype(np.float32), np.ones(len(r_nx)), r_nx)
    r_ga, r_gb = oracle.intersect_pairs_grad(d["a_xy"], d["b_xy"], gX, r_nx, r_xf)
    n = len(r_nx)
    gg = np.concatenate([a.grad.cpu().numpy().reshape(n, -1), b.grad.cpu().numpy().reshape(n, -1)], 1)
    rr = np.concatenate([r_ga.reshape(n, -1), r_gb.reshape(n, -1)], 1)
    assert grad_rel_err(gg, rr)[ok].max() <= GRAD_TOL
