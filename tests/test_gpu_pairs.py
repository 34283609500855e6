"""GPU parity of the elementwise-pair path (forward + backward kernels through
the C ABI) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (GRAD_TOL, IOU_TOL, compare_pairs, conditioned_mask, dev_t,
                      grad_rel_err, run_pairs)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


def _say(msg):
    print(msg, flush=True)


def _thin_boxes(n, seed):
    """Thin rotated rectangles (widths 1e-3..1e-2, lengths 1..3) against a copy
    moved by up to 2e-3 and turned by about 0.05 rad: unions of 1e-3..1e-1
    against coordinates of about 1, so fp32 areas carry ~u F^2 / U of IoU
    error (above 1e-5 for most pairs without the fp64 rebuild)."""
    rng = np.random.default_rng(seed)
    w, l = rng.uniform(1e-3, 1e-2, n), rng.uniform(1, 3, n)
    cx, cy, yaw = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-np.pi, np.pi, n)
    a = synth.boxes_to_quads(cx, cy, w, l, yaw)
    b = synth.boxes_to_quads(cx + rng.uniform(-2e-3, 2e-3, n), cy + rng.uniform(-2e-3, 2e-3, n),
                             w * rng.uniform(0.5, 2, n), l, yaw + rng.normal(0, 0.05, n))
    return a, b


def _needles(n, seed):
    """Thin triangles (apex angles 1e-3..1e-1 rad, length 1..2) whose apex
    pokes 1e-4..1e-2 deep into a convex 3..8-gon: intersections of area
    ~1e-11..1e-5 against coordinates of about 1, the pairs whose fp32
    gradient carries ~u F / sqrt(I) of relative error."""
    rng = np.random.default_rng(seed)
    d = synth.c4_polygons(n=n, seed=seed)
    a, anv = d["a_xy"], d["a_nv"]
    b = np.zeros((n, 3, 2), np.float32)
    for i in range(n):
        k = int(anv[i])
        e = int(rng.integers(k))
        p0, p1 = a[i, e].astype(np.float64), a[i, (e + 1) % k].astype(np.float64)
        t = rng.uniform(0.2, 0.8)
        foot = p0 + t * (p1 - p0)
        out = np.array([p1[1] - p0[1], p0[0] - p1[0]])  # outward normal of a CCW edge
        out /= np.linalg.norm(out)
        ang = rng.uniform(-0.6, 0.6)                    # the needle's tilt off the normal
        dirn = np.array([out[0] * np.cos(ang) - out[1] * np.sin(ang),
                         out[0] * np.sin(ang) + out[1] * np.cos(ang)])
        apex = foot - dirn * rng.uniform(1e-4, 1e-2)
        length, half = rng.uniform(1, 2), 0.5 * rng.uniform(1e-3, 1e-1)
        side = np.array([-dirn[1], dirn[0]])
        base = apex + dirn * length
        b[i] = [apex, base - side * length * np.tan(half), base + side * length * np.tan(half)]
    return a, anv, b


def test_thin_rectangles(dg):
    """Thin polygons: every pair's IoU within 1e-5 (the areas are rebuilt in
    fp64 where F^2 / U is large), the gradient on every pair whose crossings
    meet at |sin| >= 1e-3."""
    _say("case: thin rectangles 65536 pairs")
    a, b = _thin_boxes(65536, seed=61)
    g = np.random.default_rng(62).uniform(-1, 1, len(a)).astype(np.float32)
    s = compare_pairs(dg, a, b, grad=g, require_filtered_frac=0.0)
    _say(str(s))


def test_tiny_intersections(dg):
    """Needle triangles poking into polygons: no sliver filter; the gradient
    of every pair (crossings at |sin| >= 1e-3) within 1e-3, tiny
    intersections taking the fp64 backward."""
    _say("case: needles 8192 pairs")
    a, anv, b = _needles(8192, seed=63)
    g = np.random.default_rng(64).uniform(-1, 1, len(a)).astype(np.float32)
    s = compare_pairs(dg, a, b, a_nv=anv, grad=g, require_filtered_frac=0.0)
    _say(str(s))


def test_rectangles_c1(dg):
    _say("case: c1 rectangles 1024 pairs")
    d = synth.c1_pairs()
    s = compare_pairs(dg, d["a_xy"], d["b_xy"], grad=d["grad"])
    _say(str(s))
    # the backward kernel, fed the oracle's state, matches on every pair
    assert s["max_grad_err_oracle_state_all"] <= GRAD_TOL


def test_rectangles_ragged_many_tiles(dg):
    n = 65536 * 2 + 77          # many workgroups and a ragged tail
    _say(f"case: c3 rectangles {n} pairs")
    d = synth.c3_pairs(n=n, seed=7)
    s = compare_pairs(dg, d["a_xy"], d["b_xy"], grad=d["grad"])
    _say(str(s))


def test_polygons_mixed_counts(dg):
    n = 40000 + 13
    _say(f"case: c4 polygons {n} pairs")
    d = synth.c4_polygons(n=n, seed=8)
    s = compare_pairs(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], grad=d["grad"])
    _say(str(s))


def test_polygons_padding_is_ignored(dg):
    """Slots past a polygon's count may hold anything (NaN here)."""
    d = synth.c4_polygons(n=5000, seed=9)
    a, b = d["a_xy"].copy(), d["b_xy"].copy()
    for xy, nv in ((a, d["a_nv"]), (b, d["b_nv"])):
        mask = np.arange(8)[None, :] >= nv[:, None]
        xy[mask] = np.nan
    r1 = run_pairs(dg, a, b, d["a_nv"], d["b_nv"], grad=d["grad"])
    r0 = run_pairs(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], grad=d["grad"])
    assert np.array_equal(r1["iou"], r0["iou"])
    assert np.array_equal(r1["xflags"], r0["xflags"])
    assert np.array_equal(r1["ga"], r0["ga"]) and np.array_equal(r1["gb"], r0["gb"])
    mask = np.arange(8)[None, :] >= d["a_nv"][:, None]
    assert not r1["ga"][mask].any()


@pytest.mark.parametrize("k", [3, 5, 6, 7])
def test_polygon_capacities(dg, k):
    """kmax other than 4 / 8: unaligned rows, scalar loads, byte-wise flags."""
    d = synth.c4_polygons(n=3001, seed=20 + k)
    nv_a = np.minimum(d["a_nv"], k).astype(np.uint8)
    nv_b = np.minimum(d["b_nv"], k).astype(np.uint8)
    # polygons with fewer vertices: re-draw so that the first nv points are a polygon
    rng = np.random.default_rng(k)
    a, nva = synth.workloads.random_convex(rng, 3001, kmin=3, kmax=k)
    b, nvb = synth.workloads.random_convex(rng, 3001, kmin=3, kmax=k)
    s = compare_pairs(dg, a, b, nva, nvb, grad=d["grad"])
    _say(f"kmax={k}: {s}")


def test_triangles_without_counts(dg):
    rng = np.random.default_rng(31)
    a, _ = synth.workloads.random_convex(rng, 4000, kmin=3, kmax=3)
    b, _ = synth.workloads.random_convex(rng, 4000, kmin=3, kmax=3)
    g = rng.uniform(-1, 1, 4000).astype(np.float32)
    compare_pairs(dg, a, b, grad=g)


def test_3d_pairs(dg):
    d = synth.c1_pairs(n=20000, seed=41)
    rng = np.random.default_rng(42)
    z = rng.uniform(-2, 1, (20000, 2))
    h = rng.uniform(1.4, 1.8, (20000, 2))
    az = ((z[:, 0] - h[:, 0] / 2).astype(np.float32), (z[:, 0] + h[:, 0] / 2).astype(np.float32))
    bz = ((z[:, 1] - h[:, 1] / 2).astype(np.float32), (z[:, 1] + h[:, 1] / 2).astype(np.float32))
    s = compare_pairs(dg, d["a_xy"], d["b_xy"], a_z=az, b_z=bz, grad=d["grad"])
    _say(str(s))


def test_zero_height_boxes(dg):
    """Reading R5 on the GPU: flat 3D boxes (zlo == zhi) that overlap in BEV
    have a union volume of zero, so their IoU is exactly 0 and their gradient
    all zero, as in the oracle (no NaN from 0 / 0).  In a self-pair matrix of
    flat boxes every element off the diagonal is 0 (the diagonal keeps R15's
    exact 1) and the gradient is zero."""
    d = synth.c1_pairs(n=4096, seed=61)
    a, b = d["a_xy"], d["b_xy"]
    z = np.random.default_rng(62).uniform(-2, 1, 4096).astype(np.float32)
    zz = (z, z)
    tz = (dev_t(z), dev_t(z))
    iou, nx, xf = dg.iou_pairs(dev_t(a), dev_t(b), a_z=tz, b_z=tz)
    ref, rnx, _, _ = oracle.iou_pairs(a, b, a_z=zz, b_z=zz, threads=8)
    assert (ref == 0.0).all()
    assert (iou.cpu().numpy() == 0.0).all()
    assert int((rnx > 0).sum()) > 1000  # many pairs reach the zero-union branch
    g = torch.ones(4096, device="cuda")
    ga, gb, gaz, gbz = dg.iou_pairs_backward(dev_t(a), dev_t(b), g, nx, xf, a_z=tz, b_z=tz)
    for t in (ga, gb, gaz, gbz):
        assert torch.isfinite(t).all() and not t.any()
    off = np.array([0, 700, 701, 2048], np.int64)
    xy = a[:2048]
    mz = (dev_t(z[:2048]), dev_t(z[:2048]))
    out, saved, seg = dg.iou_matrix(dev_t(xy), a_z=mz, a_off=off, self_pairs=True, save=True)
    dg.check_errors()
    flat = out.cpu().numpy()
    diag = np.zeros(flat.shape[0], bool)
    o = 0
    for s in range(len(off) - 1):
        n = int(off[s + 1] - off[s])
        diag[o + np.arange(n) * (n + 1)] = True
        o += n * n
    assert (flat[diag] == 1.0).all() and (flat[~diag] == 0.0).all()
    gm = torch.ones(flat.shape[0], device="cuda")
    ga, _, gaz, _ = dg.iou_matrix_backward(gm, saved, seg, dev_t(xy), a_z=mz, self_pairs=True)
    assert not ga.any() and not gaz.any()


def test_degenerate_stress(dg):
    """Exactly degenerate contacts: the fp64 fallback and the tie rule give the
    oracle's vertex count, flag sequence (the boundary order of the moved
    pair, also where points coincide), IoU and one-sided gradient."""
    a, b, names = synth.degenerate_stress()
    g = np.ones(len(names), np.float32)
    gpu = run_pairs(dg, a, b, grad=g)
    ref, nx, xf, _ = oracle.iou_pairs(a, b)
    d = np.abs(gpu["iou"] - ref)
    assert d.max() <= IOU_TOL, [(names[i], gpu["iou"][i], ref[i]) for i in np.argsort(-d)[:3]]
    assert np.array_equal(gpu["nx"], nx), [(names[i], gpu["nx"][i], nx[i]) for i in range(len(nx))]
    same = np.all(gpu["xflags"] == xf, axis=1)
    assert same.all(), [(names[i], gpu["xflags"][i], xf[i]) for i in np.nonzero(~same)[0]]
    # the one-sided gradient of the tie rule's structure (exact dyadic vertices)
    ga, gb, _, _ = oracle.iou_pairs_grad(a, b, g, nx, xf)
    err = grad_rel_err(np.concatenate([gpu["ga"].reshape(len(a), -1),
                                       gpu["gb"].reshape(len(a), -1)], 1),
                       np.concatenate([ga.reshape(len(a), -1), gb.reshape(len(a), -1)], 1))
    assert err.max() <= GRAD_TOL, [(names[i], err[i]) for i in np.argsort(-err)[:3]]
    # swapped roles and translated copies (exact: dyadic shifts)
    for shift in (0.0, 1024.0, -3.5):
        gpu2 = run_pairs(dg, b + np.float32(shift), a + np.float32(shift))
        assert np.abs(gpu2["iou"] - ref).max() <= IOU_TOL


def test_near_degenerate_fallback(dg):
    """Pairs within fp32 rounding of a vertex/edge contact: signs are decided in
    fp64, so nx and the flag sequence match the oracle exactly."""
    d = synth.c1_pairs(n=4096, seed=51)
    a = d["a_xy"].copy()
    b = d["b_xy"].copy()
    # move a vertex of b onto (or within one ulp of) an edge of a
    t = np.float32(0.37)
    p = a[:, 0] + t * (a[:, 1] - a[:, 0])
    b[:, 2] = p.astype(np.float32)
    b[1::2, 2] = np.nextafter(b[1::2, 2], np.float32(np.inf))
    valid = np.array([oracle.polygon_valid(b[i].astype(np.float64)) for i in range(len(b))])
    a, b = a[valid], b[valid]
    gpu = run_pairs(dg, a, b)
    ref, nx, xf, _ = oracle.iou_pairs(a, b)
    assert np.abs(gpu["iou"] - ref).max() <= IOU_TOL
    assert np.array_equal(gpu["nx"], nx)
    assert np.array_equal(gpu["xflags"], xf)


def test_grid_contacts(dg):
    """Integer rectangles and diamonds on a small grid: shared and collinear
    edges, vertices on edges and corner touches on most pairs; count and flag
    sequence equal the oracle's on every pair, IoU on every pair."""
    rng = np.random.default_rng(2200)
    shapes = []
    for _ in range(40000):
        x0, y0 = rng.integers(-3, 3, 2)
        w, h = rng.integers(1, 4, 2)
        if rng.integers(0, 2):
            v = [(x0, y0), (x0 + w, y0), (x0 + w, y0 + h), (x0, y0 + h)]
        else:
            v = [(x0 + w, y0), (x0, y0 + w), (x0 - w, y0), (x0, y0 - w)]
        shapes.append(v)
    a = np.array(shapes[:20000], np.float32)
    b = np.array(shapes[20000:], np.float32)
    _say("case: grid contacts 20000")
    g = rng.uniform(-1, 1, 20000).astype(np.float32)
    _say(str(compare_pairs(dg, a, b, grad=g, require_filtered_frac=0.0)))


@pytest.mark.parametrize("sigma", [1e-6, 1e-7])
def test_near_identical_boxes(dg, sigma):
    """b within about an ulp of a: nearly parallel edges that share ends, and
    a filtered set that is nearly empty; IoU, count and flag sequence on every
    pair."""
    d = synth.c1_pairs(n=65536, seed=5000, center_sigma=sigma, yaw_sigma=sigma)
    _say(f"case: near-identical boxes sigma {sigma}")
    s = compare_pairs(dg, d["a_xy"], d["b_xy"], grad=d["grad"], require_filtered_frac=0.0)
    _say(str(s))


@pytest.mark.parametrize("shift,scale", [((1.0e4, -3.0e4), 1.0), ((0.0, 0.0), 2.0 ** -10),
                                         ((0.0, 0.0), 2.0 ** 10), ((-5.0e3, 7.0e3), 2.0 ** -4)])
def test_precision_far_and_scaled(dg, shift, scale):
    """IoU is invariant to translation and scale; the kernels work in the
    frame of the first polygon's first vertex, where differences of nearby
    fp32 coordinates are exact, so pairs far from the origin or at other
    scales keep the 1e-5 IoU bound against the oracle on the same fp32
    inputs (power-of-two scales keep the shapes exact)."""
    d = synth.c1_pairs(n=8192, seed=73)
    off = np.array(shift, np.float64)
    a = (d["a_xy"].astype(np.float64) * scale + off).astype(np.float32)
    b = (d["b_xy"].astype(np.float64) * scale + off).astype(np.float32)
    _say(f"case: c1 pairs shifted {shift} scaled {scale}")
    _say(str(compare_pairs(dg, a, b, grad=d["grad"], require_filtered_frac=0.9)))


def test_empty_and_single(dg):
    e = np.zeros((0, 4, 2), np.float32)
    iou, nx, xf = dg.iou_pairs(dev_t(e), dev_t(e))
    assert iou.numel() == 0 and xf.shape == (0, 8)
    d = synth.c1_pairs(n=1, seed=3)
    compare_pairs(dg, d["a_xy"], d["b_xy"], grad=d["grad"], require_filtered_frac=0.0)


def test_full_size_rectangles_sampled(dg):
    """1,048,576 pairs in the benchmark's launch configuration; sampled pairs
    against the oracle, every pair against invariants."""
    d = synth.c3_pairs()
    n = len(d["a_xy"])
    _say(f"case: c3 full {n} pairs")
    gpu = run_pairs(dg, d["a_xy"], d["b_xy"], grad=d["grad"])
    idx = np.random.default_rng(0).choice(n, 60000, replace=False)
    idx = np.concatenate([idx, np.arange(n - 100, n)])
    sub = {k: d[k][idx] for k in ("a_xy", "b_xy", "grad")}
    ref, nx, xf, _ = oracle.iou_pairs(sub["a_xy"], sub["b_xy"], threads=8)
    keep = conditioned_mask(oracle.pair_margins(sub["a_xy"], sub["b_xy"], threads=8))
    assert np.abs(gpu["iou"][idx] - ref).max() <= IOU_TOL
    assert np.array_equal(gpu["nx"][idx], nx)
    assert np.array_equal(gpu["xflags"][idx], xf)
    ga, gb, _, _ = oracle.iou_pairs_grad(sub["a_xy"], sub["b_xy"], sub["grad"], nx, xf, threads=8)
    err = grad_rel_err(np.concatenate([gpu["ga"][idx].reshape(len(idx), -1),
                                       gpu["gb"][idx].reshape(len(idx), -1)], 1),
                       np.concatenate([ga.reshape(len(idx), -1), gb.reshape(len(idx), -1)], 1))
    assert err[keep].max() <= GRAD_TOL
    # every pair: IoU in [0, 1], nx in {0} u [3, 8], translation invariance of the gradient
    assert gpu["iou"].min() >= 0 and gpu["iou"].max() <= 1 + 1e-6
    assert np.all((gpu["nx"] == 0) | ((gpu["nx"] >= 3) & (gpu["nx"] <= 8)))
    tot = gpu["ga"].sum(1) + gpu["gb"].sum(1)
    scale = np.abs(gpu["ga"]).sum((1, 2)) + np.abs(gpu["gb"]).sum((1, 2)) + 1e-30
    assert np.max(np.abs(tot).max(1) / scale) <= 1e-4


def test_full_size_polygons_sampled(dg):
    d = synth.c4_polygons()
    n = len(d["a_xy"])
    _say(f"case: c4 full {n} pairs")
    gpu = run_pairs(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], grad=d["grad"])
    idx = np.random.default_rng(1).choice(n, 30000, replace=False)
    sub = {k: d[k][idx] for k in ("a_xy", "b_xy", "grad", "a_nv", "b_nv")}
    ref, nx, xf, _ = oracle.iou_pairs(sub["a_xy"], sub["b_xy"], sub["a_nv"], sub["b_nv"], threads=8)
    assert np.abs(gpu["iou"][idx] - ref).max() <= IOU_TOL
    assert np.array_equal(gpu["nx"][idx], nx)
    assert np.array_equal(gpu["xflags"][idx], xf)


def test_deterministic(dg):
    d = synth.c4_polygons(n=20000, seed=61)
    r1 = run_pairs(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], grad=d["grad"])
    r2 = run_pairs(dg, d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], grad=d["grad"])
    for k in ("iou", "nx", "xflags", "ga", "gb"):
        assert np.array_equal(r1[k], r2[k]), k


def test_autograd_function(dg):
    d = synth.c1_pairs(n=2048, seed=71)
    a = dev_t(d["a_xy"]).requires_grad_(True)
    b = dev_t(d["b_xy"]).requires_grad_(True)
    iou = dg.IoUPairs.apply(a, b)
    (iou * dev_t(d["grad"])).sum().backward()
    ref, nx, xf, _ = oracle.iou_pairs(d["a_xy"], d["b_xy"])
    ga, gb, _, _ = oracle.iou_pairs_grad(d["a_xy"], d["b_xy"], d["grad"], nx, xf)
    keep = conditioned_mask(oracle.pair_margins(d["a_xy"], d["b_xy"]))
    err = grad_rel_err(np.concatenate([a.grad.cpu().numpy().reshape(2048, -1),
                                       b.grad.cpu().numpy().reshape(2048, -1)], 1),
                       np.concatenate([ga.reshape(2048, -1), gb.reshape(2048, -1)], 1))
    assert err[keep].max() <= GRAD_TOL


def test_autograd_vs_central_differences(dg):
    """The differentiation form on 4,096 pairs of the 1 Mi rectangle workload's
    distribution: torch.autograd through the library's backward against
    central differences of the FP64 IoU at h = 1e-3 (Richardson on h and h/2,
    which removes the h^2 term), on pairs whose nx / xflags stay the same at
    every perturbed point (the IoU is smooth there)."""
    d = synth.c3_pairs(n=4096, seed=72)
    a32, b32, g32 = d["a_xy"], d["b_xy"], d["grad"]
    a = dev_t(a32).requires_grad_(True)
    b = dev_t(b32).requires_grad_(True)
    iou = dg.IoUPairs.apply(a, b)
    (iou * dev_t(g32)).sum().backward()
    gpu = np.concatenate([a.grad.cpu().numpy().reshape(4096, -1),
                          b.grad.cpu().numpy().reshape(4096, -1)], 1).astype(np.float64)
    a64, b64 = a32.astype(np.float64), b32.astype(np.float64)
    _, nx0, xf0 = oracle.iou_pairs_f64(a64, b64)
    stable = np.ones(4096, bool)
    fd = np.zeros((4096, 16))
    for c in range(16):
        poly, k, ax = c // 8, (c % 8) // 2, c % 2

        def at(step):
            aa, bb = a64.copy(), b64.copy()
            (aa if poly == 0 else bb)[:, k, ax] += step
            v, nx, xf = oracle.iou_pairs_f64(aa, bb)
            stable[:] &= (nx == nx0) & np.all(xf == xf0, axis=1)
            return v

        h = 1e-3
        d1 = (at(h) - at(-h)) / (2 * h)
        d2 = (at(h / 2) - at(-h / 2)) / h
        fd[:, c] = g32 * (4 * d2 - d1) / 3
    assert stable.mean() > 0.9
    err = grad_rel_err(gpu, fd)
    assert err[stable].max() <= GRAD_TOL, err[stable].max()
    _say(str({"pairs_smooth_at_h": int(stable.sum()), "max_grad_err_vs_fd": float(err[stable].max())}))


def test_invalid_arguments(dg):
    ctx = dg.context()
    ok = dg.Polys(0, None, None, None, 1, 4)  # pointer checked only when used
    a = dev_t(np.zeros((2, 4, 2), np.float32))
    pa, _ = dg.polys(a)
    bad_k = dg.Polys(pa.xy, None, None, None, 2, 9)
    out = torch.empty(2, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert dg.lib.dgal_iou_pairs(ctx, pa, bad_k, out.data_ptr(), None, None, s) == dg.DGAL_EINVAL
    pb = dg.Polys(pa.xy, None, None, None, 3, 4)          # count mismatch
    assert dg.lib.dgal_iou_pairs(ctx, pa, pb, out.data_ptr(), None, None, s) == dg.DGAL_EINVAL
    mis = dg.Polys(pa.xy + 4, None, None, None, 1, 4)     # 4-byte aligned only
    assert dg.lib.dgal_iou_pairs(ctx, mis, mis, out.data_ptr(), None, None, s) == dg.DGAL_EINVAL
    nx = torch.empty(2, dtype=torch.uint8, device="cuda")
    assert dg.lib.dgal_iou_pairs(ctx, pa, pa, out.data_ptr(), nx.data_ptr(), None, s) == dg.DGAL_EINVAL
    zonly = dg.Polys(pa.xy, None, out.data_ptr(), None, 2, 4)
    assert dg.lib.dgal_iou_pairs(ctx, zonly, zonly, out.data_ptr(), None, None, s) == dg.DGAL_EINVAL
    assert dg.lib.dgal_iou_backward(ctx, 5, pa, pa, None, None, None, 0, 0, out.data_ptr(), 0,
                                    None, None, None, None, None, None, None, s) == dg.DGAL_EINVAL
    del ok
    dg.check_errors()


def test_graph_replay_matches_eager(dg):
    """Elementwise forward + backward of the corner form, the box-parameter
    form and simple polygons captured in one HIP graph (via torch), replayed
    several times with eager work in between; every replay equals eager."""
    c = synth.c3_pairs(n=20000, seed=61)
    bx = synth.c3_boxes(n=20000, seed=62)
    sp = synth.c4_simple(n=8192, seed=63)
    ta, tb, tg = dev_t(c["a_xy"]), dev_t(c["b_xy"]), dev_t(c["grad"])
    ba, bb, bg = dev_t(bx["a_box"]), dev_t(bx["b_box"]), dev_t(bx["grad"])
    sa, sb, san, sbn = dev_t(sp["a_xy"]), dev_t(sp["b_xy"]), dev_t(sp["a_nv"]), dev_t(sp["b_nv"])
    sg = dev_t(sp["grad"])

    def step():
        iou, nx, xf = dg.iou_pairs(ta, tb)
        ga, gb, _, _ = dg.iou_pairs_backward(ta, tb, tg, nx, xf)
        biou, bnx, bxf = dg.iou_boxes(ba, bb)
        bga, bgb = dg.iou_boxes_backward(ba, bb, bg, bnx, bxf)
        siou, xm, sm, ins = dg.iou_simple_pairs(sa, sb, san, sbn)
        sga, sgb = dg.iou_simple_backward(sa, sb, sg, xm, sm, ins, san, sbn)
        return (iou, nx, xf, ga, gb, biou, bga, bgb, siou, xm, sga, sgb)

    eager = step()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):  # warm up on the side stream (and settle any tuning)
            step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = step()
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        for k, (g_, e_) in enumerate(zip(out, eager)):
            assert torch.equal(g_, e_), (rep, k)
        del junk
    dg.check_errors()


def test_pairs_beyond_int32_elements(dg):
    """2^28 + 1000 rectangle pairs (element offsets of the [n, 4, 2] inputs
    and gradients past 2^31; ~39 GB of device memory), built on the device;
    sampled pairs across the whole range against the oracle: IoU, count and
    codes, gradients on the non-degenerate ones."""
    n = (1 << 28) + 1000
    gen = torch.Generator("cuda").manual_seed(71)

    def quads(cx, cy, w, l, yaw):
        c, s_ = torch.cos(yaw), torch.sin(yaw)
        ux, uy = 0.5 * w * c, 0.5 * w * s_
        vx, vy = -0.5 * l * s_, 0.5 * l * c
        xs = torch.stack([cx - ux - vx, cx + ux - vx, cx + ux + vx, cx - ux + vx], 1)
        ys = torch.stack([cy - uy - vy, cy + uy - vy, cy + uy + vy, cy - uy + vy], 1)
        return torch.stack([xs, ys], 2).contiguous()

    def u(lo, hi):
        return torch.rand(n, device="cuda", generator=gen) * (hi - lo) + lo

    cx, cy, w, l, yaw = u(-2, 2), u(-2, 2), u(1, 3), u(1, 3), u(-3.14, 3.14)
    a = quads(cx, cy, w, l, yaw)
    b = quads(cx + u(-0.5, 0.5), cy + u(-0.5, 0.5), w + u(-0.1, 0.1), l + u(-0.1, 0.1),
              yaw + u(-0.2, 0.2))
    del cx, cy, w, l, yaw
    g = u(-1, 1)
    _say(f"case: {n} rectangle pairs")
    iou, nx, xf = dg.iou_pairs(a, b)
    ga, gb, _, _ = dg.iou_pairs_backward(a, b, g, nx, xf)
    dg.check_errors()
    rng = np.random.default_rng(72)
    idx = np.concatenate([rng.integers(0, n, 30000), np.arange(n - 1000, n)])
    ti = torch.from_numpy(idx).cuda()
    sa, sb, sg = a[ti].cpu().numpy(), b[ti].cpu().numpy(), g[ti].cpu().numpy()
    ref, r_nx, r_xf, bad = oracle.iou_pairs(sa, sb, threads=16)
    assert bad == 0
    assert np.abs(iou[ti].cpu().numpy() - ref).max() <= IOU_TOL
    assert np.array_equal(nx[ti].cpu().numpy(), r_nx)
    assert np.array_equal(xf[ti].cpu().numpy(), r_xf)
    keep = conditioned_mask(oracle.pair_margins(sa, sb, threads=16))
    r_ga, r_gb = oracle.iou_pairs_grad(sa, sb, sg, r_nx, r_xf, threads=16)[:2]
    err = grad_rel_err(np.concatenate([ga[ti].cpu().numpy().reshape(len(idx), -1),
                                       gb[ti].cpu().numpy().reshape(len(idx), -1)], 1),
                       np.concatenate([r_ga.reshape(len(idx), -1), r_gb.reshape(len(idx), -1)], 1))
    assert keep.mean() > 0.9 and err[keep].max() <= GRAD_TOL



def test_path_stats_count_the_fp64_path(dg):
    """The device path statistics: every evaluated pair is counted once;
    pairs with a vertex of b on (or an ulp off) an edge of a take the fp64
    signs (fp32 cannot certify a near-zero orientation), generic pairs
    rarely; the matrix's exact pass counts its saved survivors."""
    d = synth.c1_pairs(n=4096, seed=51)
    a, b = d["a_xy"].copy(), d["b_xy"].copy()
    t = np.float32(0.37)
    b[:, 2] = (a[:, 0] + t * (a[:, 1] - a[:, 0])).astype(np.float32)
    b[1::2, 2] = np.nextafter(b[1::2, 2], np.float32(np.inf))
    valid = np.array([oracle.polygon_valid(b[i].astype(np.float64)) for i in range(len(b))])
    a, b = a[valid], b[valid]
    dg.set_path_stats(True)
    try:
        assert dg.path_stats() == (0, 0, 0)
        dg.iou_pairs(dev_t(a), dev_t(b))
        n, k, t = dg.path_stats()
        assert n == len(a) and k >= 0.9 * n and t == 0, (n, k, t)
        g = synth.c3_pairs(n=65536, seed=52)
        dg.iou_pairs(dev_t(g["a_xy"]), dev_t(g["b_xy"]))
        n, k, t = dg.path_stats()
        assert n == 65536 and k <= 0.05 * n and t == 0, (n, k, t)
        m = synth.c2_matrix(n=300, m=257, seed=3)
        _, saved, _ = dg.iou_matrix(dev_t(m["a_xy"]), dev_t(m["b_xy"]), save=True)
        n, k, t = dg.path_stats()
        assert n == int(saved.count.item()) and 0 <= k <= n and t == 0, (n, k, t)
        _say(f"path stats: matrix {n} survivors, {k} with fp64 signs")
        # thin rectangles: every overlapping pair rebuilds its areas
        ta, tb = _thin_boxes(2048, seed=53)
        iou, nx, _ = dg.iou_pairs(dev_t(ta), dev_t(tb))
        n, k, t = dg.path_stats()
        assert n == 2048 and t == int((nx.cpu().numpy() >= 3).sum()), (n, t)
    finally:
        dg.set_path_stats(False)
    dg.iou_pairs(dev_t(a), dev_t(b))
    assert dg.path_stats() == (0, 0, 0)
