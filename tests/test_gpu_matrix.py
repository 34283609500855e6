"""GPU parity of the IoU-matrix path (LDS tiles, cull, survivor compaction,
persistent segment schedule, saved non-empty pairs, a backward that sums rows
without atomics and adds a second set's columns with global atomics) and of
per-scene 3D self-pairs, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import GRAD_TOL, IOU_TOL, dev_t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available()
    return d


def _say(msg):
    print(msg, flush=True)


def _crowd(xy, factor):
    """Moves box centres towards the origin (boxes keep their shape)."""
    c = xy.astype(np.float64).mean(1, keepdims=True)
    return (xy - c + factor * c).astype(np.float32)


def _saved_entries(saved):
    """(pair_id, nx) of the work-list entries, tile by tile, and the table."""
    nt = saved.tiles_used
    st = saved.tile_start[:nt].cpu().numpy()
    sc = saved.tile_count[:nt].cpu().numpy()
    pid_all = saved.pair_id.cpu().numpy()
    nx_all = saved.nx.cpu().numpy()
    idx = np.concatenate([np.arange(a, a + c) for a, c in zip(st, sc)]) if nt else np.zeros(0, int)
    return pid_all[idx], nx_all[idx], st, sc


def _aabb_candidates(a, b, a_off=None, b_off=None, self_pairs=False):
    """Index pairs whose axis-aligned bounding boxes overlap (every other pair
    is disjoint, so its IoU is exactly 0).  Returns (ia, ib, flat index)."""
    lo_a, hi_a = a.min(1), a.max(1)
    lo_b, hi_b = b.min(1), b.max(1)
    segs = [(0, len(a), 0, len(b), 0)] if a_off is None else []
    if a_off is not None:
        out = 0
        for s in range(len(a_off) - 1):
            segs.append((a_off[s], a_off[s + 1], b_off[s], b_off[s + 1], out))
            out += (a_off[s + 1] - a_off[s]) * (b_off[s + 1] - b_off[s])
    IA, IB, FL = [], [], []
    for a0, a1, b0, b1, o in segs:
        nb = b1 - b0
        for r0 in range(a0, a1, 512):
            r1 = min(a1, r0 + 512)
            ov = ((lo_a[r0:r1, None, 0] <= hi_b[None, b0:b1, 0]) &
                  (lo_b[None, b0:b1, 0] <= hi_a[r0:r1, None, 0]) &
                  (lo_a[r0:r1, None, 1] <= hi_b[None, b0:b1, 1]) &
                  (lo_b[None, b0:b1, 1] <= hi_a[r0:r1, None, 1]))
            r, c = np.nonzero(ov)
            IA.append(r + r0)
            IB.append(c + b0)
            FL.append(o + (r + r0 - a0) * nb + c)
    return np.concatenate(IA), np.concatenate(IB), np.concatenate(FL)


def _check_matrix_exact(iou_flat, a, b, a_z=None, b_z=None, a_off=None, b_off=None,
                        self_pairs=False):
    ia, ib, fl = _aabb_candidates(a, b, a_off, b_off, self_pairs)
    ref, nx, xf = oracle.iou_index_pairs(ia, ib, a, b, a_z=a_z, b_z=b_z, threads=8)
    if self_pairs:
        ref = np.where(ia == ib, 1.0, ref)
    d = np.abs(iou_flat[fl].astype(np.float64) - ref)
    assert d.max() <= IOU_TOL, (d.max(), ia[d.argmax()], ib[d.argmax()])
    outside = np.ones(iou_flat.shape[0], bool)
    outside[fl] = False
    assert not iou_flat[outside].any(), "non-zero IoU for a pair with disjoint AABBs"
    return ia, ib, fl, ref, nx, xf


def _grad_reference(a, b, g, ia, ib, fl, a_nv=None, b_nv=None, a_z=None, b_z=None,
                    self_pairs=False):
    """Reference of the matrix backward from the oracle's per-pair gradients
    over the entries (ia[t], ib[t]) at flat index fl[t] (a superset of the
    non-empty pairs: every other entry has zero gradient).  Returns, per box
    of a and of b (one set when self_pairs), the summed gradient [n, 2K (+2)]
    (xy, then d/dzlo, d/dzhi) and its scale: the sum over the box's pairs of
    the norm of that pair's term.  An fp32 sum of terms that each carry a
    relative error e is within e times that scale, whatever their
    cancellation.  Self pairs: entry (r, c) is the pair with the lower index
    first, and the diagonal is constant."""
    if self_pairs:
        keep = ia != ib
        ia, ib, fl = ia[keep], ib[keep], fl[keep]
        ia, ib = np.minimum(ia, ib), np.maximum(ia, ib)
        b, b_nv, b_z = a, a_nv, a_z
    sub = lambda v, i: None if v is None else v[i]
    subz = lambda z, i: None if z is None else (z[0][i], z[1][i])
    _, nx, xf = oracle.iou_index_pairs(ia, ib, a, b, a_nv, b_nv, a_z=a_z, b_z=b_z, threads=8)
    gp, gq, gzp, gzq = oracle.iou_pairs_grad(a[ia], b[ib], g[fl], nx, xf, sub(a_nv, ia),
                                             sub(b_nv, ib), subz(a_z, ia), subz(b_z, ib),
                                             threads=8)
    tp, tq = gp.reshape(len(ia), -1), gq.reshape(len(ib), -1)
    if a_z is not None:
        tp, tq = np.concatenate([tp, gzp], 1), np.concatenate([tq, gzq], 1)
    out = []
    sets = [(len(a), ia, tp, ib, tq)] if self_pairs else [(len(a), ia, tp, None, None),
                                                          (len(b), ib, tq, None, None)]
    for n, i1, t1, i2, t2 in sets:
        ref = np.zeros((n, t1.shape[1]))
        scale = np.zeros(n)
        np.add.at(ref, i1, t1)
        np.add.at(scale, i1, np.linalg.norm(t1, axis=1))
        if i2 is not None:
            np.add.at(ref, i2, t2)
            np.add.at(scale, i2, np.linalg.norm(t2, axis=1))
        out += [ref, scale]
    return out


def _box_grads(ga, gaz=None):
    n = ga.shape[0]
    parts = [ga.cpu().numpy().reshape(n, -1)]
    if gaz is not None:
        parts.append(gaz.cpu().numpy())
    return np.concatenate(parts, 1)


def _assert_box_grads(got, ref, scale, what):
    """Every box: |g - g_ref| <= GRAD_TOL x (sum of its pair terms' norms);
    a box with no contributing pair must be exactly zero."""
    err = np.linalg.norm(got - ref, axis=1)
    rel = err / np.maximum(scale, 1e-30)
    k = int(np.argmax(rel))
    assert rel[k] <= GRAD_TOL, (what, float(rel[k]), k, float(err[k]), float(scale[k]))
    return float(rel.max())


def test_matrix_small_dense_overlap(dg):
    d = synth.c2_matrix(n=300, m=257, seed=3)
    a, b = _crowd(d["a_xy"], 0.1), _crowd(d["b_xy"], 0.1)
    iou, saved, seg = dg.iou_matrix(dev_t(a), dev_t(b), save=True)
    dg.check_errors()
    got = iou.cpu().numpy()
    ref, _ = oracle.iou_matrix(a, b)
    ref = ref.reshape(300, 257)
    assert np.abs(got - ref).max() <= IOU_TOL
    # work list: every cull survivor once, with the oracle's vertex counts; the
    # entries with nx > 0 are exactly the pairs with a non-empty intersection;
    # tile t covers rows R (t // ct) .. +R-1 and columns C (t % ct) .. +C-1 (R
    # rows and C = 2048 / R columns per tile, the shape the forward used)
    pid, snx, st, sc = _saved_entries(saved)
    cnt = int((snx > 0).sum())
    assert len(np.unique(pid)) == len(pid) == int(saved.count.item())
    r, c = np.meshgrid(np.arange(300), np.arange(257), indexing="ij")
    _, nx_all, xf_all = oracle.iou_index_pairs(r.ravel(), c.ravel(), a, b, threads=8)
    assert np.array_equal(np.sort(pid[snx > 0]), np.nonzero(nx_all > 0)[0])
    assert np.array_equal(snx, nx_all[pid])
    # and on every entry the oracle's flag sequence
    ent = np.concatenate([np.arange(a0, a0 + c0) for a0, c0 in zip(st, sc)])
    sxf = saved.xflags.cpu().numpy()[ent]
    assert np.array_equal(sxf, xf_all[pid])
    R = saved.tile_rows
    C = dg.TILE_PAIRS // R
    ct = (257 + C - 1) // C
    assert saved.tiles_used == ((300 + R - 1) // R) * ct
    for t in range(saved.tiles_used):
        ent = saved.pair_id[st[t]:st[t] + sc[t]].cpu().numpy()
        rows, cols = ent // 257, ent % 257
        assert np.all((rows >= R * (t // ct)) & (rows < R * (t // ct) + R))
        assert np.all((cols >= C * (t % ct)) & (cols < C * (t % ct) + C))
    _say(f"small matrix: {cnt} non-empty of {300 * 257}")


def test_matrix_backward_small(dg):
    d = synth.c2_matrix(n=200, m=150, seed=4)
    a, b = _crowd(d["a_xy"], 0.08), _crowd(d["b_xy"], 0.08)
    g = np.random.default_rng(5).uniform(-1, 1, (200, 150)).astype(np.float32)
    iou, saved, seg = dg.iou_matrix(dev_t(a), dev_t(b), save=True)
    ga, gb, _, _ = dg.iou_matrix_backward(dev_t(g).reshape(-1), saved, seg, dev_t(a), dev_t(b))
    ia, ib, fl = _aabb_candidates(a, b)
    ra, sa, rb, sb = _grad_reference(a, b, g.reshape(-1), ia, ib, fl)
    # the per-pair reference is the oracle's matrix gradient
    om_a, om_b, _, _ = oracle.iou_matrix_grad(g.reshape(-1), a, b)
    assert np.abs(ra - om_a.reshape(len(a), -1)).max() <= 1e-12 * (1 + np.abs(om_a).max())
    assert np.abs(rb - om_b.reshape(len(b), -1)).max() <= 1e-12 * (1 + np.abs(om_b).max())
    ea = _assert_box_grads(_box_grads(ga), ra, sa, "rows")
    eb = _assert_box_grads(_box_grads(gb), rb, sb, "columns")
    _say(f"matrix backward small: max rel err rows {ea:.2e} columns {eb:.2e}")
    # autograd wrapper
    ta = dev_t(a).requires_grad_(True)
    tb = dev_t(b).requires_grad_(True)
    out = dg.IoUMatrix.apply(ta, tb)
    (out * dev_t(g)).sum().backward()
    assert torch.allclose(ta.grad, ga, atol=1e-5) and torch.allclose(tb.grad, gb, atol=1e-5)


def test_matrix_full_size_exact(dg):
    """4096 x 4096 BEV boxes (the benchmark shape), every pair checked: AABB-
    disjoint pairs must be 0, all others equal the oracle."""
    d = synth.c2_matrix()
    _say("case: c2 4096x4096")
    iou, saved, seg = dg.iou_matrix(dev_t(d["a_xy"]), dev_t(d["b_xy"]), save=True)
    dg.check_errors()
    flat = iou.cpu().numpy().reshape(-1)
    ia, ib, fl, ref, nx, xf = _check_matrix_exact(flat, d["a_xy"], d["b_xy"])
    cnt = int(saved.count.item())
    pid, snx, _, _ = _saved_entries(saved)
    assert cnt == len(fl)          # survivors are exactly the AABB-overlapping pairs
    assert np.array_equal(np.sort(pid[snx > 0]), np.sort(fl[nx > 0]))
    _say(f"c2: {len(fl)} AABB candidates, {cnt} survivors, {int((snx > 0).sum())} non-empty "
         f"({(snx > 0).sum() / flat.size:.4%})")


def test_matrix_ragged_tiles(dg):
    """Sizes that are not multiples of the tile, including a single row."""
    for n, m in ((1, 1), (1, 200), (65, 64), (130, 1), (129, 191)):
        d = synth.c2_matrix(n=n, m=m, seed=n * 1000 + m)
        a, b = _crowd(d["a_xy"], 0.05), _crowd(d["b_xy"], 0.05)
        iou, _, _ = dg.iou_matrix(dev_t(a), dev_t(b))
        ref, _ = oracle.iou_matrix(a, b)
        assert np.abs(iou.cpu().numpy().reshape(-1) - ref).max() <= IOU_TOL, (n, m)


def test_matrix_polygons(dg):
    d = synth.c4_polygons(n=300, seed=5)
    a, anv, b, bnv = d["a_xy"][:180], d["a_nv"][:180], d["b_xy"][:220], d["b_nv"][:220]
    iou, saved, seg = dg.iou_matrix(dev_t(a), dev_t(b), dev_t(anv), dev_t(bnv), save=True)
    ref, _ = oracle.iou_matrix(a, b, anv, bnv)
    assert np.abs(iou.cpu().numpy().reshape(-1) - ref).max() <= IOU_TOL
    g = np.random.default_rng(6).uniform(-1, 1, 180 * 220).astype(np.float32)
    ga, gb, _, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(a), dev_t(b), dev_t(anv),
                                          dev_t(bnv))
    ia, ib, fl = _aabb_candidates(a, b)
    ra, sa, rb, sb = _grad_reference(a, b, g, ia, ib, fl, anv, bnv)
    om_a, om_b, _, _ = oracle.iou_matrix_grad(g, a, b, anv, bnv)
    assert np.abs(ra - om_a.reshape(len(a), -1)).max() <= 1e-12 * (1 + np.abs(om_a).max())
    _assert_box_grads(_box_grads(ga), ra, sa, "rows")
    _assert_box_grads(_box_grads(gb), rb, sb, "columns")


def _scenes(scenes, nmin, nmax, seed, crowd):
    d = synth.c5_scenes(scenes=scenes, nmin=nmin, nmax=nmax, seed=seed)
    xy = d["a_xy"]
    if crowd is not None:
        xy = _crowd(xy, crowd)
    return xy, d["a_zlo"], d["a_zhi"], d["off"], d["out_off"]


def test_scenes_small_forward_backward(dg):
    xy, lo, hi, off, out_off = _scenes(5, 10, 140, 7, 0.12)
    total = int(out_off[-1])
    g = np.random.default_rng(8).uniform(-1, 1, total).astype(np.float32)
    txy, tlo, thi = dev_t(xy), dev_t(lo), dev_t(hi)
    iou, saved, seg = dg.iou_matrix(txy, a_z=(tlo, thi), a_off=off, self_pairs=True, save=True)
    ref, ref_off = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    got = iou.cpu().numpy()
    assert np.array_equal(ref_off, out_off)
    assert np.abs(got - ref).max() <= IOU_TOL
    for s in range(5):
        n = off[s + 1] - off[s]
        blk = got[out_off[s]:out_off[s + 1]].reshape(n, n)
        assert np.all(np.diag(blk) == 1.0)
    ga, _, gaz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, txy, a_z=(tlo, thi),
                                           self_pairs=True)
    ia, ib, fl = _aabb_candidates(xy, xy, off, off, True)
    ref, scale = _grad_reference(xy, xy, g, ia, ib, fl, a_z=(lo, hi), b_z=(lo, hi),
                                 self_pairs=True)
    ref_a, _, ref_z, _ = oracle.iou_matrix_grad(g, xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    om = np.concatenate([ref_a.reshape(len(xy), -1), ref_z], 1)
    assert np.abs(ref - om).max() <= 1e-12 * (1 + np.abs(om).max())
    e = _assert_box_grads(_box_grads(ga, gaz), ref, scale, "scenes")
    _say(f"scenes small: {int(saved.count.item())} saved pairs, max rel err {e:.2e}")
    # every row sum is added in a fixed order: a second call gives the same bits
    ga2, _, gaz2, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, txy, a_z=(tlo, thi),
                                             self_pairs=True)
    assert torch.equal(ga2, ga) and torch.equal(gaz2, gaz)


@pytest.mark.parametrize("two_sets", [False, True])
def test_extruded_polygons_3d(dg, two_sets):
    """3D IoU of extruded convex 3..8-gons (counted vertices with z-extents:
    the 8-slot 3D kernels, whose backward sums nine value pairs per row, so
    a row group's 72 (row, pair) sums take a second round of lanes), as
    ragged per-scene self pairs (a one-box scene included) or ragged two-set
    segments: IoU on every pair and gradients against the oracle."""
    d = synth.c4_polygons(n=700, seed=15)
    rng = np.random.default_rng(19)
    xy, nv = d["a_xy"][:700], d["a_nv"][:700]
    lo = rng.uniform(-2.0, 1.0, 700).astype(np.float32)
    hi = (lo + rng.uniform(0.5, 2.0, 700)).astype(np.float32)
    if two_sets:
        a, anv, az = xy[:350], nv[:350], (lo[:350], hi[:350])
        b, bnv, bz = xy[350:], nv[350:], (lo[350:], hi[350:])
        a_off = np.array([0, 120, 120, 300, 350], np.int64)
        b_off = np.array([0, 60, 200, 201, 350], np.int64)
        _say(f"case: extruded polygons, two sets, segments {a_off.tolist()} / {b_off.tolist()}")
        iou, saved, seg = dg.iou_matrix(dev_t(a), dev_t(b), dev_t(anv), dev_t(bnv),
                                        (dev_t(az[0]), dev_t(az[1])),
                                        (dev_t(bz[0]), dev_t(bz[1])), a_off, b_off, save=True)
        ref, _ = oracle.iou_matrix(a, b, anv, bnv, az, bz, a_off, b_off)
    else:
        off = np.array([0, 150, 151, 400, 700], np.int64)
        _say(f"case: extruded polygons, self pairs, scenes {off.tolist()}")
        a, anv, az = xy, nv, (lo, hi)
        iou, saved, seg = dg.iou_matrix(dev_t(a), None, dev_t(anv), None,
                                        (dev_t(lo), dev_t(hi)), None, off, self_pairs=True,
                                        save=True)
        ref, _ = oracle.iou_matrix(a, a_nv=anv, a_z=az, a_off=off, self_pairs=True)
    dg.check_errors()
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    g = rng.uniform(-1, 1, ref.shape[0]).astype(np.float32)
    if two_sets:
        ga, gb, gaz, gbz = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(a), dev_t(b),
                                                  dev_t(anv), dev_t(bnv),
                                                  (dev_t(az[0]), dev_t(az[1])),
                                                  (dev_t(bz[0]), dev_t(bz[1])))
        ia, ib, fl = _aabb_candidates(a, b, a_off, b_off)
        ra, sa, rb, sb = _grad_reference(a, b, g, ia, ib, fl, anv, bnv, az, bz)
        _assert_box_grads(_box_grads(ga, gaz), ra, sa, "rows")
        e = _assert_box_grads(_box_grads(gb, gbz), rb, sb, "columns")
    else:
        ga, _, gaz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(a), None, dev_t(anv),
                                               None, (dev_t(lo), dev_t(hi)), None,
                                               self_pairs=True)
        ia, ib, fl = _aabb_candidates(a, a, off, off, True)
        rr, sc = _grad_reference(a, a, g, ia, ib, fl, anv, anv, az, az, self_pairs=True)
        e = _assert_box_grads(_box_grads(ga, gaz), rr, sc, "scenes")
    _say(f"extruded polygons ({'two sets' if two_sets else 'self pairs'}): "
         f"{int(saved.count.item())} saved pairs, max rel err {e:.2e}")


def test_scenes_with_empty_and_single_box_segments(dg):
    d = synth.c5_scenes(scenes=6, nmin=5, nmax=40, seed=9)
    xy, lo, hi = _crowd(d["a_xy"], 0.1), d["a_zlo"], d["a_zhi"]
    counts = np.diff(d["off"]).copy()
    counts[1] = 0
    counts[3] = 1
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n = int(off[-1])
    xy, lo, hi = xy[:n], lo[:n], hi[:n]
    iou, saved, seg = dg.iou_matrix(dev_t(xy), a_z=(dev_t(lo), dev_t(hi)), a_off=off,
                                    self_pairs=True, save=True)
    dg.check_errors()
    ref, _ = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL


def test_segmented_two_sets(dg):
    """Segments that pair different row and column sets (not self pairs)."""
    d = synth.c2_matrix(n=400, m=300, seed=10)
    a, b = _crowd(d["a_xy"], 0.1), _crowd(d["b_xy"], 0.1)
    a_off = np.array([0, 100, 100, 250, 400], np.int64)
    b_off = np.array([0, 50, 120, 121, 300], np.int64)
    iou, saved, seg = dg.iou_matrix(dev_t(a), dev_t(b), a_off=a_off, b_off=b_off, save=True)
    ref, _ = oracle.iou_matrix(a, b, a_off=a_off, b_off=b_off)
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    g = np.random.default_rng(11).uniform(-1, 1, ref.shape[0]).astype(np.float32)
    ga, gb, _, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(a), dev_t(b))
    ia, ib, fl = _aabb_candidates(a, b, a_off, b_off)
    ra, sa, rb, sb = _grad_reference(a, b, g, ia, ib, fl)
    om_a, om_b, _, _ = oracle.iou_matrix_grad(g, a, b, a_off=a_off, b_off=b_off)
    assert np.abs(rb - om_b.reshape(len(b), -1)).max() <= 1e-12 * (1 + np.abs(om_b).max())
    _assert_box_grads(_box_grads(ga), ra, sa, "rows")
    _assert_box_grads(_box_grads(gb), rb, sb, "columns")


def _shape_run(dg, rows, a, b, anv=None, bnv=None, z=None, off=None, self_pairs=False,
               g=None):
    """Forward (+ backward with g) with the tile shape fixed to `rows` rows."""
    ta = dev_t(a)
    tb = ta if self_pairs else dev_t(b)
    tz = None if z is None else (dev_t(z[0]), dev_t(z[1]))
    tanv = None if anv is None else dev_t(anv)
    tbnv = tanv if self_pairs else (None if bnv is None else dev_t(bnv))
    seg = dg.segments(len(a), len(a) if self_pairs else len(b), off, self_pairs=self_pairs)
    sv = dg.SavedPairs(1 << 20, a.shape[1] + (a if self_pairs else b).shape[1], seg[5],
                       ta.device, tile_rows=rows)
    iou, saved, seg4 = dg.iou_matrix(ta, None if self_pairs else tb, tanv,
                                     None if self_pairs else tbnv, tz, None, off,
                                     self_pairs=self_pairs, save=True, seg=seg, saved=sv)
    dg.check_errors()
    assert saved.tile_rows == rows
    pid, snx, _, _ = _saved_entries(saved)
    grads = None
    if g is not None:
        if self_pairs:
            ga, _, gz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg4, ta, None, tanv, None,
                                                  tz, None, self_pairs=True)
            grads = (_box_grads(ga, gz),)
        else:
            ga, gb, _, _ = dg.iou_matrix_backward(dev_t(g), saved, seg4, ta, tb, tanv, tbnv)
            grads = (_box_grads(ga), _box_grads(gb))
    return iou.cpu().numpy().reshape(-1), np.sort(pid), grads


@pytest.mark.parametrize("rows", [4, 16])
def test_tile_shapes_agree(dg, rows):
    """A tile shape other than the default computes the same IoU bit for bit
    and the same survivor set as 8-row tiles, and its backward meets the
    gradient bar against the oracle: a ragged two-set block of counted
    polygons, and ragged 3D self-pair scenes (the diagonal crosses tiles
    differently in every shape)."""
    _say(f"case: tile rows {rows}, polygon block 333 x 517 and 7 scenes")
    d = synth.c4_polygons(n=600, seed=15)
    a, anv, b, bnv = d["a_xy"][:333], d["a_nv"][:333], d["b_xy"][:517], d["b_nv"][:517]
    g = np.random.default_rng(16).uniform(-1, 1, 333 * 517).astype(np.float32)
    ref = _shape_run(dg, 8, a, b, anv, bnv)
    got = _shape_run(dg, rows, a, b, anv, bnv, g=g)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    om, _ = oracle.iou_matrix(a, b, anv, bnv)
    assert np.abs(got[0] - om).max() <= IOU_TOL
    ia, ib, fl = _aabb_candidates(a, b)
    ra, sa, rb, sb = _grad_reference(a, b, g, ia, ib, fl, anv, bnv)
    _assert_box_grads(got[2][0], ra, sa, "rows")
    _assert_box_grads(got[2][1], rb, sb, "columns")

    xy, lo, hi, off, out_off = _scenes(7, 3, 600, 17, 0.12)
    gs = np.random.default_rng(18).uniform(-1, 1, int(out_off[-1])).astype(np.float32)
    ref = _shape_run(dg, 8, xy, None, z=(lo, hi), off=off, self_pairs=True)
    got = _shape_run(dg, rows, xy, None, z=(lo, hi), off=off, self_pairs=True, g=gs)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    om, _ = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.abs(got[0] - om).max() <= IOU_TOL
    ia, ib, fl = _aabb_candidates(xy, xy, off, off, True)
    rg, sg = _grad_reference(xy, xy, gs, ia, ib, fl, a_z=(lo, hi), b_z=(lo, hi), self_pairs=True)
    e = _assert_box_grads(got[2][0], rg, sg, "scenes")
    _say(f"tile rows {rows}: {len(got[1])} scene survivors, max rel err {e:.2e}")


def test_scenes_full_size(dg):
    """64 ragged scenes, 3D self pairs, the benchmark shape: the forward is
    checked on every pair (AABB-disjoint pairs 0, the rest against the oracle);
    the backward against the oracle's gradients summed over the saved pairs."""
    d = synth.c5_scenes()
    xy, lo, hi, off, out_off = d["a_xy"], d["a_zlo"], d["a_zhi"], d["off"], d["out_off"]
    _say(f"case: c5 full, {len(xy)} boxes, {int(out_off[-1])} pairs")
    txy, tlo, thi = dev_t(xy), dev_t(lo), dev_t(hi)
    iou, saved, seg = dg.iou_matrix(txy, a_z=(tlo, thi), a_off=off, self_pairs=True, save=True)
    dg.check_errors()
    flat = iou.cpu().numpy()
    ia, ib, fl, ref, nx, xf = _check_matrix_exact(flat, xy, xy, (lo, hi), (lo, hi), off, off,
                                                  self_pairs=True)
    cnt = int(saved.count.item())
    nonempty = (nx > 0) & (ia != ib)
    # z-disjoint pairs are culled before the intersection: the saved entries
    # with nx > 0 are the pairs with a non-empty BEV intersection and
    # overlapping z-extents
    zov = np.minimum(hi[ia], hi[ib]) > np.maximum(lo[ia], lo[ib])
    pid, snx, _, _ = _saved_entries(saved)
    assert np.array_equal(np.sort(pid[snx > 0]), np.sort(fl[nonempty & zov]))
    g = d["grad"]
    ga, _, gaz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, txy, a_z=(tlo, thi),
                                           self_pairs=True)
    sel = nonempty & zov
    ref, scale = _grad_reference(xy, xy, g, ia[sel], ib[sel], fl[sel], a_z=(lo, hi),
                                 b_z=(lo, hi), self_pairs=True)
    e = _assert_box_grads(_box_grads(ga, gaz), ref, scale, "c5")
    _say(f"c5: {cnt} survivors, {int((snx > 0).sum())} non-empty, grad rel err max {e:.2e} "
         f"over {len(xy)} boxes")


def _tie_scenes(seed, scenes=5):
    """Scenes of 3D boxes full of exact contacts: integer axis-aligned boxes
    with collinear and touching edges, exact duplicates, a common ground
    plane (shared zlo) and shared tops, yaw-0 rows next to rotated boxes."""
    rng = np.random.default_rng(seed)
    xs, los, his, sizes = [], [], [], []
    for s in range(scenes):
        n_int = int(rng.integers(8, 40))
        x0 = rng.integers(0, 6, n_int).astype(np.float64)
        y0 = rng.integers(0, 6, n_int).astype(np.float64)
        w = rng.integers(1, 4, n_int).astype(np.float64)
        h = rng.integers(1, 4, n_int).astype(np.float64)
        q = np.stack([np.stack([x0, y0], 1), np.stack([x0 + w, y0], 1),
                      np.stack([x0 + w, y0 + h], 1), np.stack([x0, y0 + h], 1)], 1)
        nr = int(rng.integers(2, 10))
        rot = synth.boxes_to_quads(rng.uniform(1, 5, nr), rng.uniform(1, 5, nr),
                                   rng.uniform(1, 3, nr), rng.uniform(1, 3, nr),
                                   rng.uniform(-np.pi, np.pi, nr))
        yaw0 = synth.boxes_to_quads(rng.integers(1, 5, 3).astype(float) + 0.5,
                                    rng.integers(1, 5, 3).astype(float), np.full(3, 2.0),
                                    np.full(3, 3.0), np.zeros(3))
        xy = np.concatenate([q.astype(np.float32), rot, yaw0, q[:4].astype(np.float32)], 0)
        n = len(xy)
        lo = np.where(rng.uniform(size=n) < 0.6, 0.0, rng.integers(-1, 2, n)).astype(np.float32)
        hi = (lo + rng.integers(1, 3, n)).astype(np.float32)
        hi[::4] = 2.0
        lo = np.minimum(lo, hi - 1.0).astype(np.float32)
        xs.append(xy)
        los.append(lo)
        his.append(hi)
        sizes.append(n)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.concatenate(xs), np.concatenate(los), np.concatenate(his), off


def test_scenes_with_ties(dg):
    """Self-pair scenes where the tie rule decides on most pairs (collinear and
    touching integer edges, duplicate boxes, shared ground planes and tops):
    IoU on every pair, the block exactly symmetric, and every box's gradient
    against the oracle's (one structure per unordered pair, lower index
    first), at the maximum."""
    xy, lo, hi, off = _tie_scenes(61)
    _say(f"case: tie scenes {np.diff(off).tolist()}")
    z = (dev_t(lo), dev_t(hi))
    iou, saved, seg = dg.iou_matrix(dev_t(xy), a_z=z, a_off=off, self_pairs=True, save=True)
    dg.check_errors()
    got = iou.cpu().numpy()
    ref, out_off = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.abs(got - ref).max() <= IOU_TOL
    for s in range(len(off) - 1):
        n = int(off[s + 1] - off[s])
        blk = got[out_off[s]:out_off[s + 1]].reshape(n, n)
        assert np.array_equal(blk, blk.T), s
    assert np.count_nonzero(ref) > 2 * len(xy)
    g = np.random.default_rng(62).uniform(-1, 1, ref.shape[0]).astype(np.float32)
    ga, _, gz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(xy), a_z=z, self_pairs=True)
    ra, _, rz, _ = oracle.iou_matrix_grad(g, xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    ia, ib, fl = _aabb_candidates(xy, xy, off, off, True)
    rr, scale = _grad_reference(xy, xy, g, ia, ib, fl, a_z=(lo, hi), b_z=(lo, hi),
                                self_pairs=True)
    om = np.concatenate([ra.reshape(len(xy), -1), rz], 1)
    assert np.abs(rr - om).max() <= 1e-12 * (1 + np.abs(om).max())
    e = _assert_box_grads(_box_grads(ga, gz), rr, scale, "tie scenes")
    _say(f"tie scenes: {int(saved.count.item())} saved pairs, max rel err {e:.2e}")


def test_scenes_full_size_graph_replay(dg):
    """The benchmark's step as a user writes it: per-scene 3D self-pair IoU
    forward + backward through the autograd wrapper in its capturable form
    (device segment table and work list made before capture), captured in a
    HIP graph at full size (64 scenes, ~94 M pairs) and replayed with eager
    work in between; every replay equals the eager step bit for bit, and the
    eager step equals the oracle on sampled boxes."""
    d = synth.c5_scenes()
    xy, lo, hi, off = d["a_xy"], d["a_zlo"], d["a_zhi"], d["off"]
    _say(f"case: c5 graph replay, {len(xy)} boxes, {int(d['out_off'][-1])} pairs")
    txy, tlo, thi = dev_t(xy), dev_t(lo), dev_t(hi)
    g = dev_t(d["grad"])
    seg = dg.segments(len(xy), len(xy), off, self_pairs=True)
    work = (seg, dg.SavedPairs(1 << 21, 8, seg[5], txy.device))
    params = [t.clone().requires_grad_(True) for t in (txy, tlo, thi)]

    def step():
        for p_ in params:
            p_.grad = None
        out = dg.IoU3DScenes.apply(params[0], params[1], params[2], off, None, work)
        out.backward(g)
        return out

    out_e = step().detach().clone()
    grads_e = [p_.grad.clone() for p_ in params]
    dg.check_errors()
    cnt = int(work[1].count.item())
    assert 0 < cnt <= work[1].capacity
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out_g = step()
    grads_g = [p_.grad for p_ in params]
    for rep in range(3):
        junk = torch.randn(1 << 22, device="cuda").sum()  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_g, out_e), rep
        # self pairs: every row sum is added in a fixed order, so the
        # gradients are the same bits too
        for a_, b_ in zip(grads_g, grads_e):
            assert torch.equal(a_, b_), rep
        del junk
    dg.check_errors()
    # the eager step against the oracle on sampled boxes (all their pairs)
    rng = np.random.default_rng(63)
    flat = out_e.cpu().numpy()
    boxes = rng.choice(len(xy), 300, replace=False)
    scene = np.searchsorted(off, boxes, side="right") - 1
    ia_l, ib_l, fl_l = [], [], []
    for bx, sc in zip(boxes, scene):
        n = int(off[sc + 1] - off[sc])
        r = int(bx - off[sc])
        cols = np.arange(n)
        ia_l += [np.full(n, bx), off[sc] + cols]
        ib_l += [off[sc] + cols, np.full(n, bx)]
        fl_l += [d["out_off"][sc] + r * n + cols, d["out_off"][sc] + cols * n + r]
    ia, ib, fl = np.concatenate(ia_l), np.concatenate(ib_l), np.concatenate(fl_l)
    fl, first = np.unique(fl, return_index=True)  # two sampled boxes may share entries
    ia, ib = ia[first], ib[first]
    v, _, _ = oracle.iou_index_pairs(np.minimum(ia, ib), np.maximum(ia, ib), xy, xy,
                                     a_z=(lo, hi), b_z=(lo, hi), threads=8)
    v = np.where(ia == ib, 1.0, v)
    assert np.abs(flat[fl] - v).max() <= IOU_TOL
    ov = (v != 0) & (ia != ib)
    gz = torch.stack([grads_e[1], grads_e[2]], 1)
    ref, scale = _grad_reference(xy, xy, d["grad"], ia[ov], ib[ov], fl[ov], a_z=(lo, hi),
                                 b_z=(lo, hi), self_pairs=True)
    e = _assert_box_grads(_box_grads(grads_e[0], gz)[boxes], ref[boxes], scale[boxes], "c5 graph")
    _say(f"c5 graph replay: {cnt} survivors, sampled max rel err {e:.2e}")


def test_graph_replay_matches_eager(dg):
    """Scenes forward + backward captured in a HIP graph (via torch), replayed
    several times with eager work in between; every replay equals eager."""
    xy, lo, hi, off, out_off = _scenes(4, 30, 300, 12, 0.15)
    g = dev_t(np.random.default_rng(13).uniform(-1, 1, int(out_off[-1])).astype(np.float32))
    txy, tlo, thi = dev_t(xy), dev_t(lo), dev_t(hi)
    iou_e, saved_e, seg_e = dg.iou_matrix(txy, a_z=(tlo, thi), a_off=off, self_pairs=True,
                                          save=True)
    ga_e, _, gaz_e, _ = dg.iou_matrix_backward(g, saved_e, seg_e, txy, a_z=(tlo, thi),
                                               self_pairs=True)
    seg_t = dg.segments(len(xy), len(xy), off, self_pairs=True)  # device table, before capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):  # warm up on the side stream
            iou_w, saved_w, seg_w = dg.iou_matrix(txy, a_z=(tlo, thi), a_off=off, self_pairs=True,
                                                  save=True, check=False, seg=seg_t)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        iou_g, saved_g, seg_g = dg.iou_matrix(txy, a_z=(tlo, thi), a_off=off, self_pairs=True,
                                              save=True, check=False, seg=seg_t)
        ga_g, _, gaz_g, _ = dg.iou_matrix_backward(g, saved_g, seg_g, txy, a_z=(tlo, thi),
                                                   self_pairs=True)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(iou_g, iou_e), rep
        assert int(saved_g.count.item()) == int(saved_e.count.item())
        # the tiles of the shape used (the table has room for every shape's)
        assert saved_g.tiles_used == saved_e.tiles_used
        nt = saved_e.tiles_used
        assert torch.equal(saved_g.tile_count[:nt], saved_e.tile_count[:nt])
        assert torch.equal(ga_g, ga_e), rep
        assert torch.equal(gaz_g, gaz_e), rep
        del junk


def test_invalid_segments_are_rejected(dg):
    xy, lo, hi, off, out_off = _scenes(3, 10, 20, 14, None)
    txy = dev_t(xy)
    pa, _ = dg.polys(txy)
    bad_a = torch.tensor([0, 5, 3, int(off[-1])], dtype=torch.int64, device="cuda")  # decreasing
    good_o = torch.tensor([0, 25, 25], dtype=torch.int64, device="cuda")
    out = torch.zeros(int(out_off[-1]), device="cuda")
    work = dg.SavedPairs(1 << 12, 8, 64, torch.device("cuda"))
    ws = work.struct()
    # a work list is required
    assert dg.lib.dgal_iou_matrix(dg.context(), pa, pa, None, None, None, 0, 0, out.data_ptr(),
                                  out.numel(), None, 0) == dg.DGAL_EINVAL
    st = dg.lib.dgal_iou_matrix(dg.context(), pa, pa, bad_a.data_ptr(), bad_a.data_ptr(),
                                good_o.data_ptr(), 3, 1, out.data_ptr(), out.numel(),
                                dg.ctypes.byref(ws), torch.cuda.current_stream().cuda_stream)
    assert st == dg.DGAL_OK          # offsets live on the device: reported by the check
    with pytest.raises(dg.DgalError) as e:
        dg.check_errors()
    assert e.value.status == dg.DGAL_EINVAL
    dg.check_errors()                # the error word was cleared
    # immediate errors
    assert dg.lib.dgal_iou_matrix(dg.context(), pa, pa, bad_a.data_ptr(), None, None, 3, 1,
                                  out.data_ptr(), out.numel(), dg.ctypes.byref(ws),
                                  0) == dg.DGAL_EINVAL
    assert dg.lib.dgal_iou_matrix(dg.context(), pa, pa, None, None, None, 0, 0,
                                  out.data_ptr(), 10, dg.ctypes.byref(ws),
                                  0) == dg.DGAL_EINVAL  # out too small


@pytest.mark.parametrize("rows", [4, 8, 16])
def test_cull_keeps_nothing_past_the_block(dg, rows):
    """Rows and columns past a block (its last tiles are ragged) never
    survive the count pass, whatever infinite bounds the other side has: a
    column box reaching x = -inf meets the padded rows of the last tile row,
    and a row box reaching x = -inf the padded columns of the last tile
    column, in a pair test whose difference with the padding's -inf bound is
    NaN.  The finite boxes are placed so that no pair overlaps at all: the
    work list is empty and the output all 0."""
    na, nb = 13, 300  # 13 % rows != 0 and 300 % (2048 / rows) != 0: padded rows and columns
    rng = np.random.default_rng(81)

    def boxes(n, x_lo, x_hi, y_lo, y_hi):
        return synth.boxes_to_quads(rng.uniform(x_lo, x_hi, n), rng.uniform(y_lo, y_hi, n),
                                    np.full(n, 1.0), np.full(n, 2.0), rng.uniform(-np.pi, np.pi, n))

    # x in [-inf, 1], y in [-2, 2]: a padded row or column (bounds 0 .. -1, x1
    # = -inf) passes the test against it unless the padding is excluded
    star = np.array([[-np.inf, -2.0], [1.0, -2.0], [1.0, 2.0], [-np.inf, 2.0]], np.float32)
    for side in ("column", "row"):
        _say(f"case: infinite {side} bound, {na} x {nb}, tile rows {rows}")
        a = boxes(na, 100.0, 200.0, -50.0, 50.0)  # rows: far right of the star
        b = boxes(nb, -300.0, -200.0, 10.0, 20.0)  # columns: left of it, above y = 2
        if side == "column":
            b[5] = star
        else:
            a[2] = star
        seg = dg.segments(na, nb, None)
        sv = dg.SavedPairs(1 << 12, 8, seg[5], torch.device("cuda"), tile_rows=rows)
        iou, saved, _ = dg.iou_matrix(dev_t(a), dev_t(b), save=True, seg=seg, saved=sv)
        dg.check_errors()
        assert saved.tile_rows == rows
        assert int(saved.count.item()) == 0, side
        assert not iou.cpu().numpy().any(), side


def test_saved_capacity_overflow_is_reported(dg):
    d = synth.c2_matrix(n=100, m=100, seed=15)
    a = _crowd(d["a_xy"], 0.02)
    with pytest.raises(dg.DgalError) as e:
        dg.iou_matrix(dev_t(a), dev_t(a), save=True, capacity=4)
    assert e.value.status == dg.DGAL_ECAPACITY
    dg.check_errors()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_ragged_segments(dg, seed):
    """Random ragged segmentations (empty segments included, sizes that are
    not multiples of the 8 x 256 tile): two sets, and 3D self-pair scenes;
    IoU on every pair and gradients against the oracle."""
    rng = np.random.default_rng(3000 + seed)
    na, nb = int(rng.integers(1, 700)), int(rng.integers(1, 700))
    d = synth.c2_matrix(n=na, m=nb, seed=3100 + seed)
    a = _crowd(d["a_xy"], float(rng.uniform(0.05, 0.3)))
    b = _crowd(d["b_xy"], float(rng.uniform(0.05, 0.3)))
    ns = int(rng.integers(1, 7))
    a_off = np.concatenate([[0], np.sort(rng.integers(0, na + 1, ns - 1)), [na]]).astype(np.int64)
    b_off = np.concatenate([[0], np.sort(rng.integers(0, nb + 1, ns - 1)), [nb]]).astype(np.int64)
    _say(f"case: two sets {na} x {nb}, segments {a_off.tolist()} / {b_off.tolist()}")
    iou, saved, seg = dg.iou_matrix(dev_t(a), dev_t(b), a_off=a_off, b_off=b_off, save=True)
    ref, _ = oracle.iou_matrix(a, b, a_off=a_off, b_off=b_off)
    if ref.size:
        assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    g = rng.uniform(-1, 1, ref.shape[0]).astype(np.float32)
    ga, gb, _, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(a), dev_t(b))
    if ref.size:
        ia, ib, fl = _aabb_candidates(a, b, a_off, b_off)
        ra, sa, rb, sb = _grad_reference(a, b, g, ia, ib, fl)
        _assert_box_grads(_box_grads(ga), ra, sa, "rows")
        _assert_box_grads(_box_grads(gb), rb, sb, "columns")
    else:
        assert not ga.any() and not gb.any()
    sizes = rng.integers(0, 300, int(rng.integers(1, 9)))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    if n == 0:
        return
    d5 = synth.c5_scenes(scenes=1, nmin=n, nmax=n, seed=3200 + seed)
    xy = _crowd(d5["a_xy"][:n], float(rng.uniform(0.1, 0.4)))
    lo, hi = d5["a_zlo"][:n], d5["a_zhi"][:n]
    _say(f"case: scenes {sizes.tolist()}")
    z = (dev_t(lo), dev_t(hi))
    iou, saved, seg = dg.iou_matrix(dev_t(xy), a_z=z, a_off=off, self_pairs=True, save=True)
    ref, _ = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    g = rng.uniform(-1, 1, ref.shape[0]).astype(np.float32)
    ga, _, gz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(xy), a_z=z, self_pairs=True)
    ia, ib, fl = _aabb_candidates(xy, xy, off, off, True)
    rr, scale = _grad_reference(xy, xy, g, ia, ib, fl, a_z=(lo, hi), b_z=(lo, hi),
                                self_pairs=True)
    _assert_box_grads(_box_grads(ga, gz), rr, scale, "scenes")


def test_max_segments(dg):
    """DGAL_MAX_SEGMENTS (4096) self-pair scenes of 0..6 boxes each: the
    segment prefix spread over the prefix kernel's threads, many empty and
    one-box scenes; IoU and gradients against the oracle."""
    rng = np.random.default_rng(44)
    sizes = rng.integers(0, 7, dg.MAX_SEGMENTS)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    d = synth.c5_scenes(scenes=1, nmin=n, nmax=n, seed=45)
    xy, lo, hi = d["a_xy"][:n], d["a_zlo"][:n], d["a_zhi"][:n]
    # every scene's boxes near one point, so that they overlap
    centre = np.repeat(rng.uniform(0, 50, (len(sizes), 2)), sizes, axis=0)
    xy = (xy - xy.mean(1, keepdims=True) + centre[:, None, :]
          + rng.normal(0, 0.5, (n, 1, 2))).astype(np.float32)
    _say(f"case: {len(sizes)} scenes, {n} boxes")
    z = (dev_t(lo), dev_t(hi))
    iou, saved, seg = dg.iou_matrix(dev_t(xy), a_z=z, a_off=off, self_pairs=True, save=True)
    ref, _ = oracle.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.abs(iou.cpu().numpy() - ref).max() <= IOU_TOL
    assert np.count_nonzero(ref) > 3 * n
    g = rng.uniform(-1, 1, ref.shape[0]).astype(np.float32)
    ga, _, gz, _ = dg.iou_matrix_backward(dev_t(g), saved, seg, dev_t(xy), a_z=z, self_pairs=True)
    ia, ib, fl = _aabb_candidates(xy, xy, off, off, True)
    rr, scale = _grad_reference(xy, xy, g, ia, ib, fl, a_z=(lo, hi), b_z=(lo, hi),
                                self_pairs=True)
    _assert_box_grads(_box_grads(ga, gz), rr, scale, "scenes")


def test_default_capacity_grows(dg):
    """Boxes crowded so that nearly every pair survives the cull, far more
    than the default capacity (pairs / 16): the binding repeats the call
    once with room for all survivors; IoU and gradients match the oracle."""
    d = synth.c2_matrix(n=1500, m=1500, seed=16)
    a = _crowd(d["a_xy"], 0.01)
    ta = dev_t(a)
    iou, saved, seg = dg.iou_matrix(ta, ta, save=True)
    cnt = int(saved.count.item())
    assert cnt > 1500 * 1500 // 16 and saved.capacity >= cnt
    rng = np.random.default_rng(17)
    r, c = rng.integers(0, 1500, 20000), rng.integers(0, 1500, 20000)
    ref, _, _ = oracle.iou_index_pairs(r, c, a, a, threads=8)
    assert np.abs(iou.cpu().numpy()[r, c] - ref).max() <= IOU_TOL
    g = rng.uniform(-1, 1, (1500, 1500)).astype(np.float32)
    ga, gb, _, _ = dg.iou_matrix_backward(dev_t(g).reshape(-1), saved, seg, ta, ta)
    ia, ib, fl = _aabb_candidates(a, a)
    ra, sa, rb, sb = _grad_reference(a, a, g.reshape(-1), ia, ib, fl)
    _assert_box_grads(_box_grads(ga), ra, sa, "rows")
    _assert_box_grads(_box_grads(gb), rb, sb, "columns")


def test_matrix_beyond_int32(dg):
    """A 65,536 x 33,000 matrix: 2.16e9 pairs (8.6 GB of output), flat indices
    past 2^31.  Checked without copying the output: the saved survivors
    (those past 2^31 and a sample of the rest) against the oracle, the
    output's non-zero count against the survivors with a positive IoU,
    random flat indices on both sides of 2^31 against the AABB test and the
    oracle, and sampled row / column gradients against the oracle's pair
    gradients summed over the saved survivors."""
    na, nb = 65536, 33000
    total = na * nb
    assert total > 2 ** 31
    rng = np.random.default_rng(41)

    def boxes(n):
        cx, cy = rng.uniform(0, 400, n), rng.uniform(0, 400, n)
        w, l = rng.uniform(1, 3, n), rng.uniform(1, 3, n)
        return synth.boxes_to_quads(cx, cy, w, l, rng.uniform(-np.pi, np.pi, n))

    a, b = boxes(na), boxes(nb)
    _say(f"case: matrix {na} x {nb} = {total} pairs")
    ta, tb = dev_t(a), dev_t(b)
    iou, saved, seg = dg.iou_matrix(ta, tb, save=True, capacity=1 << 22)
    dg.check_errors()
    assert iou.shape == (na, nb)
    iou = iou.reshape(-1)  # flat, as the saved pair ids index it
    cnt = int(saved.count.item())
    assert 0 < cnt <= saved.capacity
    st = saved.tile_start[:saved.tiles_used].cpu().numpy()
    sc = saved.tile_count[:saved.tiles_used].cpu().numpy().astype(np.int64)
    ent = np.repeat(st, sc) + (np.arange(int(sc.sum())) - np.repeat(np.cumsum(sc) - sc, sc))
    pid = saved.pair_id.cpu().numpy()[ent]
    assert len(pid) == cnt and len(np.unique(pid)) == cnt
    # checked on the host before any device gather uses them
    assert pid.min() >= 0 and pid.max() < total
    assert pid.max() > 2 ** 31
    got = iou[torch.from_numpy(pid).cuda()].cpu().numpy()
    # every non-zero output value is a saved survivor's
    assert int(torch.count_nonzero(iou).item()) == int(np.count_nonzero(got))
    # saved survivors: all those past 2^31 (up to 40,000) and 40,000 others
    hi = np.flatnonzero(pid >= 2 ** 31)[:40000]
    lo = rng.choice(np.flatnonzero(pid < 2 ** 31), min(40000, int((pid < 2 ** 31).sum())),
                    replace=False)
    sel = np.concatenate([hi, lo])
    ref, _, _ = oracle.iou_index_pairs(pid[sel] // nb, pid[sel] % nb, a, b, threads=16)
    assert np.abs(got[sel] - ref).max() <= IOU_TOL
    # random flat indices on both sides of 2^31
    flat = np.concatenate([rng.integers(0, 2 ** 31, 500000), rng.integers(2 ** 31, total, 500000)])
    val = iou[torch.from_numpy(flat).cuda()].cpu().numpy()
    ia, ib = flat // nb, flat % nb
    lo_a, hi_a, lo_b, hi_b = a.min(1), a.max(1), b.min(1), b.max(1)
    ov = np.all((lo_a[ia] <= hi_b[ib]) & (lo_b[ib] <= hi_a[ia]), axis=1)
    assert not val[~ov].any()
    if ov.any():
        r2, _, _ = oracle.iou_index_pairs(ia[ov], ib[ov], a, b, threads=16)
        assert np.abs(val[ov] - r2).max() <= IOU_TOL
    # backward: rows and columns of the saved survivors' pair gradients
    g = torch.rand(total, device="cuda", generator=torch.Generator("cuda").manual_seed(5)) - 0.5
    ga, gb, _, _ = dg.iou_matrix_backward(g, saved, seg, ta, tb)
    dg.check_errors()
    gs = g[torch.from_numpy(pid).cuda()].cpu().numpy()
    rows = rng.choice(np.unique(pid // nb), 300, replace=False)
    cols = rng.choice(np.unique(pid % nb), 300, replace=False)
    on_rows = np.isin(pid // nb, rows)
    on_cols = np.isin(pid % nb, cols)
    pick = on_rows | on_cols
    ra, sa, rb, sb = _grad_reference(a, b, gs[pick], pid[pick] // nb, pid[pick] % nb,
                                     np.arange(int(pick.sum())))
    _assert_box_grads(_box_grads(ga)[rows], ra[rows], sa[rows], "rows")
    _assert_box_grads(_box_grads(gb)[cols], rb[cols], sb[cols], "columns")
    _say(f"matrix beyond int32: {cnt} survivors, {len(hi)} past 2^31")


def test_scenes_beyond_int32(dg):
    """Two self-pair scenes of 33,000 boxes: 2.18e9 pairs in one flat output,
    the second scene's block starting past 2^31.  Saved survivors of both
    scenes against the oracle, non-zero count, the diagonal, and sampled
    per-box gradients (row role with the transpose's upstream gradient)."""
    ns = 33000
    off = np.array([0, ns, 2 * ns], np.int64)
    total = 2 * ns * ns
    assert total > 2 ** 31 and ns * ns < 2 ** 31
    rng = np.random.default_rng(43)
    n = 2 * ns
    xy = synth.boxes_to_quads(rng.uniform(0, 300, n), rng.uniform(0, 300, n),
                              rng.uniform(1, 3, n), rng.uniform(1, 3, n),
                              rng.uniform(-np.pi, np.pi, n))
    _say(f"case: 2 scenes x {ns} boxes = {total} self pairs")
    txy = dev_t(xy)
    iou, saved, seg = dg.iou_matrix(txy, a_off=off, self_pairs=True, save=True,
                                    capacity=1 << 22)
    dg.check_errors()
    cnt = int(saved.count.item())
    st = saved.tile_start[:saved.tiles_used].cpu().numpy()
    sc = saved.tile_count[:saved.tiles_used].cpu().numpy().astype(np.int64)
    ent = np.repeat(st, sc) + (np.arange(int(sc.sum())) - np.repeat(np.cumsum(sc) - sc, sc))
    pid = saved.pair_id.cpu().numpy()[ent]
    assert len(pid) == cnt and len(np.unique(pid)) == cnt
    assert pid.min() >= 0 and pid.max() < total  # before any device gather uses them
    s_ = (pid >= ns * ns).astype(np.int64)  # scene of each survivor
    assert s_.sum() > 0
    local = pid - s_ * ns * ns
    ia, ib = off[s_] + local // ns, off[s_] + local % ns
    got = iou[torch.from_numpy(pid).cuda()].cpu().numpy()
    # the diagonal is written as 1 by the cull and not saved
    diag = ia == ib
    assert not diag.any()
    dflat = np.concatenate([k * ns * ns + np.arange(ns) * (ns + 1) for k in range(2)])
    assert np.all(iou[torch.from_numpy(dflat).cuda()].cpu().numpy() == 1.0)
    assert int(torch.count_nonzero(iou).item()) == int(np.count_nonzero(got)) + n
    sel = np.concatenate([np.flatnonzero(pid >= 2 ** 31)[:30000],
                          np.flatnonzero(pid < 2 ** 31)[:30000]])
    ref, _, _ = oracle.iou_index_pairs(ia[sel], ib[sel], xy, xy, threads=16)
    assert np.abs(got[sel] - ref).max() <= IOU_TOL
    g = torch.rand(total, device="cuda", generator=torch.Generator("cuda").manual_seed(6)) - 0.5
    ga, _, _, _ = dg.iou_matrix_backward(g, saved, seg, txy, self_pairs=True)
    dg.check_errors()
    # the saved entries hold both (i, k) and (k, i); every entry of a sampled
    # box, weighted by its own upstream gradient, gives that box its role's
    # gradient of the unordered pair (lower index first)
    boxes = rng.choice(np.unique(ia), 400, replace=False)
    pick = np.isin(ia, boxes) | np.isin(ib, boxes)
    gs = g[torch.from_numpy(pid[pick]).cuda()].cpu().numpy()
    ref, scale = _grad_reference(xy, xy, gs, ia[pick], ib[pick], np.arange(int(pick.sum())),
                                 self_pairs=True)
    _assert_box_grads(_box_grads(ga)[boxes], ref[boxes], scale[boxes], "scenes")
    _say(f"scenes beyond int32: {cnt} survivors, {int((pid >= 2 ** 31).sum())} past 2^31")

