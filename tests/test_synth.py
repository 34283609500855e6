"""Seeded generators: shapes, reproducibility, distributions and the
convex/counter-clockwise precondition of every generated polygon."""
import math

import numpy as np

import synth


def _ccw_strict(xy, n):
    p = xy[:n].astype(np.float64)
    u = p - np.roll(p, 1, 0)
    v = np.roll(p, -1, 0) - p
    return bool(np.all(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0] > 0))


def test_reproducible():
    for name, kw in (("c1", {}), ("c3", {"n": 5000}), ("c4", {"n": 3000}),
                     ("c2", {"n": 300, "m": 200}), ("c5", {"scenes": 4})):
        d1, d2 = synth.get(name, **kw), synth.get(name, **kw)
        for k in d1:
            if isinstance(d1[k], np.ndarray):
                assert np.array_equal(d1[k], d2[k]), (name, k)


def test_rectangles_ccw_and_distribution():
    d = synth.c1_pairs()
    a, b = d["a_xy"], d["b_xy"]
    assert a.shape == (1024, 4, 2) and a.dtype == np.float32
    assert all(_ccw_strict(a[i], 4) and _ccw_strict(b[i], 4) for i in range(1024))
    c = a.astype(np.float64).mean(1)
    assert np.all(np.abs(c) <= 2.0 + 1e-5)
    side = np.hypot(*(a[:, 1] - a[:, 0]).T.astype(np.float64))  # = w
    assert side.min() >= 1.0 - 1e-5 and side.max() <= 3.0 + 1e-5
    dc = b.astype(np.float64).mean(1) - c
    assert abs(dc.std() - 0.5) < 0.05
    assert np.all((d["grad"] >= -1) & (d["grad"] <= 1))


def test_perturbed_pairs_sizes():
    d = synth.c3_pairs(n=20000)
    b = d["b_xy"].astype(np.float64)
    w = np.hypot(*(b[:, 2] - b[:, 1]).T)
    l = np.hypot(*(b[:, 1] - b[:, 0]).T)
    assert w.min() >= 0.1 - 1e-6 and l.min() >= 0.1 - 1e-6


def test_bev_boxes():
    d = synth.c2_matrix(n=2000, m=10)
    a = d["a_xy"].astype(np.float64)
    c = a.mean(1)
    assert c[:, 0].min() >= 0 and c[:, 0].max() <= 70
    assert c[:, 1].min() >= -40 and c[:, 1].max() <= 40
    w = np.hypot(*(a[:, 1] - a[:, 0]).T)     # corners 0 -> 1 run across the heading
    l = np.hypot(*(a[:, 2] - a[:, 1]).T)
    assert w.min() >= 1.5 - 1e-4 and w.max() <= 2.2 + 1e-4
    assert l.min() >= 3.5 - 1e-4 and l.max() <= 5.0 + 1e-4


def test_convex_polygons():
    d = synth.c4_polygons(n=20000)
    for xy, nv in ((d["a_xy"], d["a_nv"]), (d["b_xy"], d["b_nv"])):
        assert xy.shape == (20000, 8, 2) and nv.min() == 3 and nv.max() == 8
        counts = np.bincount(nv, minlength=9)[3:]
        assert counts.min() > 0.8 * counts.mean()
        for i in range(0, 20000, 37):
            n = int(nv[i])
            assert _ccw_strict(xy[i], n)
            assert not xy[i, n:].any()


def test_scenes():
    d = synth.c5_scenes()
    off, out_off = d["off"], d["out_off"]
    counts = np.diff(off)
    assert counts.shape == (64,) and counts.min() >= 50 and counts.max() <= 2000
    assert np.array_equal(np.diff(out_off), counts ** 2)
    assert d["grad"].shape == (out_off[-1],)
    assert np.all(d["a_zhi"] > d["a_zlo"])
    h = (d["a_zhi"] - d["a_zlo"]).astype(np.float64)
    assert h.min() >= 1.4 - 1e-5 and h.max() <= 1.8 + 1e-5


def test_degenerate_stress_inputs_are_valid_polygons():
    a, b, names = synth.degenerate_stress()
    assert len(names) == a.shape[0] == b.shape[0]
    for i in range(a.shape[0]):
        assert _ccw_strict(a[i], 4) and _ccw_strict(b[i], 4), names[i]


def test_box_corner_convention():
    q = synth.boxes_to_quads([0.0], [0.0], [2.0], [4.0], [math.pi / 2])[0]
    # length 4 along the heading (+y), width 2 across; first corner (+l/2, -w/2)
    assert np.allclose(q, [[1, 2], [-1, 2], [-1, -2], [1, -2]], atol=1e-6)
