"""Pins of the simple-polygon (non-convex) oracle against facts other than
itself: exact rational areas by a signed fan of convex triangles, exact cell
counts of integer rectilinear shapes, the convex oracle on convex inputs,
symmetry, scaling, finite differences and the invariances of the gradient.

Sec. III keeps polygons convex and plans arbitrary polygons; the oracle
computes the plain definition (the area of the intersection region) by a
vertical slab decomposition, and its gradient by moving each vertex's two
edges where they lie inside the other polygon.
"""
import numpy as np

import exact_geom as X
import synth


def _fan(poly):
    """Signed fan of triangles (P_0, P_i, P_i+1), each made counter-clockwise,
    with its sign; zero-area triangles dropped.  The winding number of a
    closed polygon is the signed sum of the triangles' indicators."""
    out = []
    for i in range(1, len(poly) - 1):
        t = [poly[0], poly[i], poly[i + 1]]
        o = X.orient(*t)
        if o > 0:
            out.append((1, t))
        elif o < 0:
            out.append((-1, [t[0], t[2], t[1]]))
    return out


def _exact_inter_area(p, q):
    """Exact intersection area of two simple CCW polygons: the double signed
    sum of the areas of the fan triangles' pairwise (convex) intersections."""
    fp, fq = _fan(X.fpoly(p)), _fan(X.fpoly(q))
    tot = 0
    for sp, tp in fp:
        for sq, tq in fq:
            v = X.clip(tp, tq)
            if v:
                tot += sp * sq * X.area(v)
    return tot


def test_generated_polygons_are_simple(orc):
    d = synth.c4_simple(n=3000, seed=201)
    for key, nk in (("a_xy", "a_nv"), ("b_xy", "b_nv")):
        xy, nv = d[key], d[nk]
        assert all(orc.simple_valid(xy[i, :nv[i]]) for i in range(len(xy)))
    # about half are not convex
    conv = np.mean([orc.polygon_valid(d["a_xy"][i, :d["a_nv"][i]].astype(np.float64))
                    for i in range(3000)])
    assert 0.3 < conv < 0.7


def test_simple_validity_facts(orc):
    L = np.array([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]], float)
    assert orc.simple_valid(L)
    assert not orc.simple_valid(L[::-1].copy())                       # clockwise
    assert not orc.simple_valid(np.array([[0, 0], [1, 1], [1, 0], [0, 1]], float))  # bow tie
    assert not orc.simple_valid(np.array([[0, 0], [2, 0], [1, 0], [1, 1]], float))  # folds back
    assert orc.simple_valid(np.array([[0, 0], [1, 0], [2, 0], [1, 1]], float))      # straight vertex
    # status codes on fp32 rows: valid, edges meet / overlap, clockwise, count
    rows = [
        ([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]], 6, 0),            # L shape
        ([[0, 0], [0, 2], [1, 2], [1, 1], [2, 1], [2, 0]], 6, 3),            # L, clockwise
        ([[0, 0], [3, 0], [3, 2], [2, 2], [2, 1], [1, 1], [1, 2], [0, 2]], 8, 0),  # U: collinear top edges apart
        ([[0, 0], [1, 1], [1, 0], [0, 1]], 4, 2),                            # bow tie
        ([[0, 0], [2, 0], [1, 0], [1, 1]], 4, 2),                            # folds back
        ([[0, 0], [1, 0], [1, 0], [1, 1], [0, 1]], 5, 2),                    # repeated vertex
        ([[0, 0], [1, 0], [2, 0], [1, 1]], 4, 0),                            # straight vertex
        ([[0, 0], [2, 0], [2, 2], [1, 0.0], [0, 2]], 5, 2),                  # vertex on an edge
        ([[0, 0], [1, 0], [0, 1]], 2, 1),
        ([[0, 0], [1, 0], [0, 1]], 9, 1),
    ]
    xy = np.zeros((len(rows), 8, 2), np.float32)
    for r, (v, n, _) in enumerate(rows):
        xy[r, :len(v)] = v
    nv = np.array([r[1] for r in rows], np.uint8)
    assert list(orc.simple_status(xy, nv)) == [r[2] for r in rows]


def test_slab_area_exact_fan(orc):
    """Slab area against the exact rational fan decomposition."""
    d = synth.c4_simple(n=120, seed=202)
    worst = 0.0
    for i in range(120):
        p = d["a_xy"][i, :d["a_nv"][i]]
        q = d["b_xy"][i, :d["b_nv"][i]]
        ex = _exact_inter_area(p, q)
        got = orc.simple_inter_area(p.astype(np.float64), q.astype(np.float64))
        scale = max(1.0, float(X.area(X.fpoly(p))))
        worst = max(worst, abs(got - float(ex)) / scale)
    assert worst <= 1e-13, worst


def _rect_shapes(rng):
    """An integer rectilinear polygon: rectangle, L or U shape, CCW."""
    w, h = int(rng.integers(3, 8)), int(rng.integers(3, 8))
    kind = int(rng.integers(0, 3))
    if kind == 0:
        v = [(0, 0), (w, 0), (w, h), (0, h)]
    elif kind == 1:
        a, b = int(rng.integers(1, w)), int(rng.integers(1, h))
        v = [(0, 0), (w, 0), (w, b), (a, b), (a, h), (0, h)]
    else:
        a1 = int(rng.integers(1, w - 1))
        a2 = int(rng.integers(a1 + 1, w))
        b = int(rng.integers(1, h))
        v = [(0, 0), (w, 0), (w, h), (a2, h), (a2, b), (a1, b), (a1, h), (0, h)]
    v = np.array(v, float)
    for _ in range(int(rng.integers(0, 4))):  # quarter turns keep it CCW
        v = np.stack([-v[:, 1], v[:, 0]], 1)
    return v + rng.integers(-4, 5, 2)


def _cells_inside(v, xs, ys):
    """Crossing-number test of the cell centres (never on an integer edge)."""
    px, py = np.meshgrid(xs + 0.5, ys + 0.5)
    inside = np.zeros(px.shape, bool)
    n = len(v)
    for k in range(n):
        (ax, ay), (bx, by) = v[k], v[(k + 1) % n]
        if ay == by:
            continue
        cond = (ay > py) != (by > py)
        x = ax + (py - ay) * (bx - ax) / (by - ay)
        inside ^= cond & (x > px)
    return inside


def test_rectilinear_cell_count(orc):
    """Integer rectilinear shapes: the intersection is a union of unit cells,
    counted exactly; contacts along edges and at vertices included."""
    rng = np.random.default_rng(203)
    xs = np.arange(-20, 20)
    for _ in range(300):
        p, q = _rect_shapes(rng), _rect_shapes(rng)
        cells = int(np.count_nonzero(_cells_inside(p, xs, xs) & _cells_inside(q, xs, xs)))
        assert orc.simple_inter_area(p, q) == float(cells)


def _moved_state(p, q, eps):
    """Saved state of the pair with q moved by (eps, eps^2), eps a small
    exact rational: crossing and entering masks by strict sign tests of the
    exact orientations, vertex-0 inclusion by the crossing-number test on
    exact rationals (for small eps the moved pair has no contact)."""
    from fractions import Fraction
    P = X.fpoly(p)
    Q = [(x + eps, y + eps * eps) for x, y in X.fpoly(q)]
    n1, n2 = len(P), len(Q)

    def sgn(v):
        return (v > 0) - (v < 0)

    def inside(pt, V):
        c = 0
        for k in range(len(V)):
            (ax, ay), (bx, by) = V[k], V[(k + 1) % len(V)]
            if (ay > pt[1]) != (by > pt[1]):
                x = ax + (pt[1] - ay) * (bx - ax) / (by - ay)
                assert x != pt[0]
                c ^= int(x > pt[0])
        return c

    xm = sm = 0
    for i in range(n1):
        a, b = P[i], P[(i + 1) % n1]
        for j in range(n2):
            c, d = Q[j], Q[(j + 1) % n2]
            s1, s2 = sgn(X.orient(c, d, a)), sgn(X.orient(c, d, b))
            s3, s4 = sgn(X.orient(a, b, c)), sgn(X.orient(a, b, d))
            assert 0 not in (s1, s2, s3, s4)
            if s1 != s2 and s3 != s4:
                xm |= 1 << (8 * i + j)
                if s1 < 0:
                    sm |= 1 << (8 * i + j)
    return xm, sm, inside(P[0], Q) | (inside(Q[0], P) << 1)


def test_tie_rule_state_is_the_moved_pairs(orc):
    """Integer rectilinear shapes touch along edges and at vertices; the
    oracle's saved state (crossing / entering masks, vertex-0 inclusion) is
    that of the pair with q moved by (eps, eps^2): here eps = 2^-12, below
    every ratio of the integer orientations, so the moved pair's exact state
    equals the limit the tie rule names."""
    from fractions import Fraction
    rng = np.random.default_rng(207)
    eps = Fraction(1, 2 ** 12)
    contacts = 0
    for _ in range(300):
        p, q = _rect_shapes(rng), _rect_shapes(rng)
        a = np.zeros((1, 8, 2), np.float32)
        b = np.zeros((1, 8, 2), np.float32)
        a[0, :len(p)], b[0, :len(q)] = p, q
        an, bn = np.array([len(p)], np.uint8), np.array([len(q)], np.uint8)
        _, xm, sm, ins, bad = orc.simple_iou_pairs(a, b, an, bn)
        assert bad == 0
        r_xm, r_sm, r_ins = _moved_state(p, q, eps)
        assert (int(xm[0]), int(sm[0]), int(ins[0])) == (r_xm, r_sm, r_ins)
        P, Q = X.fpoly(p), X.fpoly(q)
        contacts += any(X.orient(Q[j], Q[(j + 1) % len(Q)], v) == 0
                        for v in P for j in range(len(Q)))
    assert contacts > 100  # the set is mostly degenerate


def test_convex_inputs_match_convex_oracle(orc):
    for d in (synth.c1_pairs(n=400, seed=204), synth.c4_polygons(n=400, seed=205)):
        a, b = d["a_xy"], d["b_xy"]
        an, bn = d.get("a_nv"), d.get("b_nv")
        ref, nx, xf, _ = orc.iou_pairs(a, b, an, bn)
        iou, xm, sm, ins, bad = orc.simple_iou_pairs(a, b, an, bn)
        assert bad == 0
        assert np.abs(iou - ref).max() <= 1e-12
        keep = orc.filtered_mask(orc.pair_margins(a, b, an, bn))
        for i in np.flatnonzero(keep):
            codes = [int(c) for c in xf[i, :nx[i]]]
            cross = sum(1 << (((c >> 3) & 7) * 8 + (c & 7)) for c in codes if c >= 0x40)
            assert int(xm[i]) == cross
            assert int(ins[i]) & 1 == int(0 in codes)
            assert (int(ins[i]) >> 1) & 1 == int(0x10 in codes)
            # an edge of a that enters b at a crossing carries the boundary of
            # the intersection on: the next vertex (counter-clockwise) lies on
            # the same edge of a (its end vertex or a later crossing of it)
            n1 = 4 if an is None else int(an[i])
            m = len(codes)
            for k, c in enumerate(codes):
                if c < 0x40:
                    continue
                e = (c >> 3) & 7
                nxt = codes[(k + 1) % m]
                on_a = nxt == (e + 1) % n1 or (nxt >= 0x40 and (nxt >> 3) & 7 == e)
                assert bool((int(sm[i]) >> (e * 8 + (c & 7))) & 1) == on_a


def test_degenerate_convex_pairs_match_convex_oracle(orc):
    """Exactly degenerate convex contacts (shared edges, a vertex on an edge,
    collinear overlaps, corner touches), both roles: the two oracles apply the
    same tie rule, so the crossing mask and vertex-0 inclusion follow from
    the convex oracle's codes on every pair."""
    a, b, names = synth.degenerate_stress()
    for p, q in ((a, b), (b, a)):
        _, nx, xf, _ = orc.iou_pairs(p, q)
        _, xm, _, ins, bad = orc.simple_iou_pairs(p, q)
        assert bad == 0
        for i in range(len(p)):
            codes = [int(c) for c in xf[i, :nx[i]]]
            cross = sum(1 << (((c >> 3) & 7) * 8 + (c & 7)) for c in codes if c >= 0x40)
            assert int(xm[i]) == cross, (names[i], hex(int(xm[i])), codes)
            assert int(ins[i]) & 1 == int(0 in codes), names[i]
            assert (int(ins[i]) >> 1) & 1 == int(0x10 in codes), names[i]


def test_symmetry_identity_scaling(orc):
    d = synth.c4_simple(n=200, seed=206)
    for i in range(200):
        p = d["a_xy"][i, :d["a_nv"][i]].astype(np.float64)
        q = d["b_xy"][i, :d["b_nv"][i]].astype(np.float64)
        assert abs(orc.simple_inter_area(p, q) - orc.simple_inter_area(q, p)) <= 1e-12
        ap = float(X.area(X.fpoly(p)))
        assert abs(orc.simple_inter_area(p, p) - ap) <= 1e-12 * max(1, ap)
        # disjoint after a far translation; a copy scaled by 1/2 meets
        # itself in a quarter of the area
        far = p + np.array([100.0, 0.0])
        assert orc.simple_inter_area(p, far) == 0.0
        half = 0.5 * p
        assert abs(orc.simple_inter_area(half, half) - ap / 4) <= 1e-12 * max(1, ap)


def test_gradient_finite_differences(orc):
    """Analytic gradient against central differences of the slab IoU
    (Richardson on steps h and h/2), on pairs far from any contact."""
    d = synth.c4_simple(n=400, seed=207)
    a, b, an, bn = d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"]
    marg = orc.simple_margins(a, b, an, bn)
    iou = orc.simple_iou_pairs(a, b, an, bn)[0]
    sel = np.flatnonzero((marg[:, 0] > 2e-3) & (marg[:, 1] > 1e-2) & (iou > 1e-3))[:60]
    assert len(sel) >= 40
    ga, gb = orc.simple_iou_pairs_grad(a[sel], b[sel], np.ones(len(sel)), an[sel], bn[sel])
    h = 2.0 ** -14
    worst = 0.0
    for r, i in enumerate(sel):
        p = a[i, :an[i]].astype(np.float64)
        q = b[i, :bn[i]].astype(np.float64)

        def f(pp, qq):
            return orc.simple_inter_area(pp, qq) / (
                abs(_shoelace(pp)) + abs(_shoelace(qq)) - orc.simple_inter_area(pp, qq))

        num = []
        for poly, which in ((p, 0), (q, 1)):
            for k in range(len(poly)):
                for c in range(2):
                    def at(step):
                        pp, qq = p.copy(), q.copy()
                        (pp if which == 0 else qq)[k, c] += step
                        return f(pp, qq)
                    d1 = (at(h) - at(-h)) / (2 * h)
                    d2 = (at(h / 2) - at(-h / 2)) / h
                    num.append((4 * d2 - d1) / 3)
        ana = np.concatenate([ga[r, :an[i]].ravel(), gb[r, :bn[i]].ravel()])
        num = np.array(num)
        worst = max(worst, np.linalg.norm(ana - num) / max(np.linalg.norm(num), 1e-8))
    assert worst <= 1e-6, worst


def _shoelace(v):
    x, y = v[:, 0], v[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def test_gradient_invariances(orc):
    """IoU is invariant under translation, rotation and scaling, so its
    gradient sums to zero, has no torque and no radial component."""
    d = synth.c4_simple(n=500, seed=208)
    a, b, an, bn = d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"]
    keep = orc.simple_filtered_mask(orc.simple_margins(a, b, an, bn))
    ga, gb = orc.simple_iou_pairs_grad(a, b, np.ones(len(a)), an, bn)
    v = np.concatenate([a, b], 1).astype(np.float64)
    g = np.concatenate([ga, gb], 1)
    scale = np.abs(g).sum((1, 2)) + 1e-30
    assert np.max(np.abs(g.sum(1)).max(1)[keep] / scale[keep]) <= 1e-12
    torque = (v[:, :, 0] * g[:, :, 1] - v[:, :, 1] * g[:, :, 0]).sum(1)
    radial = (v * g).sum((1, 2))
    vs = np.abs(v).max((1, 2)) * scale
    assert np.max(np.abs(torque)[keep] / vs[keep]) <= 1e-12
    assert np.max(np.abs(radial)[keep] / vs[keep]) <= 1e-12
