"""Pins of the FP64 oracle against things other than itself: exact rational
geometry, closed forms, invariances, rasterised area and finite differences.

The IoU of convex polygons is the ratio of true areas (Sec. II-B listing), so
its exact value on the (exactly representable) fp32 inputs is computable in
rationals; the provenance flags (Sec. II-B, encoded as the oracle's header
states) name exact points; the gradient is that of the IoU function, which
central differences approximate.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import exact_geom as X
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.jsonl")


def _filtered(orc, a, b, a_nv=None, b_nv=None):
    return orc.filtered_mask(orc.pair_margins(a, b, a_nv, b_nv))


def _exact_pair_check(orc, p, q):
    """Oracle intersection of one generic pair against exact rationals."""
    P, Q = X.fpoly(p), X.fpoly(q)
    V = X.clip(P, Q)
    verts, codes = orc.intersect(p, q)
    assert len(codes) == len(V), (len(codes), len(V))
    if not V:
        return
    assert int(codes[0]) == int(codes.min()), "sequence must start at the smallest code"
    assert len(set(codes.tolist())) == len(codes)
    ex = [X.vertex_from_code(P, Q, int(c)) for c in codes]
    # every code names a vertex of the exact intersection, and only that code does
    assert set(ex) == set(V)
    for c, v in zip(codes, ex):
        assert X.classify(P, Q, v) == {int(c)}
    # the oracle's fp64 vertices are the exact ones
    scale = max(1.0, float(np.abs(p).max()), float(np.abs(q).max()))
    for k, v in enumerate(ex):
        assert abs(verts[k, 0] - float(v[0])) <= 1e-13 * scale
        assert abs(verts[k, 1] - float(v[1])) <= 1e-13 * scale
    # counter-clockwise and the same cyclic sequence as the exact clip
    m = len(ex)
    for k in range(m):
        assert X.orient(ex[k], ex[(k + 1) % m], ex[(k + 2) % m]) > 0
    s = V.index(ex[0])
    assert V[s:] + V[:s] == ex
    # area
    ai = X.area(V)
    assert abs(orc.area(verts) - float(ai)) <= 1e-13 * max(1.0, float(ai))
    a1, a2 = X.area(P), X.area(Q)
    iou_exact = ai / (a1 + a2 - ai)
    return iou_exact


def _pair_sets():
    sets = []
    d = synth.c1_pairs(n=160, seed=11)
    sets.append((d["a_xy"], d["b_xy"], None, None))
    d = synth.c3_pairs(n=160, seed=12)
    sets.append((d["a_xy"], d["b_xy"], None, None))
    d = synth.c4_polygons(n=200, seed=13)
    sets.append((d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"]))
    return sets


def test_exact_rational_intersections(orc):
    checked = 0
    for a, b, anv, bnv in _pair_sets():
        keep = _filtered(orc, a, b, anv, bnv)
        iou, nx, xf, bad = orc.iou_pairs(a, b, anv, bnv)
        assert bad == 0
        for i in np.nonzero(keep)[0]:
            n1 = int(anv[i]) if anv is not None else a.shape[1]
            n2 = int(bnv[i]) if bnv is not None else b.shape[1]
            iou_ex = _exact_pair_check(orc, a[i, :n1].astype(np.float64),
                                       b[i, :n2].astype(np.float64))
            if iou_ex is None:
                assert nx[i] == 0 and iou[i] == 0.0
            else:
                assert abs(iou[i] - float(iou_ex)) <= 1e-13
            checked += 1
    assert checked > 400


def test_clip_crosscheck_all_inputs(orc):
    """Sutherland-Hodgman (a different algorithm) agrees on every input,
    degenerate ones included."""
    sets = _pair_sets()
    sa, sb, _ = synth.degenerate_stress()
    sets.append((sa, sb, None, None))
    for a, b, anv, bnv in sets:
        iou, nx, xf, bad = orc.iou_pairs(a, b, anv, bnv)
        for i in range(a.shape[0]):
            n1 = int(anv[i]) if anv is not None else a.shape[1]
            n2 = int(bnv[i]) if bnv is not None else b.shape[1]
            p, q = a[i, :n1].astype(np.float64), b[i, :n2].astype(np.float64)
            ci = orc.clip_area(p, q)
            if nx[i] == 0:
                assert abs(ci) <= 1e-12
                continue
            verts, _ = orc.intersect(p, q)
            assert abs(orc.area(verts) - ci) <= 1e-12 * max(1.0, abs(ci))
            a1, a2 = orc.area(p), orc.area(q)
            assert abs(iou[i] - ci / (a1 + a2 - ci)) <= 1e-12


def test_golden_closed_forms(orc):
    for line in open(GOLDEN):
        c = json.loads(line)
        P = np.array(c["P"], np.float64)
        Q = np.array(c["Q"], np.float64)
        # the stored fractions agree with the stated closed form
        I, A1, A2 = Fraction(c["I"]), Fraction(c["A1"]), Fraction(c["A2"])
        exp = Fraction(0) if I == 0 else I / (A1 + A2 - I)
        assert exp == Fraction(c["iou"]), c["name"]
        assert X.area(X.fpoly(P)) == A1 and X.area(X.fpoly(Q)) == A2
        # oracle
        k = max(P.shape[0], Q.shape[0])
        a = np.zeros((1, k, 2), np.float32)
        b = np.zeros((1, k, 2), np.float32)
        a[0, :P.shape[0]] = P
        b[0, :Q.shape[0]] = Q
        anv = np.array([P.shape[0]], np.uint8)
        bnv = np.array([Q.shape[0]], np.uint8)
        iou, nx, xf, bad = orc.iou_pairs(a, b, anv, bnv)
        assert abs(iou[0] - float(exp)) <= 1e-15, c["name"]
        if not c["degenerate"]:
            assert int(nx[0]) == c["nx"], c["name"]
            assert xf[0, :nx[0]].tolist() == c["flags"], c["name"]
            assert np.all(xf[0, nx[0]:] == 0xFF)


def _aabb(x0, y0, x1, y1):
    return np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]], np.float32)


def test_closed_form_axis_aligned(orc):
    rng = np.random.default_rng(5)
    n = 400
    lo = rng.integers(-32, 32, (n, 2, 2)) / 8.0          # dyadic: exact in fp32
    size = rng.integers(1, 24, (n, 2, 2)) / 8.0
    hi = lo + size
    a = np.stack([_aabb(lo[i, 0, 0], lo[i, 0, 1], hi[i, 0, 0], hi[i, 0, 1]) for i in range(n)])
    b = np.stack([_aabb(lo[i, 1, 0], lo[i, 1, 1], hi[i, 1, 0], hi[i, 1, 1]) for i in range(n)])
    iou, nx, xf, bad = orc.iou_pairs(a, b)
    for i in range(n):
        wx = min(hi[i, 0, 0], hi[i, 1, 0]) - max(lo[i, 0, 0], lo[i, 1, 0])
        wy = min(hi[i, 0, 1], hi[i, 1, 1]) - max(lo[i, 0, 1], lo[i, 1, 1])
        inter = max(0.0, wx) * max(0.0, wy)
        a1 = size[i, 0, 0] * size[i, 0, 1]
        a2 = size[i, 1, 0] * size[i, 1, 1]
        exp = inter / (a1 + a2 - inter)
        assert abs(iou[i] - exp) <= 1e-14, (i, iou[i], exp)


def _square(theta, half=1.0):
    c, s = math.cos(theta), math.sin(theta)
    base = [(half, -half), (half, half), (-half, half), (-half, -half)]
    return np.array([[c * x - s * y, s * x + c * y] for x, y in base], np.float64)


def _rot_squares_closed(theta):
    """Concentric squares of half-size 1 at relative angle theta in (0, pi/2):
    each of the 8 corners cut off is a right triangle with legs a, b below."""
    a = 1.0 - math.tan(theta / 2)
    b = 1.0 - math.tan(math.pi / 4 - theta / 2)
    inter = 4.0 - 2.0 * a * b
    da = -0.5 / math.cos(theta / 2) ** 2
    db = 0.5 / math.cos(math.pi / 4 - theta / 2) ** 2
    dinter = -2.0 * (da * b + a * db)
    return inter, dinter


def test_closed_form_rotated_squares(orc):
    thetas = np.linspace(0.05, math.pi / 2 - 0.05, 23)
    a = np.stack([_square(0.0)] * len(thetas))
    b = np.stack([_square(t) for t in thetas])
    iou, nx, xf = orc.iou_pairs_f64(a, b)
    ga, gb, _, _ = orc.iou_pairs_grad_f64(a, b, np.ones(len(thetas)), nx, xf)
    for k, t in enumerate(thetas):
        inter, dinter = _rot_squares_closed(t)
        assert nx[k] == 8
        assert all(c >= 0x40 for c in xf[k])          # only crossings
        assert abs(iou[k] - inter / (8.0 - inter)) <= 1e-13
        # d IoU / d theta through the rotation field (-y, x) applied to Q
        dq = np.stack([-b[k, :, 1], b[k, :, 0]], axis=-1)
        dIoU = float((gb[k] * dq).sum())
        exp = 8.0 / (8.0 - inter) ** 2 * dinter
        assert abs(dIoU - exp) <= 1e-11, (t, dIoU, exp)
    # at 45 degrees: 1/sqrt(2) and a stationary intersection area
    iou45, nx45, xf45 = orc.iou_pairs_f64(_square(0.0)[None], _square(math.pi / 4)[None])
    assert abs(iou45[0] - 1 / math.sqrt(2)) <= 1e-14 and nx45[0] == 8


def _moved_codes(p, q, eps):
    """Codes of the intersection of p with q moved by (eps, eps^2), eps a
    small exact rational: P_i strictly inside the moved q, Q_j (moved)
    strictly inside p, and the proper crossings of their edges."""
    P = X.fpoly(p)
    Q = [(x + eps, y + eps * eps) for x, y in X.fpoly(q)]
    n1, n2 = len(P), len(Q)
    codes = set()
    for i in range(n1):
        if all(X.orient(Q[j], Q[(j + 1) % n2], P[i]) > 0 for j in range(n2)):
            codes.add(i)
    for j in range(n2):
        if all(X.orient(P[i], P[(i + 1) % n1], Q[j]) > 0 for i in range(n1)):
            codes.add(0x10 | j)
    for i in range(n1):
        a, b = P[i], P[(i + 1) % n1]
        for j in range(n2):
            c, d = Q[j], Q[(j + 1) % n2]
            o = [X.orient(c, d, a), X.orient(c, d, b), X.orient(a, b, c), X.orient(a, b, d)]
            assert all(v != 0 for v in o)  # the moved pair has no contact
            if (o[0] > 0) != (o[1] > 0) and (o[2] > 0) != (o[3] > 0):
                codes.add(0x40 | (i << 3) | j)
    return codes


def test_near_identical_boxes_exact(orc):
    """Boxes within about an ulp of each other: edges that are nearly parallel
    and share an end (angles down to ~1e-12) still give the exact IoU, never
    above 1, on every pair (exact rational clipping of the same fp32 inputs).
    Placing such a crossing by the meet of the two lines' coefficients in fp64
    was ~1e-4 off here."""
    checked = 0
    for sig in (1e-7, 1e-6):
        d = synth.c1_pairs(n=150, seed=5000, center_sigma=sig, yaw_sigma=sig)
        a, b = d["a_xy"], d["b_xy"]
        iou, nx, xf, bad = orc.iou_pairs(a, b)
        assert bad == 0 and np.all(iou <= 1.0)
        for i in range(len(a)):
            P, Q = X.fpoly(a[i]), X.fpoly(b[i])
            inter = X.clip(P, Q)
            ia = X.area(inter) if len(inter) >= 3 else 0
            ex = ia / (X.area(P) + X.area(Q) - ia)
            assert abs(iou[i] - float(ex)) <= 1e-12, (sig, i, iou[i], float(ex))
            checked += 1
    assert checked == 300


def test_tie_rule_codes_are_the_moved_pairs(orc):
    """Exact contacts (shared and collinear edges, vertices on edges, corner
    touches, identical polygons): the oracle's vertex count and set of codes
    are those of the pair with b moved by (eps, eps^2) (eps = 2^-12, below
    every ratio of these small dyadic orientations), computed in exact
    rationals (the order is pinned by the sequence test below)."""
    from fractions import Fraction
    eps = Fraction(1, 2 ** 12)
    sa, sb, _ = synth.degenerate_stress()
    rng = np.random.default_rng(26)
    # integer rectangles and diamonds on a small grid: contacts are common
    shapes = []
    for _ in range(400):
        x0, y0 = rng.integers(-3, 3, 2)
        w, h = rng.integers(1, 4, 2)
        if rng.integers(0, 2):
            v = [(x0, y0), (x0 + w, y0), (x0 + w, y0 + h), (x0, y0 + h)]
        else:
            v = [(x0 + w, y0), (x0, y0 + w), (x0 - w, y0), (x0, y0 - w)]
        shapes.append(v)
    ga = np.array(shapes[:200], np.float32)
    gb = np.array(shapes[200:], np.float32)
    checked = contacts = 0
    for a, b in ((sa, sb), (sb, sa), (ga, gb), (gb, ga)):
        _, nx, xf, bad = orc.iou_pairs(a, b)
        assert bad == 0
        for i in range(len(a)):
            want = _moved_codes(a[i].astype(np.float64), b[i].astype(np.float64), eps)
            got = [int(c) for c in xf[i, :nx[i]]]
            assert len(got) == len(set(got)) and set(got) == want, (i, got, sorted(want))
            P, Q = X.fpoly(a[i]), X.fpoly(b[i])
            contacts += any(X.orient(Q[j], Q[(j + 1) % 4], v) == 0 for v in P for j in range(4))
            checked += 1
    assert checked == 2 * len(sa) + 400 and contacts > 100


def _moved(q, eps):
    return [(x + eps, y + eps * eps) for x, y in q]


def _moved_sequence(P, Q, eps):
    """Codes of the intersection of P with Q moved by (eps, eps^2), in the
    counter-clockwise order of exact rational Sutherland-Hodgman clipping,
    rotated to start at the smallest code (empty: [])."""
    Qm = _moved(Q, eps)
    poly = X.clip(P, Qm)
    if len(poly) < 3:
        return []
    seq = []
    for v in poly:
        c = X.classify(P, Qm, v)
        assert len(c) == 1, c  # the moved pair is generic: one name per point
        seq.append(c.pop())
    k = seq.index(min(seq))
    return seq[k:] + seq[:k]


def _contact_pairs(seed, n):
    """Integer rectangles and diamonds on a small grid (exact contacts are
    common), as pairs (a [n,4,2], b [n,4,2])."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(2 * n):
        x0, y0 = rng.integers(-3, 3, 2)
        w, h = rng.integers(1, 4, 2)
        if rng.integers(0, 2):
            v = [(x0, y0), (x0 + w, y0), (x0 + w, y0 + h), (x0, y0 + h)]
        else:
            v = [(x0 + w, y0), (x0, y0 + w), (x0 - w, y0), (x0, y0 - w)]
        shapes.append(v)
    s = np.array(shapes, np.float32)
    return s[:n], s[n:]


def test_tie_rule_sequences_are_the_moved_pairs(orc):
    """Reading R2 on exact contacts: the whole flag sequence, not only its set
    of codes, is the counter-clockwise boundary of the pair moved by the tie
    rule, taken from exact rational clipping of the moved pair (eps = 2^-12).
    Where points coincide (a vertex on an edge, touching boxes, duplicates)
    an order by angle about a centre cannot tell them apart; ordering such
    ties by code reverses, for instance, the zero-area intersection of two
    boxes that share part of an edge."""
    eps = Fraction(1, 2 ** 12)
    sa, sb, _ = synth.degenerate_stress()
    ga, gb = _contact_pairs(27, 300)
    checked = coincident = 0
    for a, b in ((sa, sb), (sb, sa), (ga, gb), (gb, ga)):
        _, nx, xf, bad = orc.iou_pairs(a, b)
        assert bad == 0
        for i in range(len(a)):
            P, Q = X.fpoly(a[i]), X.fpoly(b[i])
            want = _moved_sequence(P, Q, eps)
            got = [int(c) for c in xf[i, :nx[i]]]
            assert got == want, (i, [hex(c) for c in got], [hex(c) for c in want])
            pts = [X.vertex_from_code(P, Q, c) for c in got]
            coincident += len(set(pts)) < len(pts)
            checked += 1
    assert checked == 2 * len(sa) + 600 and coincident > 50, (checked, coincident)


def _exact_iou(P, Q):
    inter = X.clip(P, Q)
    ai = X.area(inter) if len(inter) >= 3 else Fraction(0)
    return ai / (X.area(P) + X.area(Q) - ai)


def test_tie_rule_gradients_are_the_moved_pairs(orc):
    """Reading R9 on exact contacts: the gradient the oracle takes from its
    flags is the one-sided gradient in the direction of the tie rule, i.e.
    the limit of the gradient of the moved pair.  Reference: exact rational
    central differences of the exact IoU of the pair moved by eps = 2^-16,
    with steps of 2^-44 (far below the eps^2 = 2^-32 separation of its
    contacts, so the moved pair keeps its structure); the two differ by
    O(eps).  Touching pairs (zero area, non-zero one-sided gradient) are
    among them."""
    eps = Fraction(1, 2 ** 16)
    h = Fraction(1, 2 ** 44)
    sa, sb, _ = synth.degenerate_stress()
    ga, gb = _contact_pairs(28, 40)
    a = np.concatenate([sa, ga])
    b = np.concatenate([sb, gb])
    g = np.ones(len(a))
    _, nx, xf, _ = orc.iou_pairs(a, b)
    oa, ob, _, _ = orc.iou_pairs_grad(a, b, g, nx, xf)
    worst = 0.0
    touching = 0
    for i in range(len(a)):
        P, Q = X.fpoly(a[i]), _moved(X.fpoly(b[i]), eps)
        ref = np.zeros((2, 4, 2))
        for side in range(2):
            for k in range(4):
                for d in range(2):
                    def shifted(s):
                        pp, qq = [list(v) for v in P], [list(v) for v in Q]
                        (pp if side == 0 else qq)[k][d] += s
                        return _exact_iou([tuple(v) for v in pp], [tuple(v) for v in qq])
                    ref[side, k, d] = float((shifted(h) - shifted(-h)) / (2 * h))
        got = np.stack([oa[i], ob[i]])
        err = np.abs(got - ref).max()
        worst = max(worst, err)
        assert err <= 1e-3 * (1.0 + np.abs(ref).max()), (i, got, ref)
        touching += nx[i] >= 3 and _exact_iou(X.fpoly(a[i]), X.fpoly(b[i])) == 0
    assert touching >= 3, touching


def _exact_iou3(P, Q, z1, z2):
    """Exact 3D IoU: BEV intersection area times the z-overlap, over the
    union volume."""
    inter = X.clip(P, Q)
    ai = X.area(inter) if len(inter) >= 3 else Fraction(0)
    hz = max(Fraction(0), min(z1[1], z2[1]) - max(z1[0], z2[0]))
    v = ai * hz
    return v / (X.area(P) * (z1[1] - z1[0]) + X.area(Q) * (z2[1] - z2[0]) - v)


def test_z_tie_gradients_are_the_moved_pairs(orc):
    """Reading R9 on z-extent ties (boxes on a common ground plane, equal
    tops, equal extents): the oracle gives the overlap's derivative to the
    first box's end, which is the gradient of the pair with the second box's
    ends moved outward by eps (lower end down, upper end up), so that the
    first box's ends bind the overlap.  Reference: exact rational central
    differences (steps 2^-40) of the exact 3D IoU of the moved pair (eps =
    2^-20), on axis-aligned rectangles with dyadic corners (exact areas);
    the two differ by O(eps).  A plain one-sided difference of the tied pair
    would pick a side per end; this one fixes which."""
    eps = Fraction(1, 2 ** 20)
    h = Fraction(1, 2 ** 40)
    rng = np.random.default_rng(91)
    zsets = [((0.5, 2.0), (0.5, 1.5)),    # common lower end
             ((0.5, 2.0), (0.25, 2.0)),   # common upper end
             ((0.5, 1.75), (0.5, 1.75)),  # equal extents
             ((-1.0, 0.5), (-1.0, 2.5))]
    rows = []
    for zi, (z1, z2) in enumerate(zsets):
        for k in range(5):
            x0, y0 = (rng.integers(-8, 8, 2) / 4.0)
            w, l = rng.integers(4, 12, 2) / 4.0
            dx, dy = rng.integers(1, 6, 2) / 8.0  # partial BEV overlap, no BEV ties
            a = [(x0, y0), (x0 + w, y0), (x0 + w, y0 + l), (x0, y0 + l)]
            b = [(x0 + dx, y0 + dy), (x0 + dx + w, y0 + dy), (x0 + dx + w, y0 + dy + l),
                 (x0 + dx, y0 + dy + l)]
            rows.append((a, b, z1, z2))
    a = np.array([r[0] for r in rows], np.float32)
    b = np.array([r[1] for r in rows], np.float32)
    za = tuple(np.array([r[2][i] for r in rows], np.float32) for i in range(2))
    zb = tuple(np.array([r[3][i] for r in rows], np.float32) for i in range(2))
    g = np.ones(len(rows))
    iou, nx, xf, _ = orc.iou_pairs(a, b, a_z=za, b_z=zb)
    _, _, gaz, gbz = orc.iou_pairs_grad(a, b, g, nx, xf, a_z=za, b_z=zb)
    for i, (pa, pb, z1, z2) in enumerate(rows):
        P, Q = [tuple(map(Fraction, v)) for v in pa], [tuple(map(Fraction, v)) for v in pb]
        f1 = [Fraction(z1[0]), Fraction(z1[1])]
        f2 = [Fraction(z2[0]) - eps, Fraction(z2[1]) + eps]  # the second box moved outward
        assert abs(iou[i] - float(_exact_iou3(P, Q, [Fraction(v) for v in z1],
                                              [Fraction(v) for v in z2]))) <= 1e-12
        ref = np.zeros((2, 2))
        for side, zz in ((0, f1), (1, f2)):
            for e in range(2):
                def shifted(s):
                    za_, zb_ = list(f1), list(f2)
                    (za_ if side == 0 else zb_)[e] += s
                    return _exact_iou3(P, Q, za_, zb_)
                ref[side, e] = float((shifted(h) - shifted(-h)) / (2 * h))
        got = np.stack([gaz[i], gbz[i]])
        assert np.abs(got - ref).max() <= 1e-4 * (1.0 + np.abs(ref).max()), (i, got, ref)


def test_zero_union_volume(orc):
    """Reading R5 (a union of measure zero gives IoU 0 and gradient 0) on the
    valid input that reaches it: flat 3D boxes (zlo == zhi) whose BEV
    rectangles overlap, where the quotient would be 0 / 0.  The same boxes
    with a positive height give the exact 3D IoU (identical boxes: 1, the
    closed form) and finite gradients; flat, they give exactly 0 and an
    all-zero gradient, never NaN.  A guard dropped from either the forward
    or the backward shows up here as NaN."""
    rng = np.random.default_rng(57)
    rows = []
    for k in range(10):
        x0, y0 = rng.integers(-8, 8, 2) / 4.0
        w, l = rng.integers(4, 12, 2) / 4.0
        dx, dy = (rng.integers(1, 6, 2) / 8.0) if k % 2 else (0.0, 0.0)  # odd: partial overlap
        a = [(x0, y0), (x0 + w, y0), (x0 + w, y0 + l), (x0, y0 + l)]
        b = [(x0 + dx, y0 + dy), (x0 + dx + w, y0 + dy), (x0 + dx + w, y0 + dy + l),
             (x0 + dx, y0 + dy + l)]
        rows.append((a, b))
    a = np.array([r[0] for r in rows], np.float32)
    b = np.array([r[1] for r in rows], np.float32)
    z0 = (rng.integers(-4, 4, len(rows)) / 4.0).astype(np.float32)
    same = np.arange(len(rows)) % 2 == 0
    for height in (0.0, 0.5, 2.0):
        z = (z0, (z0 + np.float32(height)).astype(np.float32))
        iou, nx, xf, _ = orc.iou_pairs(a, b, a_z=z, b_z=z)
        ga, gb, gaz, gbz = orc.iou_pairs_grad(a, b, np.ones(len(rows)), nx, xf, a_z=z, b_z=z)
        assert (nx >= 3).all()  # every BEV intersection is non-empty
        grads = np.concatenate([ga.ravel(), gb.ravel(), gaz.ravel(), gbz.ravel()])
        assert np.isfinite(iou).all() and np.isfinite(grads).all(), height
        if height == 0.0:
            assert (iou == 0.0).all() and (grads == 0.0).all()
            continue
        assert np.abs(iou[same] - 1.0).max() <= 1e-12
        for i in np.nonzero(~same)[0]:
            P = [tuple(map(Fraction, v)) for v in rows[i][0]]
            Q = [tuple(map(Fraction, v)) for v in rows[i][1]]
            zz = [Fraction(float(z[0][i])), Fraction(float(z[1][i]))]
            assert abs(iou[i] - float(_exact_iou3(P, Q, zz, zz))) <= 1e-12
        assert np.abs(grads).max() > 0


def test_identity_disjoint_nested(orc):
    d = synth.c4_polygons(n=300, seed=21)
    a, anv = d["a_xy"], d["a_nv"]
    iou, nx, xf, bad = orc.iou_pairs(a, a, anv, anv)
    # identical polygons resolve (tie rule) into crossings of adjacent edges at
    # the shared vertices, each placed at an end of its edge (t = 0 or 1)
    assert np.all(np.abs(iou - 1.0) <= 1e-12)
    # disjoint: shift far away
    b = a.copy()
    b[..., 0] += 100.0
    iou, nx, xf, _ = orc.iou_pairs(a, b, anv, anv)
    assert np.all(iou == 0) and np.all(nx == 0) and np.all(xf == 0xFF)
    # nested: shrink about an interior point (the vertex mean) by 1/2 (exact)
    c = np.zeros_like(a)
    for i in range(a.shape[0]):
        n = int(anv[i])
        m = a[i, :n].astype(np.float64).mean(axis=0)
        m = np.round(m * 64) / 64          # dyadic centre keeps the scaling exact-ish
        c[i, :n] = (m + 0.5 * (a[i, :n] - m)).astype(np.float32)
    iou, nx, xf, _ = orc.iou_pairs(a, c, anv, anv)
    for i in range(a.shape[0]):
        n = int(anv[i])
        inside = all(orc.polygon_valid(c[i, :n]) for _ in [0])
        if not inside:
            continue
        P, Q = X.fpoly(a[i], n), X.fpoly(c[i], n)
        if not all(X.orient(P[j], P[(j + 1) % n], q) > 0 for q in Q for j in range(n)):
            continue
        assert nx[i] == n and xf[i, :n].tolist() == [0x10 | j for j in range(n)]
        assert abs(iou[i] - float(X.area(Q) / X.area(P))) <= 1e-13


def test_symmetry_and_rigid_motion(orc):
    d = synth.c1_pairs(n=500, seed=31)
    a, b = d["a_xy"], d["b_xy"]
    iou, nx, xf, _ = orc.iou_pairs(a, b)
    iou_t, nx_t, _, _ = orc.iou_pairs(b, a)
    assert np.all(nx == nx_t)
    assert np.max(np.abs(iou - iou_t)) <= 1e-14
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    t = np.array([13.25, -7.5])
    iou_m, nx_m, _ = orc.iou_pairs_f64(a64 @ R.T + t, b64 @ R.T + t)
    iou0, nx0, _ = orc.iou_pairs_f64(a64, b64)
    assert np.max(np.abs(iou_m - iou0)) <= 1e-12
    assert np.all(nx_m == nx0)


def test_power_of_two_scaling_is_exact(orc):
    d = synth.c4_polygons(n=400, seed=41)
    a, b, anv, bnv, g = d["a_xy"], d["b_xy"], d["a_nv"], d["b_nv"], d["grad"]
    iou, nx, xf, _ = orc.iou_pairs(a, b, anv, bnv)
    ga, gb, _, _ = orc.iou_pairs_grad(a, b, g, nx, xf, anv, bnv)
    for k in (-3, 5):
        s = np.float32(2.0 ** k)
        iou_s, nx_s, xf_s, _ = orc.iou_pairs(a * s, b * s, anv, bnv)
        assert np.array_equal(iou_s, iou) and np.array_equal(nx_s, nx) and np.array_equal(xf_s, xf)
        ga_s, gb_s, _, _ = orc.iou_pairs_grad(a * s, b * s, g, nx_s, xf_s, anv, bnv)
        assert np.array_equal(ga_s, ga * 2.0 ** -k) and np.array_equal(gb_s, gb * 2.0 ** -k)


def _inside(poly, pts):
    n = poly.shape[0]
    ok = np.ones(pts.shape[0], bool)
    for k in range(n):
        a, b = poly[k], poly[(k + 1) % n]
        ok &= (b[0] - a[0]) * (pts[:, 1] - a[1]) - (b[1] - a[1]) * (pts[:, 0] - a[0]) >= 0
    return ok


def test_rasterised_area(orc):
    d = synth.c1_pairs(n=12, seed=51)
    a, b = d["a_xy"].astype(np.float64), d["b_xy"].astype(np.float64)
    iou, nx, xf, _ = orc.iou_pairs(d["a_xy"], d["b_xy"])
    h = 0.004
    for i in range(a.shape[0]):
        lo = np.minimum(a[i].min(0), b[i].min(0))
        hi = np.maximum(a[i].max(0), b[i].max(0))
        xs = np.arange(lo[0] + h / 2, hi[0], h)
        ys = np.arange(lo[1] + h / 2, hi[1], h)
        gx, gy = np.meshgrid(xs, ys)
        pts = np.stack([gx.ravel(), gy.ravel()], -1)
        est = np.count_nonzero(_inside(a[i], pts) & _inside(b[i], pts)) * h * h
        verts, _ = orc.intersect(a[i], b[i])
        ai = orc.area(verts) if len(verts) else 0.0
        per = sum(np.hypot(*(p[(k + 1) % 4] - p[k])) for p in (a[i], b[i]) for k in range(4))
        assert abs(ai - est) <= 2.0 * per * h, (i, ai, est)


# ---------------------------------------------------------------- gradient

def _fd_grads(orc, a, b, az, bz, h, nx, xf, keep):
    n, ka = a.shape[:2]
    kb = b.shape[1]
    coords = [("a", k, c) for k in range(ka) for c in range(2)] + \
             [("b", k, c) for k in range(kb) for c in range(2)]
    if az is not None:
        coords += [("az", 0, c) for c in range(2)] + [("bz", 0, c) for c in range(2)]
    cols = []
    for which, k, c in coords:
        vals = []
        for sgn in (1.0, -1.0):
            aa, bb = a.copy(), b.copy()
            zz1 = None if az is None else az.copy()
            zz2 = None if bz is None else bz.copy()
            if which == "a":
                aa[:, k, c] += sgn * h
            elif which == "b":
                bb[:, k, c] += sgn * h
            elif which == "az":
                zz1[:, c] += sgn * h
            else:
                zz2[:, c] += sgn * h
            v, nx_p, xf_p = orc.iou_pairs_f64(aa, bb, zz1, zz2)
            keep &= (nx_p == nx) & np.all(xf_p == xf, axis=1)
            vals.append(v)
        cols.append((vals[0] - vals[1]) / (2 * h))
    return np.stack(cols, 1)


def _fd_check(orc, a, b, az=None, bz=None, h=1e-3):
    """Central differences of IoU in fp64 (step h, and h/2 for a Richardson
    step that cancels the O(h^2) truncation term) vs the analytic gradient, on
    pairs whose nx and flags do not change at +-h, +-h/2 in any coordinate.
    Returns per-pair relative errors (plain, extrapolated) and the mask."""
    n = a.shape[0]
    iou, nx, xf = orc.iou_pairs_f64(a, b, az, bz)
    ga, gb, gaz, gbz = orc.iou_pairs_grad_f64(a, b, np.ones(n), nx, xf, az, bz)
    keep = nx > 0
    if az is not None:
        # the z-overlap min(hi) - max(lo) has kinks where the extents' ends
        # coincide or the overlap closes: keep pairs at least 2h away from them
        hz = np.minimum(az[:, 1], bz[:, 1]) - np.maximum(az[:, 0], bz[:, 0])
        keep &= (np.abs(az[:, 1] - bz[:, 1]) > 2 * h) & (np.abs(az[:, 0] - bz[:, 0]) > 2 * h)
        keep &= hz > 2 * h
    fd1 = _fd_grads(orc, a, b, az, bz, h, nx, xf, keep)
    fd2 = _fd_grads(orc, a, b, az, bz, h / 2, nx, xf, keep)
    fdr = (4.0 * fd2 - fd1) / 3.0
    an = np.concatenate([ga.reshape(n, -1), gb.reshape(n, -1)], 1)
    if az is not None:
        an = np.concatenate([an, gaz, gbz], 1)
    den = np.maximum(np.linalg.norm(an, axis=1), 1e-8)
    e1 = np.linalg.norm(an - fd1, axis=1) / den
    er = np.linalg.norm(an - fdr, axis=1) / den
    return e1[keep], er[keep], keep


def _check_fd(orc, a, b, az=None, bz=None, a_f32=None, b_f32=None):
    e1, er, keep = _fd_check(orc, a, b, az, bz)
    # extrapolated differences: truncation O(h^4), agreement to 1e-5 everywhere
    assert er.max() <= 1e-5, np.sort(er)[-5:]
    # plain h = 1e-3 differences: the truncation term grows like 1/sin^3 of the
    # crossing angle and like 1/size of the intersection, so 1e-4 is asserted
    # where every crossing has |sin| >= 0.1, every vertex is >= 1e-2 L from
    # every edge line and the IoU is >= 1e-2 (the intersection is >> h)
    if a_f32 is not None:
        m = orc.pair_margins(a_f32, b_f32)[keep]
        iou, _, _ = orc.iou_pairs_f64(a, b, az, bz)
        good = (m[:, 1] >= 0.1) & (m[:, 0] >= 1e-2) & (iou[keep] >= 1e-2)
        assert e1[good].max() <= 1e-4, np.sort(e1[good])[-5:]
    return keep


def test_gradient_vs_finite_differences_rectangles(orc):
    d = synth.c3_pairs(n=4096, seed=61)
    a, b = d["a_xy"].astype(np.float64), d["b_xy"].astype(np.float64)
    keep = _check_fd(orc, a, b, a_f32=d["a_xy"], b_f32=d["b_xy"])
    assert keep.sum() > 3000


def test_gradient_vs_finite_differences_polygons(orc):
    d = synth.c4_polygons(n=3000, seed=62)
    checked = 0
    for n1 in range(3, 9):
        for n2 in (3, 5, 8):
            sel = (d["a_nv"] == n1) & (d["b_nv"] == n2)
            if sel.sum() == 0:
                continue
            a = d["a_xy"][sel, :n1].astype(np.float64)
            b = d["b_xy"][sel, :n2].astype(np.float64)
            keep = _check_fd(orc, a, b, a_f32=d["a_xy"][sel, :n1], b_f32=d["b_xy"][sel, :n2])
            checked += keep.sum()
    assert checked > 200


def test_gradient_vs_finite_differences_3d(orc):
    d = synth.c1_pairs(n=1500, seed=63)
    rng = np.random.default_rng(64)
    a, b = d["a_xy"].astype(np.float64), d["b_xy"].astype(np.float64)
    z = rng.uniform(-2, 1, (a.shape[0], 2))
    hgt = rng.uniform(1.4, 1.8, (a.shape[0], 2))
    az = np.stack([z[:, 0] - hgt[:, 0] / 2, z[:, 0] + hgt[:, 0] / 2], 1)
    bz = np.stack([z[:, 1] - hgt[:, 1] / 2, z[:, 1] + hgt[:, 1] / 2], 1)
    keep = _check_fd(orc, a, b, az, bz, a_f32=d["a_xy"], b_f32=d["b_xy"])
    assert keep.sum() > 300


def test_gradient_invariants(orc):
    """IoU is invariant under translation, rotation and scaling, so its
    gradient field is orthogonal to those motions (summed over all vertices)."""
    for d in (synth.c3_pairs(n=2000, seed=71), synth.c4_polygons(n=2000, seed=72)):
        a, b = d["a_xy"], d["b_xy"]
        anv, bnv = d.get("a_nv"), d.get("b_nv")
        iou, nx, xf, _ = orc.iou_pairs(a, b, anv, bnv)
        ga, gb, _, _ = orc.iou_pairs_grad(a, b, d["grad"], nx, xf, anv, bnv)
        pts = np.concatenate([a, b], 1).astype(np.float64)
        grd = np.concatenate([ga, gb], 1)
        # padded slots carry zero gradient, so they drop out of the sums
        scale = np.abs(grd).sum((1, 2)) * (1 + np.abs(pts).max((1, 2)))
        tr = np.abs(grd.sum(1)).max(1)
        rot = np.abs((pts[..., 0] * grd[..., 1] - pts[..., 1] * grd[..., 0]).sum(1))
        sc = np.abs((pts[..., 0] * grd[..., 0] + pts[..., 1] * grd[..., 1]).sum(1))
        assert np.all(tr <= 1e-13 * scale + 1e-300)
        assert np.all(rot <= 1e-13 * scale + 1e-300)
        assert np.all(sc <= 1e-13 * scale + 1e-300)


def test_empty_pairs_have_zero_gradient(orc):
    a, b, _ = synth.degenerate_stress()
    iou, nx, xf, _ = orc.iou_pairs(a, b)
    ga, gb, _, _ = orc.iou_pairs_grad(a, b, np.ones(a.shape[0]), nx, xf)
    for i in range(a.shape[0]):
        if nx[i] == 0:
            assert not ga[i].any() and not gb[i].any()


# ---------------------------------------------------------------- 3D

def test_3d_closed_forms(orc):
    d = synth.c1_pairs(n=300, seed=81)
    a, b = d["a_xy"], d["b_xy"]
    rng = np.random.default_rng(82)
    lo = rng.uniform(-2, 1, 300).astype(np.float32)
    hi = (lo + rng.uniform(1.4, 1.8, 300)).astype(np.float32)
    iou2, _, _, _ = orc.iou_pairs(a, b)
    iou3, _, _, _ = orc.iou_pairs(a, b, a_z=(lo, hi), b_z=(lo, hi))
    assert np.max(np.abs(iou3 - iou2)) <= 1e-14     # equal z-extents reduce to 2D
    # identical footprints: IoU3 = hz / (h1 + h2 - hz)
    lo2 = (lo + rng.uniform(-1, 1, 300)).astype(np.float32)
    hi2 = (lo2 + rng.uniform(1.4, 1.8, 300)).astype(np.float32)
    iou3, _, _, _ = orc.iou_pairs(a, a, a_z=(lo, hi), b_z=(lo2, hi2))
    l1, h1, l2, h2 = (x.astype(np.float64) for x in (lo, hi, lo2, hi2))
    hz = np.maximum(0, np.minimum(h1, h2) - np.maximum(l1, l2))
    exp = hz / ((h1 - l1) + (h2 - l2) - hz)
    assert np.max(np.abs(iou3 - exp)) <= 1e-13


# ---------------------------------------------------------------- matrices

def test_matrix_matches_pairs_and_self_diagonal(orc):
    d = synth.c5_scenes(scenes=3, nmin=20, nmax=40, seed=91)
    xy, lo, hi, off = d["a_xy"], d["a_zlo"], d["a_zhi"], d["off"]
    m, out_off = orc.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    assert np.array_equal(out_off, d["out_off"])
    for s in range(3):
        n = int(off[s + 1] - off[s])
        blk = m[out_off[s]:out_off[s + 1]].reshape(n, n)
        assert np.all(np.diag(blk) == 1.0)
        r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        # entry (r, c) is the unordered pair with the lower index first
        ia = np.minimum(r, c).ravel() + off[s]
        ib = np.maximum(r, c).ravel() + off[s]
        v, _, _ = orc.iou_index_pairs(ia, ib, xy, xy, a_z=(lo, hi), b_z=(lo, hi))
        v = v.reshape(n, n)
        np.fill_diagonal(v, 1.0)
        assert np.array_equal(v, blk)
        assert np.array_equal(blk, blk.T)
        # and each entry is the IoU of its two boxes in either order, up to rounding
        w, _, _ = orc.iou_index_pairs(r.ravel() + off[s], c.ravel() + off[s], xy, xy,
                                      a_z=(lo, hi), b_z=(lo, hi))
        w = w.reshape(n, n)
        np.fill_diagonal(w, 1.0)
        assert np.max(np.abs(w - blk)) <= 1e-14


def test_matrix_grad_is_sum_of_pair_grads(orc):
    d = synth.c5_scenes(scenes=2, nmin=15, nmax=25, seed=92)
    xy, lo, hi, off = d["a_xy"], d["a_zlo"], d["a_zhi"], d["off"]
    # crowd the boxes so that many pairs overlap
    c = xy.astype(np.float64).mean(1, keepdims=True)
    xy = (xy - c + 0.08 * c).astype(np.float32)
    g = np.random.default_rng(93).uniform(-1, 1, int(d["out_off"][-1]))
    ga, _, gaz, _ = orc.iou_matrix_grad(g, xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    ref = np.zeros_like(ga)
    refz = np.zeros_like(gaz)
    for s in range(2):
        n = int(off[s + 1] - off[s])
        r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        sel = (r != c).ravel()
        # entry (r, c) is the pair with the lower index as the first polygon
        ia = (np.minimum(r, c).ravel() + off[s])[sel]
        ib = (np.maximum(r, c).ravel() + off[s])[sel]
        gs = g[d["out_off"][s]:d["out_off"][s + 1]][sel]
        _, nx, xf = orc.iou_index_pairs(ia, ib, xy, xy, a_z=(lo, hi), b_z=(lo, hi))
        pa, pb, pz1, pz2 = orc.iou_pairs_grad(xy[ia], xy[ib], gs, nx, xf,
                                              a_z=(lo[ia], hi[ia]), b_z=(lo[ib], hi[ib]))
        np.add.at(ref, ia, pa)
        np.add.at(ref, ib, pb)
        np.add.at(refz, ia, pz1)
        np.add.at(refz, ib, pz2)
    assert np.max(np.abs(ga - ref)) <= 1e-12
    assert np.max(np.abs(gaz - refz)) <= 1e-12
    assert np.abs(ga).max() > 0


def _tie_scene(rng):
    """A scene of 3D boxes full of exact contacts: integer axis-aligned boxes
    whose edges are collinear or touch, exact duplicates, boxes on a common
    ground plane (shared zlo) and shared tops, and a few rotated boxes."""
    n_int = 14
    x0 = rng.integers(0, 5, n_int).astype(np.float64)
    y0 = rng.integers(0, 5, n_int).astype(np.float64)
    w = rng.integers(1, 4, n_int).astype(np.float64)
    h = rng.integers(1, 4, n_int).astype(np.float64)
    quads = np.stack([np.stack([x0, y0], 1), np.stack([x0 + w, y0], 1),
                      np.stack([x0 + w, y0 + h], 1), np.stack([x0, y0 + h], 1)], 1)
    rot = synth.boxes_to_quads(rng.uniform(1, 4, 4), rng.uniform(1, 4, 4), rng.uniform(1, 3, 4),
                               rng.uniform(1, 3, 4), rng.uniform(-np.pi, np.pi, 4))
    xy = np.concatenate([quads.astype(np.float32), rot, quads[:3].astype(np.float32),
                         rot[:1]], 0)
    n = len(xy)
    zlo = np.where(rng.uniform(size=n) < 0.6, 0.0, rng.integers(-1, 2, n)).astype(np.float32)
    zhi = (zlo + rng.integers(1, 3, n)).astype(np.float32)
    zhi[::5] = 2.0  # shared tops as well
    zlo = np.minimum(zlo, zhi - 1.0).astype(np.float32)
    return xy, zlo, zhi


def test_self_pair_matrix_one_structure_per_pair(orc):
    """Reading R25 pinned by what must hold for any consistent derivative: in a
    self-pair matrix of tie-heavy 3D boxes (collinear and touching integer
    edges, duplicates, shared ground planes and tops) the matrix is exactly
    symmetric, and the summed gradient keeps the invariances of the 3D IoU:
    zero net force under translation in x, y and z, zero torque about z, and
    zero virial under scaling of the xy plane and of z.  Giving each row's
    box the first-polygon gradient of its own ordered entry, weighted by both
    entries' upstream gradients (so the two boxes of a pair take their
    gradients from two different tie structures: the rule R25 replaces)
    breaks them on the same boxes."""
    rng = np.random.default_rng(97)
    xy, lo, hi = _tie_scene(rng)
    n = len(xy)
    off = np.array([0, n], np.int64)
    m, _ = orc.iou_matrix(xy, a_z=(lo, hi), a_off=off, self_pairs=True)
    blk = m.reshape(n, n)
    assert np.array_equal(blk, blk.T)
    assert np.count_nonzero(blk) > 3 * n  # the contacts make many non-empty pairs
    p = xy.astype(np.float64)

    def residuals(gxy, gz):
        fx, fy = gxy[..., 0].sum(), gxy[..., 1].sum()
        fz = (gz[:, 0] + gz[:, 1]).sum()
        torque = (p[..., 0] * gxy[..., 1] - p[..., 1] * gxy[..., 0]).sum()
        virial = (p[..., 0] * gxy[..., 0] + p[..., 1] * gxy[..., 1]).sum()
        zvir = (lo * gz[:, 0] + hi * gz[:, 1]).sum()
        return np.abs([fx, fy, fz, torque, virial, zvir])

    worst_ordered = 0.0
    for t in range(6):
        g = rng.uniform(-1, 1, n * n)
        ga, _, gz, _ = orc.iou_matrix_grad(g, xy, a_z=(lo, hi), a_off=off, self_pairs=True)
        scale = np.abs(ga).sum() + np.abs(gz).sum()
        assert scale > 0
        assert residuals(ga, gz).max() <= 1e-12 * scale, residuals(ga, gz)
        # the replaced rule: row i takes (g[i, k] + g[k, i]) times the first-
        # polygon gradient of entry (i, k) evaluated in that order
        r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        sel = (r != c).ravel()
        ia, ib = r.ravel()[sel], c.ravel()[sel]
        w = (g.reshape(n, n) + g.reshape(n, n).T).ravel()[sel]
        _, nx, xf = orc.iou_index_pairs(ia, ib, xy, xy, a_z=(lo, hi), b_z=(lo, hi))
        pa, _, pz1, _ = orc.iou_pairs_grad(xy[ia], xy[ib], w, nx, xf,
                                           a_z=(lo[ia], hi[ia]), b_z=(lo[ib], hi[ib]))
        oa = np.zeros_like(ga)
        oz = np.zeros_like(gz)
        np.add.at(oa, ia, pa)
        np.add.at(oz, ia, pz1)
        worst_ordered = max(worst_ordered, residuals(oa, oz).max() / scale)
    assert worst_ordered > 1e-3, worst_ordered


def test_pair_margins_closed_forms(orc):
    """The five degeneracy margins that select the parity set, on pairs whose
    values are known in closed form (a mistake in any margin, such as a
    dropped normalisation, segment instead of line distances, a wrong edge
    index or the wrong polygon's area, changes at least one):
      [0] smallest vertex distance to an edge line of the other polygon,
          over the union's bounding-box diagonal L;
      [1] smallest |sin| between two crossing edges;
      [2] smallest normalised turn of either polygon (sin of the exterior
          angle);
      [3] smallest normalised cross product of consecutive intersection
          vertices seen from their centroid;
      [4] intersection area over the smaller polygon's area."""
    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float64)
    # A: unit square and the unit square moved by (0.3, 0.2): the nearest
    # vertex / line distance is 0.2 (Q_0 above y = 0), L the diagonal of
    # [0, 1.3] x [0, 1.2], crossings at right angles, the intersection the
    # 0.7 x 0.8 rectangle whose corners are seen from its centre at the
    # half-diagonal angle 2 atan(0.8 / 0.7)
    pa, qa = sq, sq + [0.3, 0.2]
    ang = 2 * math.atan2(0.4, 0.35)
    want_a = [0.2 / math.hypot(1.3, 1.2), 1.0, 1.0, min(math.sin(ang), math.sin(math.pi - ang)),
              0.7 * 0.8]
    # B: squares of half-size 1 about one centre, the second turned by pi/4:
    # the regular octagon between them; vertex / line distance sqrt(2) - 1,
    # L = the diagonal of the [-sqrt 2, sqrt 2]^2 bounding box = 4, crossings
    # at 45 degrees, octagon vertices 45 degrees apart, area 8 sqrt 2 - 8 of 4
    r2 = math.sqrt(2.0)
    pb = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], np.float64)
    qb = np.array([[0, -r2], [r2, 0], [0, r2], [-r2, 0]])
    want_b = [(r2 - 1) / 4, math.sin(math.pi / 4), 1.0, math.sin(math.pi / 4), (8 * r2 - 8) / 4]
    # C: a regular hexagon of circumradius 1 inside a 10 x 10 square: every
    # turn of the hexagon is sin(60 deg); no crossing; the intersection is
    # the hexagon (ratio 1), its vertices 60 degrees apart.  The nearest
    # vertex / line pair is not the hexagon against a side (4 away) but a
    # square corner against the line of a hexagon edge whose normal points
    # 30 degrees from the x axis: 5 (cos 30 - sin 30) - cos 30 away
    t = np.arange(6) * math.pi / 3
    ph = np.stack([np.cos(t), np.sin(t)], 1)
    qh = np.array([[-5, -5], [5, -5], [5, 5], [-5, 5]], np.float64)
    c30, s30 = math.cos(math.pi / 6), math.sin(math.pi / 6)
    want_c = [(5 * (c30 - s30) - c30) / math.hypot(10, 10), 1.0, math.sin(math.pi / 3),
              math.sin(math.pi / 3), 1.0]
    # D: disjoint squares: no crossing, empty intersection (margins 3, 4 are 1)
    pd, qd = sq, sq + [3.0, 0.5]
    want_d = [0.5 / math.hypot(4, 1.5), 1.0, 1.0, 1.0, 1.0]
    for p, q, want in ((pa, qa, want_a), (pb, qb, want_b), (ph, qh, want_c), (pd, qd, want_d)):
        k = max(len(p), len(q), 4)
        a = np.zeros((1, 8, 2), np.float32)
        b = np.zeros((1, 8, 2), np.float32)
        a[0, :len(p)] = p
        b[0, :len(q)] = q
        got = orc.pair_margins(a, b, np.array([len(p)], np.uint8), np.array([len(q)], np.uint8))[0]
        # the inputs are rounded to fp32 (sqrt 2 and the hexagon)
        assert np.allclose(got, want, rtol=2e-6, atol=1e-7), (got, want, k)


# ------------------------------------------------- intersection and area primitives

def test_intersect_pairs_exact_rational(orc):
    """Batched intersection polygons (fp64 vertices, nx, flags) against exact
    rational clipping of the same fp32 inputs."""
    checked = 0
    for a, b, anv, bnv in _pair_sets():
        keep = _filtered(orc, a, b, anv, bnv)
        xy, nx, xf, bad = orc.intersect_pairs(a, b, anv, bnv)
        assert bad == 0
        cap = a.shape[1] + b.shape[1]
        assert xy.shape == (len(a), cap, 2)
        for i in np.nonzero(keep)[0][:120]:
            n1 = int(anv[i]) if anv is not None else a.shape[1]
            n2 = int(bnv[i]) if bnv is not None else b.shape[1]
            P, Q = X.fpoly(a[i, :n1]), X.fpoly(b[i, :n2])
            V = X.clip(P, Q)
            m = int(nx[i])
            assert m == len(V)
            assert np.all(xy[i, m:] == 0.0) and np.all(xf[i, m:] == 0xFF)
            if m == 0:
                continue
            s = V.index(X.vertex_from_code(P, Q, int(xf[i, 0])))
            ex = V[s:] + V[:s]
            scale = max(1.0, float(np.abs(a[i]).max()), float(np.abs(b[i]).max()))
            for k in range(m):
                assert X.classify(P, Q, ex[k]) == {int(xf[i, k])}
                assert abs(xy[i, k, 0] - float(ex[k][0])) <= 1e-13 * scale
                assert abs(xy[i, k, 1] - float(ex[k][1])) <= 1e-13 * scale
            checked += 1
    assert checked > 200


def _perturbable(x, h):
    """x + h and x - h are exact in fp32 (so differences see exactly +-h)."""
    x = np.asarray(x, np.float32)
    hp = (x + np.float32(h)).astype(np.float64) - x.astype(np.float64)
    hm = x.astype(np.float64) - (x - np.float32(h)).astype(np.float64)
    return (hp == h) & (hm == h)


def test_intersect_grad_vs_finite_differences(orc):
    """Gradient of sum <gX, X> over the intersection vertices (vertex codes
    pass through, crossings through the homogeneous meet) against central
    differences with a Richardson step, on pairs whose flags are unchanged."""
    rng = np.random.default_rng(77)
    for d in (synth.c3_pairs(n=512, seed=71), synth.c4_polygons(n=512, seed=72)):
        a, b = d["a_xy"], d["b_xy"]
        anv, bnv = d.get("a_nv"), d.get("b_nv")
        n, ka = a.shape[:2]
        kb = b.shape[1]
        cap = ka + kb
        xy, nx, xf, _ = orc.intersect_pairs(a, b, anv, bnv)
        gX = rng.uniform(-1, 1, (n, cap, 2))
        gX[np.arange(cap)[None, :] >= nx[:, None]] = 0.0
        ga, gb = orc.intersect_pairs_grad(a, b, gX, nx, xf, anv, bnv)
        keep = nx > 0
        h = 2.0 ** -10
        cols = {h: [], h / 2: []}
        for which, k, c in [("a", k, c) for k in range(ka) for c in range(2)] + \
                           [("b", k, c) for k in range(kb) for c in range(2)]:
            src = a if which == "a" else b
            keep &= _perturbable(src[:, k, c], h) & _perturbable(src[:, k, c], h / 2)
            for step in (h, h / 2):
                vals = []
                for sgn in (1.0, -1.0):
                    aa, bb = a.copy(), b.copy()
                    (aa if which == "a" else bb)[:, k, c] += np.float32(sgn * step)
                    xp, nxp, xfp, _ = orc.intersect_pairs(aa, bb, anv, bnv)
                    keep &= (nxp == nx) & np.all(xfp == xf, axis=1)
                    vals.append((gX * xp).sum(axis=(1, 2)))
                cols[step].append((vals[0] - vals[1]) / (2 * step))
        fd1, fd2 = np.stack(cols[h], 1), np.stack(cols[h / 2], 1)
        fdr = (4.0 * fd2 - fd1) / 3.0
        an = np.concatenate([ga.reshape(n, -1), gb.reshape(n, -1)], 1)
        den = np.maximum(np.linalg.norm(an, axis=1), 1e-8)
        err = (np.linalg.norm(an - fdr, axis=1) / den)[keep]
        assert keep.sum() > 200, keep.sum()
        # extrapolated differences: truncation O(h^4), the bound of the IoU test
        assert err.max() <= 1e-5, np.sort(err)[-5:]
        # padded slots of the polygons carry no gradient
        if anv is not None:
            pad_a = np.arange(ka)[None, :] >= anv[:, None]
            assert np.all(ga[pad_a] == 0.0)


def test_intersect_grad_vertex_codes_pass_through(orc):
    """Nested polygons: every intersection vertex is a vertex of the inner
    polygon, so the gradient is the upstream one, unchanged, on that polygon."""
    outer = np.array([[[-4, -4], [4, -4], [4, 4], [-4, 4]]], np.float32)
    inner = np.array([[[-1, -0.5], [1.5, -1], [1, 1], [-0.5, 1.25]]], np.float32)
    xy, nx, xf, _ = orc.intersect_pairs(outer, inner)
    assert nx[0] == 4 and set(xf[0, :4].tolist()) == {0x10, 0x11, 0x12, 0x13}
    g = np.zeros((1, 8, 2))
    g[0, :4] = np.arange(8).reshape(4, 2) + 1.0
    ga, gb = orc.intersect_pairs_grad(outer, inner, g, nx, xf)
    assert np.all(ga == 0.0)
    for r in range(4):
        assert np.array_equal(gb[0, xf[0, r] & 0x0F], g[0, r])


def test_areas_closed_forms_and_gradient(orc):
    sq = np.array([[[0, 0], [2, 0], [2, 2], [0, 2]]], np.float32)
    tri = np.array([[[0, 0], [3, 0], [0, 4], [0, 0]]], np.float32)
    assert orc.areas(sq)[0] == 4.0
    assert orc.areas(tri, np.array([3], np.uint8))[0] == 6.0
    # dA/dv_k = (y_k+1 - y_k-1, x_k-1 - x_k+1) / 2, written out for the square
    g = orc.areas_grad(sq, np.ones(1))[0]
    assert np.array_equal(g, np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], np.float64))
    gt = orc.areas_grad(tri, np.ones(1), np.array([3], np.uint8))[0]
    assert np.array_equal(gt, np.array([[-2, -1.5], [2, 0], [0, 1.5], [0, 0]], np.float64))
    # random polygons: translation invariance of the gradient and central
    # differences (the area is quadratic, so they are exact up to rounding)
    d = synth.c4_polygons(n=256, seed=81)
    xy, nv = d["a_xy"], d["a_nv"]
    gg = orc.areas_grad(xy, np.ones(len(xy)), nv)
    assert np.abs(gg.sum(axis=1)).max() <= 1e-12
    h = 2.0 ** -8
    for k in range(8):
        for c in range(2):
            ok = _perturbable(xy[:, k, c], h)
            p, m = xy.copy(), xy.copy()
            p[:, k, c] += np.float32(h)
            m[:, k, c] -= np.float32(h)
            fd = (orc.areas(p, nv) - orc.areas(m, nv)) / (2 * h)
            assert np.abs(fd - gg[:, k, c])[ok].max() <= 1e-9


# ------------------------------------------------------------ box front end

def _corners_np(box):
    """R11 written out in numpy fp64: c + R(yaw) (+-l/2, +-w/2), CCW from
    (+l/2, -w/2)."""
    b = np.asarray(box, np.float64)
    cx, cy, w, l, yaw = b[:, 0], b[:, 1], b[:, 2], b[:, 3], b[:, 4]
    sl = np.array([1, 1, -1, -1], np.float64) * 0.5
    sw = np.array([-1, 1, 1, -1], np.float64) * 0.5
    dx, dy = l[:, None] * sl, w[:, None] * sw
    c, s = np.cos(yaw)[:, None], np.sin(yaw)[:, None]
    return np.stack([cx[:, None] + c * dx - s * dy, cy[:, None] + s * dx + c * dy], -1)


def test_boxes_match_corner_form(orc):
    d = synth.c3_boxes(n=2048, seed=101, three_d=True)
    for dim in (5, 7):
        a, b = d["a_box"][:, :dim], d["b_box"][:, :dim]
        iou, nx, xf, bad = orc.iou_boxes(a, b)
        assert bad == 0
        az = bz = None
        if dim == 7:
            az = np.stack([a[:, 5].astype(np.float64) - 0.5 * a[:, 6],
                           a[:, 5].astype(np.float64) + 0.5 * a[:, 6]], 1)
            bz = np.stack([b[:, 5].astype(np.float64) - 0.5 * b[:, 6],
                           b[:, 5].astype(np.float64) + 0.5 * b[:, 6]], 1)
        ref, rnx, rxf = orc.iou_pairs_f64(_corners_np(a), _corners_np(b), az, bz)
        assert np.abs(iou - ref).max() <= 1e-13
        assert np.array_equal(nx, rnx) and np.array_equal(xf, rxf)


def test_boxes_axis_aligned_closed_form(orc):
    """yaw 0: the boxes are [cx -+ l/2] x [cy -+ w/2]; yaw pi/2 swaps the
    extents (dyadic values, exact in fp32; cos(pi/2) is ~6e-17 in fp64)."""
    a = np.array([[0, 0, 2, 4, 0], [1, 1, 1, 3, 0], [0, 0, 2, 2, 0]], np.float32)
    b = np.array([[1, 0.5, 2, 4, 0], [5, 5, 1, 1, 0], [0.5, 0.25, 2, 2, 0]], np.float32)
    iou, nx, xf, _ = orc.iou_boxes(a, b)
    # pair 0: x [-2,2] vs [-1,3] -> 3, y [-1,1] vs [-0.5,1.5] -> 1.5: I = 4.5, U = 16 - 4.5
    # pair 1: disjoint; pair 2: x [-1,1] vs [-0.5,1.5] -> 1.5, y [-1,1] vs
    # [-0.75,1.25] -> 1.75: I = 2.625, U = 8 - 2.625
    assert abs(iou[0] - 4.5 / 11.5) <= 1e-15 and iou[1] == 0.0 and nx[1] == 0
    assert abs(iou[2] - 2.625 / 5.375) <= 1e-15
    a2 = a.copy()
    a2[:, 4] = np.float32(np.pi / 2)
    a2[:, [2, 3]] = a[:, [3, 2]]  # w <-> l with a quarter turn: the same footprint
    iou2, _, _, _ = orc.iou_boxes(a2, b)
    assert np.abs(iou2 - iou).max() <= 1e-6


def test_boxes_grad_vs_finite_differences(orc):
    d = synth.c3_boxes(n=1024, seed=102, three_d=True)
    for dim in (5, 7):
        a = np.ascontiguousarray(d["a_box"][:, :dim])
        b = np.ascontiguousarray(d["b_box"][:, :dim])
        n = len(a)
        iou, nx, xf, _ = orc.iou_boxes(a, b)
        ga, gb = orc.iou_boxes_grad(a, b, np.ones(n), nx, xf)
        keep = nx > 0
        if dim == 7:
            zl1, zh1 = a[:, 5] - 0.5 * a[:, 6], a[:, 5] + 0.5 * a[:, 6]
            zl2, zh2 = b[:, 5] - 0.5 * b[:, 6], b[:, 5] + 0.5 * b[:, 6]
            hz = np.minimum(zh1, zh2) - np.maximum(zl1, zl2)
            keep &= (np.abs(zh1 - zh2) > 0.05) & (np.abs(zl1 - zl2) > 0.05) & (hz > 0.05)
        h = 2.0 ** -10
        cols = {h: [], h / 2: []}
        for which in ("a", "b"):
            for t in range(dim):
                src = a if which == "a" else b
                keep &= _perturbable(src[:, t], h) & _perturbable(src[:, t], h / 2)
                for step in (h, h / 2):
                    vals = []
                    for sgn in (1.0, -1.0):
                        aa, bb = a.copy(), b.copy()
                        (aa if which == "a" else bb)[:, t] += np.float32(sgn * step)
                        v, nxp, xfp, _ = orc.iou_boxes(aa, bb)
                        keep &= (nxp == nx) & np.all(xfp == xf, axis=1)
                        vals.append(v)
                    cols[step].append((vals[0] - vals[1]) / (2 * step))
        fd1, fd2 = np.stack(cols[h], 1), np.stack(cols[h / 2], 1)
        fdr = (4.0 * fd2 - fd1) / 3.0
        an = np.concatenate([ga, gb], 1)
        den = np.maximum(np.linalg.norm(an, axis=1), 1e-8)
        err = (np.linalg.norm(an - fdr, axis=1) / den)[keep]
        assert keep.sum() > 300, keep.sum()
        assert err.max() <= 1e-5, np.sort(err)[-5:]


def _star(p, q, k=8, r=1.0, phase=0.1):
    """Vertices of the star polygon {p/q} (q = 1: the regular p-gon), padded
    to k slots."""
    v = [[r * math.cos(phase + 2 * math.pi * q * t / p), r * math.sin(phase + 2 * math.pi * q * t / p)]
         for t in range(p)]
    v += [v[0]] * (k - p)
    return v


def test_polygon_status_geometric_facts(orc):
    """The input contract of Sec. III (convex, counter-clockwise): a regular
    p-gon is valid, its reverse is clockwise, a star polygon {p/q} turns
    left at every vertex but winds q times, a straight or repeated vertex is
    not a strict left turn, and vertex counts outside [3, kmax] are refused."""
    cases, nv, want = [], [], []

    def add(v, n, code):
        cases.append(v + [v[0]] * (8 - len(v)))
        nv.append(n)
        want.append(code)

    for p in range(3, 9):
        add(_star(p, 1, p), p, 0)
        add(_star(p, 1, p)[::-1], p, 2)
    add(_star(5, 2, 5), 5, 3)
    add(_star(7, 2, 7), 7, 3)
    add(_star(7, 3, 7), 7, 3)
    add(_star(8, 3, 8), 8, 3)
    add([[0, 0], [1, 0], [1, 0], [1, 1], [0, 1]], 5, 2)         # repeated vertex
    add([[0, 0], [0.5, 0], [1, 0], [1, 1], [0, 1]], 5, 2)       # straight vertex
    add([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]], 6, 2)  # L-shape (reflex)
    add([[0, 0], [1, 0], [1, 1], [0, 1]], 2, 1)
    add([[0, 0], [1, 0], [1, 1], [0, 1]], 0, 1)
    add([[0, 0], [1, 0], [1, 1], [0, 1]], 9, 1)
    xy = np.array(cases, np.float32)
    st = orc.polygon_status(xy, np.array(nv, np.uint8))
    assert list(st) == want
    # fixed-count form (nv NULL => kmax) on the valid p = 8 case
    assert list(orc.polygon_status(xy[10:12])) == [0, 2]
