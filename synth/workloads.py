"""Seeded generators for the five workloads of the rotated-box IoU study.

Every generator draws in fp64 with numpy's PCG64 and rounds the resulting
vertices to fp32 once; those fp32 values are the canonical input that both
the GPU library and the FP64 oracle read.

Workloads (sizes are the defaults; `n` / `scenes` shrink them with the same
distributions for tests):
  c1  1,024 elementwise pairs of rotated rectangles (Sec. IV-A case study):
      centre U[-2,2]^2, w,l U[1,3], yaw U[-pi,pi]; the second box keeps w,l,
      moves its centre by N(0, 0.5^2) per axis and its yaw by N(0, 0.3^2).
  c2  4096 x 4096 IoU matrix of BEV car boxes: x U[0,70], y U[-40,40],
      w U[1.5,2.2], l U[3.5,5.0], yaw U[-pi,pi]; two independent sets A, B.
  c3  1,048,576 elementwise rectangle pairs: base as c1, the second box
      perturbed by centre N(0, 0.3^2), size N(0, 0.1^2) (additive, redrawn
      below 0.1) and yaw N(0, 0.2^2).
  c4  262,144 pairs of convex polygons with 3..8 vertices (uniform per
      polygon) at sorted angles U[0, 2pi) on axis-aligned ellipses with radii
      U[0.5, 2] and centre U[-1,1]^2; stored [n, 8, 2] plus counts.
  c5  64 scenes with U{50..2000} boxes each, BEV as c2, centre height
      z U[-2,1], height h U[1.4,1.8]; self-pairwise 3D IoU per scene.
Upstream gradients are U[-1, 1].
"""
import math

import numpy as np

SEED_BASE = 1000


def _rng(cfg_index, seed=None):
    return np.random.Generator(np.random.PCG64(SEED_BASE + cfg_index if seed is None else seed))


def boxes_to_quads(cx, cy, w, l, yaw):
    """Rotated boxes -> 4 counter-clockwise corners [n, 4, 2] fp32.

    The length l runs along the heading yaw, the width w across it; corners
    are centre + R(yaw) (+-l/2, +-w/2) starting at (+l/2, -w/2).  Computed in
    fp64, rounded to fp32 once."""
    cx, cy, w, l, yaw = (np.asarray(v, np.float64) for v in (cx, cy, w, l, yaw))
    lx = np.array([0.5, 0.5, -0.5, -0.5])
    wy = np.array([-0.5, 0.5, 0.5, -0.5])
    u = l[:, None] * lx[None, :]
    v = w[:, None] * wy[None, :]
    c, s = np.cos(yaw)[:, None], np.sin(yaw)[:, None]
    x = cx[:, None] + c * u - s * v
    y = cy[:, None] + s * u + c * v
    return np.stack([x, y], axis=-1).astype(np.float32)


def _draw_boxes(rng, n, center_lo, center_hi, wl_lo, wl_hi, w_range=None, l_range=None):
    cx = rng.uniform(center_lo[0], center_hi[0], n)
    cy = rng.uniform(center_lo[1], center_hi[1], n)
    if w_range is None:
        w = rng.uniform(wl_lo, wl_hi, n)
        l = rng.uniform(wl_lo, wl_hi, n)
    else:
        w = rng.uniform(*w_range, n)
        l = rng.uniform(*l_range, n)
    yaw = rng.uniform(-math.pi, math.pi, n)
    return cx, cy, w, l, yaw


def c1_pairs(n=1024, seed=None, center_sigma=0.5, yaw_sigma=0.3, size_sigma=None, cfg=0,
             box_params=False):
    rng = _rng(cfg, seed)
    cx, cy, w, l, yaw = _draw_boxes(rng, n, (-2, -2), (2, 2), 1.0, 3.0)
    cx2 = cx + rng.normal(0.0, center_sigma, n)
    cy2 = cy + rng.normal(0.0, center_sigma, n)
    yaw2 = yaw + rng.normal(0.0, yaw_sigma, n)
    if size_sigma is None:
        w2, l2 = w.copy(), l.copy()
    else:
        w2 = w + rng.normal(0.0, size_sigma, n)
        l2 = l + rng.normal(0.0, size_sigma, n)
        for arr, base in ((w2, w), (l2, l)):
            bad = arr < 0.1
            while bad.any():
                arr[bad] = base[bad] + rng.normal(0.0, size_sigma, int(bad.sum()))
                bad = arr < 0.1
    a = boxes_to_quads(cx, cy, w, l, yaw)
    b = boxes_to_quads(cx2, cy2, w2, l2, yaw2)
    g = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    out = {"a_xy": a, "b_xy": b, "grad": g, "kind": "pairs"}
    if box_params:
        # the same boxes as parameter rows (cx, cy, w, l, yaw), rounded to fp32
        out["a_box"] = np.stack([cx, cy, w, l, yaw], 1).astype(np.float32)
        out["b_box"] = np.stack([cx2, cy2, w2, l2, yaw2], 1).astype(np.float32)
    return out


def c3_pairs(n=1 << 20, seed=None, box_params=False):
    return c1_pairs(n=n, seed=seed, center_sigma=0.3, yaw_sigma=0.2, size_sigma=0.1, cfg=2,
                    box_params=box_params)


def c3_boxes(n=1 << 20, seed=None, three_d=False):
    """c3's rectangle pairs as box-parameter rows for the fused box front end:
    a_box, b_box [n, 5] fp32 (cx, cy, w, l, yaw), or [n, 7] with the c5 z
    distribution appended (z centre U[-2, 1], h U[1.4, 1.8]; the second box's
    z moved by N(0, 0.3^2)); grad U[-1, 1]."""
    d = c3_pairs(n=n, seed=seed, box_params=True)
    out = {"a_box": d["a_box"], "b_box": d["b_box"], "grad": d["grad"], "kind": "boxes"}
    if three_d:
        rng = _rng(5, None if seed is None else seed + 1)
        z = rng.uniform(-2.0, 1.0, n)
        h = rng.uniform(1.4, 1.8, n)
        z2 = z + rng.normal(0.0, 0.3, n)
        h2 = rng.uniform(1.4, 1.8, n)
        out["a_box"] = np.concatenate([d["a_box"], np.stack([z, h], 1).astype(np.float32)], 1)
        out["b_box"] = np.concatenate([d["b_box"], np.stack([z2, h2], 1).astype(np.float32)], 1)
    return out


def c3_intersect(n=1 << 20, seed=None):
    """c3's rectangle pairs for the exported intersection primitive, with an
    upstream gradient per intersection vertex: grad_xy [n, 8, 2] U[-1, 1]
    (slots past a pair's vertex count are ignored by the backward)."""
    d = c3_pairs(n=n, seed=seed)
    rng = _rng(6, None if seed is None else seed + 2)
    return {"a_xy": d["a_xy"], "b_xy": d["b_xy"],
            "grad_xy": rng.uniform(-1.0, 1.0, (n, 8, 2)).astype(np.float32),
            "kind": "intersect"}


def bev_boxes(rng, n):
    return _draw_boxes(rng, n, (0.0, -40.0), (70.0, 40.0), None, None,
                       w_range=(1.5, 2.2), l_range=(3.5, 5.0))


def c2_matrix(n=4096, m=4096, seed=None):
    rng = _rng(1, seed)
    a = boxes_to_quads(*bev_boxes(rng, n))
    b = boxes_to_quads(*bev_boxes(rng, m))
    return {"a_xy": a, "b_xy": b, "kind": "matrix"}


def _strictly_convex32(xy, n, min_turn):
    """True if the first n fp32 vertices turn left by at least min_turn
    (normalised) at every vertex; a precondition of the method's inputs."""
    p = xy[:n].astype(np.float64)
    u = p - np.roll(p, 1, axis=0)
    v = np.roll(p, -1, axis=0) - p
    cr = u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0]
    nu = np.hypot(u[:, 0], u[:, 1]) * np.hypot(v[:, 0], v[:, 1])
    return bool(np.all(cr > min_turn * nu))


def random_convex(rng, n, kmin=3, kmax=8, min_turn=0.0, stats=None):
    """n convex polygons [n, kmax, 2] fp32 (zero padded) and counts [n] u8.
    A polygon whose rounded vertices do not turn left by more than min_turn
    (normalised) at every vertex is redrawn; by default only those that break
    the convex, counter-clockwise input contract (Sec. III) after rounding,
    so that near-degenerate polygons stay in the workload.  stats (a dict)
    receives the number of redraws."""
    xy = np.zeros((n, kmax, 2), np.float32)
    nv = rng.integers(kmin, kmax + 1, n).astype(np.uint8)
    todo = np.arange(n)
    while todo.size:
        t = todo.size
        ang = rng.uniform(0.0, 2 * math.pi, (t, kmax))
        rx = rng.uniform(0.5, 2.0, t)[:, None]
        ry = rng.uniform(0.5, 2.0, t)[:, None]
        cx = rng.uniform(-1.0, 1.0, t)[:, None]
        cy = rng.uniform(-1.0, 1.0, t)[:, None]
        # the first nv draws, sorted, are the polygon's angles; the rest is unused
        k = nv[todo]
        mask = np.arange(kmax)[None, :] < k[:, None]
        ang = np.where(mask, ang, np.inf)
        ang = np.sort(ang, axis=1)
        ang = np.where(mask, ang, 0.0)
        px = np.where(mask, cx + rx * np.cos(ang), 0.0)
        py = np.where(mask, cy + ry * np.sin(ang), 0.0)
        cand = np.stack([px, py], axis=-1).astype(np.float32)
        ok = np.array([_strictly_convex32(cand[r], int(k[r]), min_turn) for r in range(t)])
        xy[todo[ok]] = cand[ok]
        todo = todo[~ok]
        if stats is not None:
            stats["redrawn"] = stats.get("redrawn", 0) + int(todo.size)
    return xy, nv


def random_simple(rng, n, centers, kmin=3, kmax=8, min_gap=0.15, rmin=0.4, rmax=1.6):
    """n simple, counter-clockwise, generally non-convex polygons [n, kmax, 2]
    fp32 (zero padded) and counts [n] u8: vertices at strictly increasing
    angles about the given centres ([n, 2]), each angular gap in
    [min_gap, 0.9 pi] (so the centre is inside and the polygon is star-shaped
    about it), radii U[rmin, rmax]."""
    nv = rng.integers(kmin, kmax + 1, n).astype(np.uint8)
    gaps = np.zeros((n, kmax))
    todo = np.arange(n)
    while todo.size:
        t = todo.size
        k = nv[todo]
        mask = np.arange(kmax)[None, :] < k[:, None]
        g = np.where(mask, rng.uniform(0.2, 1.0, (t, kmax)), 0.0)
        g = g / g.sum(1, keepdims=True) * (2 * math.pi)
        ok = np.all(np.where(mask, (g >= min_gap) & (g <= 0.9 * math.pi), True), axis=1)
        gaps[todo[ok]] = g[ok]
        todo = todo[~ok]
    start = rng.uniform(0.0, 2 * math.pi, (n, 1))
    ang = start + np.cumsum(gaps, axis=1) - gaps
    r = rng.uniform(rmin, rmax, (n, kmax))
    mask = np.arange(kmax)[None, :] < nv[:, None]
    px = np.where(mask, centers[:, :1] + r * np.cos(ang), 0.0)
    py = np.where(mask, centers[:, 1:] + r * np.sin(ang), 0.0)
    return np.stack([px, py], axis=-1).astype(np.float32), nv


def c4_simple(n=1 << 18, seed=None):
    """262,144 pairs of simple 3..8-gons, generally non-convex (star-shaped
    about their centres): centres U[-1, 1]^2, the second polygon's centre
    moved by N(0, 0.5^2) per axis; grad U[-1, 1]."""
    rng = _rng(7, seed)
    ca = rng.uniform(-1.0, 1.0, (n, 2))
    cb = ca + rng.normal(0.0, 0.5, (n, 2))
    a, anv = random_simple(rng, n, ca)
    b, bnv = random_simple(rng, n, cb)
    g = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    return {"a_xy": a, "a_nv": anv, "b_xy": b, "b_nv": bnv, "grad": g, "kind": "simple"}


def c4_polygons(n=1 << 18, seed=None):
    rng = _rng(3, seed)
    st = {}
    a, anv = random_convex(rng, n, stats=st)
    b, bnv = random_convex(rng, n, stats=st)
    g = rng.uniform(-1.0, 1.0, n).astype(np.float32)
    return {"a_xy": a, "a_nv": anv, "b_xy": b, "b_nv": bnv, "grad": g, "kind": "pairs",
            "redrawn": st.get("redrawn", 0)}


def c5_scenes(scenes=64, nmin=50, nmax=2000, seed=None, with_grad=True):
    rng = _rng(4, seed)
    counts = rng.integers(nmin, nmax + 1, scenes)
    total = int(counts.sum())
    xy = boxes_to_quads(*bev_boxes(rng, total))
    z = rng.uniform(-2.0, 1.0, total)
    h = rng.uniform(1.4, 1.8, total)
    zlo = (z - 0.5 * h).astype(np.float32)
    zhi = (z + 0.5 * h).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    sizes = counts.astype(np.int64) ** 2
    out_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out = {"a_xy": xy, "a_zlo": zlo, "a_zhi": zhi, "off": off, "out_off": out_off,
           "kind": "scenes"}
    if with_grad:
        out["grad"] = rng.uniform(-1.0, 1.0, int(out_off[-1])).astype(np.float32)
    return out


def degenerate_stress():
    """Exactly degenerate rectangle pairs on dyadic coordinates (exact in fp32):
    identical, shared edge, vertex on an edge, nested, touching at a corner,
    collinear overlapping edges.  Returns (a [n,4,2], b [n,4,2], names)."""
    def rect(x0, y0, x1, y1):
        return [[x0, y0], [x1, y0], [x1, y1], [x0, y1]]

    def diamond(cx, cy, r):
        return [[cx + r, cy], [cx, cy + r], [cx - r, cy], [cx, cy - r]]

    cases = [
        ("identical", rect(0, 0, 2, 1), rect(0, 0, 2, 1)),
        ("identical_rot", diamond(0.5, 0.25, 1.0), diamond(0.5, 0.25, 1.0)),
        ("shared_edge", rect(0, 0, 1, 1), rect(1, 0, 2, 1)),
        ("half_shared_edge", rect(0, 0, 1, 1), rect(1, 0.5, 2, 1.5)),
        ("overlap_collinear_edges", rect(0, 0, 2, 1), rect(1, 0, 3, 1)),
        ("same_bottom_edge", rect(0, 0, 2, 1), rect(0.5, 0, 1.5, 2)),
        ("vertex_on_edge", rect(0, 0, 2, 2), diamond(3, 1, 1)),
        ("vertex_on_edge_inside", rect(0, 0, 2, 2), diamond(1.5, 1, 0.5)),
        ("nested_touching", rect(0, 0, 4, 4), rect(0, 1, 2, 3)),
        ("nested_strict", rect(0, 0, 4, 4), rect(1, 1, 2, 3)),
        ("corner_touch", rect(0, 0, 1, 1), rect(1, 1, 2, 2)),
        ("cross_shape", rect(0, 1, 4, 2), rect(1, 0, 2, 4)),
        ("diamond_in_square", rect(-1, -1, 1, 1), diamond(0, 0, 1.0)),
        ("disjoint", rect(0, 0, 1, 1), rect(3, 3, 4, 4)),
    ]
    a = np.array([c[1] for c in cases], np.float32)
    b = np.array([c[2] for c in cases], np.float32)
    return a, b, [c[0] for c in cases]


WORKLOADS = {
    "c1": c1_pairs,
    "c2": c2_matrix,
    "c3": c3_pairs,
    "c4": c4_polygons,
    "c5": c5_scenes,
    "c3b": c3_boxes,
    "c3i": c3_intersect,
    "c4n": c4_simple,
}


def get(name, **kw):
    return WORKLOADS[name](**kw)
