"""FP64 CPU oracle (ctypes wrapper over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline leg
of the benchmark are its only users.  It shares no code with the GPU library
and never imports it.

All batched functions take the same fp32 arrays the GPU library reads
(polygons as [n, kmax, 2] fp32, optional vertex counts [n] uint8, optional z
extents as separate [n] fp32 arrays zlo / zhi) and compute in fp64.
"""
import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        # DGAL_ORACLE_LIB: another build of the same sources (the sanitizer
        # build of the CPU tests); else the regular one, built on first use
        path = os.environ.get("DGAL_ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        i64, i32 = ctypes.c_int64, ctypes.c_int
        L.oracle_polygon_valid.argtypes = [_f64p, i32]
        L.oracle_polygon_valid.restype = i32
        L.oracle_polygon_statuses.argtypes = [i64, i64, _f32p, _u8p, i32, _u8p]
        L.oracle_polygon_statuses.restype = None
        _u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_simple_inter_area.argtypes = [_f64p, i32, _f64p, i32]
        L.oracle_simple_inter_area.restype = ctypes.c_double
        L.oracle_simple_iou_pairs.argtypes = ([i64, i64, _f32p, _u8p, i32, _f32p, _u8p, i32,
                                               _f64p, _u64p, _u64p, _u8p])
        L.oracle_simple_iou_pairs.restype = i64
        L.oracle_simple_iou_pairs_grad.argtypes = ([i64, i64, _f32p, _u8p, i32, _f32p, _u8p,
                                                    i32, _f64p, _f64p, _f64p])
        L.oracle_simple_iou_pairs_grad.restype = None
        L.oracle_simple_margins.argtypes = [i64, i64, _f32p, _u8p, i32, _f32p, _u8p, i32, _f64p]
        L.oracle_simple_margins.restype = None
        L.oracle_simple_valid.argtypes = [_f64p, i32]
        L.oracle_simple_valid.restype = i32
        L.oracle_simple_statuses.argtypes = [i64, i64, _f32p, _u8p, i32, _u8p]
        L.oracle_simple_statuses.restype = None
        L.oracle_intersect.argtypes = [_f64p, i32, _f64p, i32, _f64p, _u8p]
        L.oracle_intersect.restype = i32
        L.oracle_area.argtypes = [_f64p, i32]
        L.oracle_area.restype = ctypes.c_double
        L.oracle_clip_area.argtypes = [_f64p, i32, _f64p, i32]
        L.oracle_clip_area.restype = ctypes.c_double
        poly = [_f32p, _u8p, i32, _f32p, _f32p]
        L.oracle_iou_pairs.argtypes = [i64, i64] + poly + poly + [_f64p, _u8p, _u8p]
        L.oracle_iou_pairs.restype = i64
        L.oracle_iou_pairs_grad.argtypes = ([i64, i64] + poly + poly +
                                            [_f64p, _u8p, _u8p, _f64p, _f64p, _f64p, _f64p])
        L.oracle_iou_pairs_grad.restype = None
        L.oracle_iou_index_pairs.argtypes = ([i64, i64, _i64p, _i64p] + poly + poly +
                                             [_f64p, _u8p, _u8p])
        L.oracle_iou_index_pairs.restype = i64
        seg = [i32, _i64p, _i64p, _i64p, i32]
        L.oracle_iou_matrix.argtypes = seg + poly + poly + [_f64p]
        L.oracle_iou_matrix.restype = None
        L.oracle_iou_matrix_grad.argtypes = (seg + poly + poly +
                                             [_f64p, _f64p, _f64p, _f64p, _f64p, i64, i64])
        L.oracle_iou_matrix_grad.restype = None
        L.oracle_pair_margins.argtypes = [i64, i64, _f32p, _u8p, i32, _f32p, _u8p, i32, _f64p]
        L.oracle_pair_margins.restype = None
        p2 = [_f32p, _u8p, i32]
        L.oracle_intersect_pairs.argtypes = [i64, i64] + p2 + p2 + [_f64p, _u8p, _u8p]
        L.oracle_intersect_pairs.restype = i64
        L.oracle_intersect_pairs_grad.argtypes = ([i64, i64] + p2 + p2 +
                                                  [_f64p, _u8p, _u8p, _f64p, _f64p])
        L.oracle_intersect_pairs_grad.restype = None
        L.oracle_areas.argtypes = [i64, i64] + p2 + [_f64p]
        L.oracle_areas.restype = None
        L.oracle_areas_grad.argtypes = [i64, i64] + p2 + [_f64p, _f64p]
        L.oracle_areas_grad.restype = None
        L.oracle_iou_boxes.argtypes = [i64, i64, _f32p, _f32p, i32, _f64p, _u8p, _u8p]
        L.oracle_iou_boxes.restype = i64
        L.oracle_iou_boxes_grad.argtypes = [i64, i64, _f32p, _f32p, i32, _f64p, _u8p, _u8p,
                                            _f64p, _f64p]
        L.oracle_iou_boxes_grad.restype = None
        _lib = L
    return _lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _poly_args(xy, nv=None, zlo=None, zhi=None):
    xy = np.ascontiguousarray(xy, dtype=np.float32)
    assert xy.ndim == 3 and xy.shape[2] == 2
    k = xy.shape[1]
    if nv is not None:
        nv = np.ascontiguousarray(nv, dtype=np.uint8)
    if zlo is not None:
        zlo = np.ascontiguousarray(zlo, dtype=np.float32)
        zhi = np.ascontiguousarray(zhi, dtype=np.float32)
    keep = (xy, nv, zlo, zhi)
    return keep, [_p(xy, _f32p), _p(nv, _u8p), k, _p(zlo, _f32p), _p(zhi, _f32p)]


def _chunks(n, threads):
    threads = max(1, min(threads, n)) if n > 0 else 1
    step = (n + threads - 1) // threads
    return [(lo, min(n, lo + step)) for lo in range(0, n, step)] if n > 0 else []


def _run(fn, n, threads):
    parts = _chunks(n, threads)
    if threads <= 1 or len(parts) <= 1:
        return [fn(lo, hi) for lo, hi in parts]
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        return list(ex.map(lambda r: fn(*r), parts))


def iou_pairs(a_xy, b_xy, a_nv=None, b_nv=None, a_z=None, b_z=None, threads=1):
    """IoU of elementwise pairs (Sec. II-B listing, batched).

    a_z / b_z: optional (zlo, zhi) tuples of [n] fp32 arrays for 3D IoU.
    Returns (iou f64 [n], nx u8 [n], xflags u8 [n, ka+kb], n_invalid)."""
    ka_keep, ka_args = _poly_args(a_xy, a_nv, *(a_z or (None, None)))
    kb_keep, kb_args = _poly_args(b_xy, b_nv, *(b_z or (None, None)))
    n = ka_keep[0].shape[0]
    assert kb_keep[0].shape[0] == n
    cap = ka_keep[0].shape[1] + kb_keep[0].shape[1]
    iou = np.zeros(n, np.float64)
    nx = np.zeros(n, np.uint8)
    xf = np.full((n, cap), 0xFF, np.uint8)
    L = lib()
    bad = _run(lambda lo, hi: L.oracle_iou_pairs(lo, hi, *ka_args, *kb_args, _p(iou, _f64p),
                                                 _p(nx, _u8p), _p(xf, _u8p)), n, threads)
    return iou, nx, xf, int(sum(bad))


def iou_pairs_grad(a_xy, b_xy, g, nx, xflags, a_nv=None, b_nv=None, a_z=None, b_z=None,
                   threads=1):
    """Analytic gradient of sum(g * IoU) from the saved nx / xflags (Sec. II-B).

    Returns (ga [n,ka,2] f64, gb [n,kb,2] f64, gaz [n,2] or None, gbz or None)."""
    ka_keep, ka_args = _poly_args(a_xy, a_nv, *(a_z or (None, None)))
    kb_keep, kb_args = _poly_args(b_xy, b_nv, *(b_z or (None, None)))
    n, ka = ka_keep[0].shape[:2]
    kb = kb_keep[0].shape[1]
    g = np.ascontiguousarray(g, dtype=np.float64)
    nx = np.ascontiguousarray(nx, dtype=np.uint8)
    xflags = np.ascontiguousarray(xflags, dtype=np.uint8)
    assert xflags.shape == (n, ka + kb)
    ga = np.zeros((n, ka, 2), np.float64)
    gb = np.zeros((n, kb, 2), np.float64)
    gaz = np.zeros((n, 2), np.float64) if a_z is not None else None
    gbz = np.zeros((n, 2), np.float64) if a_z is not None else None
    L = lib()
    _run(lambda lo, hi: L.oracle_iou_pairs_grad(lo, hi, *ka_args, *kb_args, _p(g, _f64p),
                                                _p(nx, _u8p), _p(xflags, _u8p), _p(ga, _f64p),
                                                _p(gb, _f64p), _p(gaz, _f64p), _p(gbz, _f64p)),
         n, threads)
    return ga, gb, gaz, gbz


def iou_index_pairs(ia, ib, a_xy, b_xy, a_nv=None, b_nv=None, a_z=None, b_z=None,
                    threads=1):
    """IoU of (a[ia[t]], b[ib[t]]): sampled entries of a matrix."""
    ka_keep, ka_args = _poly_args(a_xy, a_nv, *(a_z or (None, None)))
    kb_keep, kb_args = _poly_args(b_xy, b_nv, *(b_z or (None, None)))
    ia = np.ascontiguousarray(ia, dtype=np.int64)
    ib = np.ascontiguousarray(ib, dtype=np.int64)
    n = ia.shape[0]
    cap = ka_keep[0].shape[1] + kb_keep[0].shape[1]
    iou = np.zeros(n, np.float64)
    nx = np.zeros(n, np.uint8)
    xf = np.full((n, cap), 0xFF, np.uint8)
    L = lib()
    _run(lambda lo, hi: L.oracle_iou_index_pairs(lo, hi, _p(ia, _i64p), _p(ib, _i64p), *ka_args,
                                                 *kb_args, _p(iou, _f64p), _p(nx, _u8p),
                                                 _p(xf, _u8p)), n, threads)
    return iou, nx, xf


def _seg_args(n_a, n_b, a_off, b_off, self_pairs):
    if a_off is None:
        a_off = np.array([0, n_a], np.int64)
        b_off = np.array([0, n_b], np.int64)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    sizes = (a_off[1:] - a_off[:-1]) * (b_off[1:] - b_off[:-1])
    out_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return a_off, b_off, out_off


def iou_matrix(a_xy, b_xy=None, a_nv=None, b_nv=None, a_z=None, b_z=None, a_off=None,
               b_off=None, self_pairs=False):
    """Segmented IoU matrix; returns (flat iou f64, out_off)."""
    if self_pairs:
        b_xy, b_nv, b_z, b_off = a_xy, a_nv, a_z, a_off
    ka_keep, ka_args = _poly_args(a_xy, a_nv, *(a_z or (None, None)))
    kb_keep, kb_args = _poly_args(b_xy, b_nv, *(b_z or (None, None)))
    a_off, b_off, out_off = _seg_args(ka_keep[0].shape[0], kb_keep[0].shape[0], a_off, b_off,
                                      self_pairs)
    iou = np.zeros(int(out_off[-1]), np.float64)
    lib().oracle_iou_matrix(len(a_off) - 1, _p(a_off, _i64p), _p(b_off, _i64p),
                            _p(out_off, _i64p), int(bool(self_pairs)), *ka_args, *kb_args,
                            _p(iou, _f64p))
    return iou, out_off


def iou_matrix_grad(g, a_xy, b_xy=None, a_nv=None, b_nv=None, a_z=None, b_z=None, a_off=None,
                    b_off=None, self_pairs=False):
    """Gradient of sum(g * IoU-matrix); returns (ga, gb, gaz, gbz); gb is None when
    self_pairs (everything accumulates into ga)."""
    if self_pairs:
        b_xy, b_nv, b_z, b_off = a_xy, a_nv, a_z, a_off
    ka_keep, ka_args = _poly_args(a_xy, a_nv, *(a_z or (None, None)))
    kb_keep, kb_args = _poly_args(b_xy, b_nv, *(b_z or (None, None)))
    n_a, ka = ka_keep[0].shape[:2]
    n_b, kb = kb_keep[0].shape[:2]
    a_off, b_off, out_off = _seg_args(n_a, n_b, a_off, b_off, self_pairs)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == (int(out_off[-1]),)
    ga = np.zeros((n_a, ka, 2), np.float64)
    gb = np.zeros((n_b, kb, 2), np.float64)
    gaz = np.zeros((n_a, 2), np.float64) if a_z is not None else None
    gbz = np.zeros((n_b, 2), np.float64) if a_z is not None else None
    lib().oracle_iou_matrix_grad(len(a_off) - 1, _p(a_off, _i64p), _p(b_off, _i64p),
                                 _p(out_off, _i64p), int(bool(self_pairs)), *ka_args, *kb_args,
                                 _p(g, _f64p), _p(ga, _f64p), _p(gb, _f64p), _p(gaz, _f64p),
                                 _p(gbz, _f64p), n_a, n_b)
    if self_pairs:
        return ga, None, gaz, None
    return ga, gb, gaz, gbz


def pair_margins(a_xy, b_xy, a_nv=None, b_nv=None, threads=1):
    """Degeneracy margins [n, 5] (see oracle_pair_margins)."""
    ka_keep, ka_args = _poly_args(a_xy, a_nv)
    kb_keep, kb_args = _poly_args(b_xy, b_nv)
    n = ka_keep[0].shape[0]
    out = np.zeros((n, 5), np.float64)
    L = lib()
    _run(lambda lo, hi: L.oracle_pair_margins(lo, hi, ka_args[0], ka_args[1], ka_args[2],
                                              kb_args[0], kb_args[1], kb_args[2],
                                              _p(out, _f64p)), n, threads)
    return out


# thresholds that define the generator-filtered (non-degenerate) parity set
FILTER_DELTA = 1e-4      # vertex/edge margin
FILTER_SIN = 1e-3        # crossing angle
FILTER_TURN = 1e-3       # polygon strict convexity
FILTER_GAP = 1e-4        # angular gap between ordered intersection vertices
FILTER_SLIVER = 1e-4     # intersection area / smaller polygon area (simple polygons only)


def filtered_mask(margins):
    """Pairs away from degeneracy by margins [0]..[3]; margin [4], the
    sliver ratio, is reported but no longer selects (thin intersections are
    computed to the bars by the library's fp64 rebuild)."""
    m = np.asarray(margins)
    return ((m[:, 0] >= FILTER_DELTA) & (m[:, 1] >= FILTER_SIN) & (m[:, 2] >= FILTER_TURN)
            & (m[:, 3] >= FILTER_GAP))


def polygon_valid(xy):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    return bool(lib().oracle_polygon_valid(_p(xy, _f64p), xy.shape[0]))


def polygon_status(xy, nv=None):
    """Input-contract status of each polygon of a [n, kmax, 2] fp32 array
    (Sec. III): 0 valid, 1 vertex count outside [3, kmax], 2 a turn not
    strictly left, 3 winds more than once.  uint8 [n]."""
    keep, args = _poly2(xy, nv)
    n = keep[0].shape[0]
    out = np.zeros(n, np.uint8)
    lib().oracle_polygon_statuses(0, n, *args, _p(out, _u8p))
    return out


def intersect(p, q):
    """Intersection polygon of one pair: (vertices [m,2] f64, codes [m] u8)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros((16, 2), np.float64)
    codes = np.zeros(16, np.uint8)
    m = lib().oracle_intersect(_p(p, _f64p), p.shape[0], _p(q, _f64p), q.shape[0],
                               _p(out, _f64p), _p(codes, _u8p))
    if m < 0:
        raise ValueError("intersection exceeds capacity (invalid polygon)")
    return out[:m].copy(), codes[:m].copy()


def area(xy):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    return lib().oracle_area(_p(xy, _f64p), xy.shape[0])


def clip_area(p, q):
    """Sutherland-Hodgman area of P clipped by Q (independent cross-check)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().oracle_clip_area(_p(p, _f64p), p.shape[0], _p(q, _f64p), q.shape[0])


def _f64_setup():
    L = lib()
    if not hasattr(L, "_f64_ready"):
        i64, i32 = ctypes.c_int64, ctypes.c_int
        L.oracle_iou_pairs_f64.argtypes = [i64, _f64p, i32, _f64p, _f64p, i32, _f64p, _f64p,
                                           _u8p, _u8p]
        L.oracle_iou_pairs_f64.restype = None
        L.oracle_iou_pairs_grad_f64.argtypes = [i64, _f64p, i32, _f64p, _f64p, i32, _f64p, _f64p,
                                                _u8p, _u8p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_iou_pairs_grad_f64.restype = None
        L._f64_ready = True
    return L


def iou_pairs_f64(a_xy, b_xy, a_z=None, b_z=None):
    """fp64-input IoU of pairs with full vertex counts; a_z/b_z are [n,2] (lo,hi)."""
    L = _f64_setup()
    a = np.ascontiguousarray(a_xy, np.float64)
    b = np.ascontiguousarray(b_xy, np.float64)
    n, ka = a.shape[:2]
    kb = b.shape[1]
    az = None if a_z is None else np.ascontiguousarray(a_z, np.float64)
    bz = None if b_z is None else np.ascontiguousarray(b_z, np.float64)
    iou = np.zeros(n)
    nx = np.zeros(n, np.uint8)
    xf = np.full((n, ka + kb), 0xFF, np.uint8)
    L.oracle_iou_pairs_f64(n, _p(a, _f64p), ka, _p(az, _f64p), _p(b, _f64p), kb, _p(bz, _f64p),
                           _p(iou, _f64p), _p(nx, _u8p), _p(xf, _u8p))
    return iou, nx, xf


def iou_pairs_grad_f64(a_xy, b_xy, g, nx, xflags, a_z=None, b_z=None):
    L = _f64_setup()
    a = np.ascontiguousarray(a_xy, np.float64)
    b = np.ascontiguousarray(b_xy, np.float64)
    n, ka = a.shape[:2]
    kb = b.shape[1]
    az = None if a_z is None else np.ascontiguousarray(a_z, np.float64)
    bz = None if b_z is None else np.ascontiguousarray(b_z, np.float64)
    g = np.ascontiguousarray(np.broadcast_to(g, (n,)), np.float64)
    nx = np.ascontiguousarray(nx, np.uint8)
    xflags = np.ascontiguousarray(xflags, np.uint8)
    ga = np.zeros((n, ka, 2))
    gb = np.zeros((n, kb, 2))
    gaz = np.zeros((n, 2))
    gbz = np.zeros((n, 2))
    L.oracle_iou_pairs_grad_f64(n, _p(a, _f64p), ka, _p(az, _f64p), _p(b, _f64p), kb,
                                _p(bz, _f64p), _p(g, _f64p), _p(nx, _u8p), _p(xflags, _u8p),
                                _p(ga, _f64p), _p(gb, _f64p), _p(gaz, _f64p), _p(gbz, _f64p))
    return ga, gb, gaz, gbz


def _poly2(xy, nv=None):
    xy = np.ascontiguousarray(xy, dtype=np.float32)
    assert xy.ndim == 3 and xy.shape[2] == 2
    if nv is not None:
        nv = np.ascontiguousarray(nv, dtype=np.uint8)
    return (xy, nv), [_p(xy, _f32p), _p(nv, _u8p), xy.shape[1]]


def intersect_pairs(a_xy, b_xy, a_nv=None, b_nv=None, threads=1):
    """Intersection polygons of elementwise pairs (Sec. III), fixed capacity
    ka + kb.  Returns (xy f64 [n, cap, 2] with slots >= nx zero, nx u8 [n],
    xflags u8 [n, cap], n_invalid)."""
    ka_keep, ka_args = _poly2(a_xy, a_nv)
    kb_keep, kb_args = _poly2(b_xy, b_nv)
    n = ka_keep[0].shape[0]
    assert kb_keep[0].shape[0] == n
    cap = ka_keep[0].shape[1] + kb_keep[0].shape[1]
    xy = np.zeros((n, cap, 2), np.float64)
    nx = np.zeros(n, np.uint8)
    xf = np.full((n, cap), 0xFF, np.uint8)
    L = lib()
    bad = _run(lambda lo, hi: L.oracle_intersect_pairs(lo, hi, *ka_args, *kb_args, _p(xy, _f64p),
                                                       _p(nx, _u8p), _p(xf, _u8p)), n, threads)
    return xy, nx, xf, int(sum(bad))


def intersect_pairs_grad(a_xy, b_xy, g_xy, nx, xflags, a_nv=None, b_nv=None, threads=1):
    """Gradient of sum <g_xy, X> over the saved intersection vertices with
    respect to both polygons.  Returns (ga [n,ka,2] f64, gb [n,kb,2] f64)."""
    ka_keep, ka_args = _poly2(a_xy, a_nv)
    kb_keep, kb_args = _poly2(b_xy, b_nv)
    n, ka = ka_keep[0].shape[:2]
    kb = kb_keep[0].shape[1]
    g = np.ascontiguousarray(g_xy, np.float64)
    assert g.shape == (n, ka + kb, 2)
    nx = np.ascontiguousarray(nx, np.uint8)
    xflags = np.ascontiguousarray(xflags, np.uint8)
    ga = np.zeros((n, ka, 2), np.float64)
    gb = np.zeros((n, kb, 2), np.float64)
    L = lib()
    _run(lambda lo, hi: L.oracle_intersect_pairs_grad(lo, hi, *ka_args, *kb_args, _p(g, _f64p),
                                                      _p(nx, _u8p), _p(xflags, _u8p),
                                                      _p(ga, _f64p), _p(gb, _f64p)), n, threads)
    return ga, gb


def areas(xy, nv=None):
    """Shoelace areas of [n, k, 2] fp32 polygons (Sec. III), f64 [n]."""
    keep, args = _poly2(xy, nv)
    n = keep[0].shape[0]
    out = np.zeros(n, np.float64)
    lib().oracle_areas(0, n, *args, _p(out, _f64p))
    return out


def areas_grad(xy, g, nv=None):
    """Gradient of sum(g * area) with respect to the vertices, f64 [n, k, 2]."""
    keep, args = _poly2(xy, nv)
    n, k = keep[0].shape[:2]
    g = np.ascontiguousarray(g, np.float64)
    out = np.zeros((n, k, 2), np.float64)
    lib().oracle_areas_grad(0, n, *args, _p(g, _f64p), _p(out, _f64p))
    return out


def iou_boxes(a, b, threads=1):
    """IoU of box pairs (Sec. IV-A): a, b are [n, 5] (cx, cy, w, l, yaw) or
    [n, 7] (+ z centre, h) fp32; corners formed in fp64.  Returns
    (iou f64 [n], nx u8 [n], xflags u8 [n, 8], n_invalid)."""
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    n, dim = a.shape
    assert b.shape == (n, dim) and dim in (5, 7)
    iou = np.zeros(n, np.float64)
    nx = np.zeros(n, np.uint8)
    xf = np.full((n, 8), 0xFF, np.uint8)
    L = lib()
    bad = _run(lambda lo, hi: L.oracle_iou_boxes(lo, hi, _p(a, _f32p), _p(b, _f32p), dim,
                                                 _p(iou, _f64p), _p(nx, _u8p), _p(xf, _u8p)),
               n, threads)
    return iou, nx, xf, int(sum(bad))


def iou_boxes_grad(a, b, g, nx, xflags, threads=1):
    """Gradient of sum(g * IoU) with respect to the box parameters, f64
    (ga [n, dim], gb [n, dim])."""
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    n, dim = a.shape
    g = np.ascontiguousarray(g, np.float64)
    nx = np.ascontiguousarray(nx, np.uint8)
    xflags = np.ascontiguousarray(xflags, np.uint8)
    ga = np.zeros((n, dim), np.float64)
    gb = np.zeros((n, dim), np.float64)
    L = lib()
    _run(lambda lo, hi: L.oracle_iou_boxes_grad(lo, hi, _p(a, _f32p), _p(b, _f32p), dim,
                                                _p(g, _f64p), _p(nx, _u8p), _p(xflags, _u8p),
                                                _p(ga, _f64p), _p(gb, _f64p)), n, threads)
    return ga, gb


# ------------------------------------------------ simple (non-convex) polygons

_u64p = ctypes.POINTER(ctypes.c_uint64)


def simple_inter_area(p, q):
    """Area of the intersection of two simple counter-clockwise polygons
    ([n, 2] each, fp64) by the vertical slab decomposition."""
    p = np.ascontiguousarray(p, np.float64)
    q = np.ascontiguousarray(q, np.float64)
    return float(lib().oracle_simple_inter_area(_p(p, _f64p), p.shape[0], _p(q, _f64p),
                                                q.shape[0]))


def simple_valid(xy):
    """True if the [n, 2] polygon is simple, counter-clockwise, 3..8 vertices."""
    xy = np.ascontiguousarray(xy, np.float64)
    return bool(lib().oracle_simple_valid(_p(xy, _f64p), xy.shape[0]))


def simple_status(xy, nv=None):
    """Simple-polygon contract status of each polygon of a [n, kmax, 2] fp32
    array: 0 valid, 1 vertex count outside [3, kmax], 2 edges meet or
    overlap, 3 area not positive (clockwise or flat).  uint8 [n]."""
    keep, args = _poly2(xy, nv)
    n = keep[0].shape[0]
    out = np.zeros(n, np.uint8)
    lib().oracle_simple_statuses(0, n, *args, _p(out, _u8p))
    return out


def simple_iou_pairs(a_xy, b_xy, a_nv=None, b_nv=None, threads=1):
    """IoU of elementwise pairs of simple polygons and the saved state.
    Returns (iou f64 [n], xmask u64 [n], smask u64 [n], inside u8 [n],
    n_invalid)."""
    ka_keep, ka_args = _poly2(a_xy, a_nv)
    kb_keep, kb_args = _poly2(b_xy, b_nv)
    n = ka_keep[0].shape[0]
    assert kb_keep[0].shape[0] == n
    iou = np.zeros(n, np.float64)
    xm = np.zeros(n, np.uint64)
    sm = np.zeros(n, np.uint64)
    ins = np.zeros(n, np.uint8)
    L = lib()
    bad = _run(lambda lo, hi: L.oracle_simple_iou_pairs(lo, hi, *ka_args, *kb_args,
                                                        _p(iou, _f64p), _p(xm, _u64p),
                                                        _p(sm, _u64p), _p(ins, _u8p)),
               n, threads)
    return iou, xm, sm, ins, int(sum(bad))


def simple_iou_pairs_grad(a_xy, b_xy, g, a_nv=None, b_nv=None, threads=1):
    """Gradient of sum(g * IoU) over pairs of simple polygons: (ga, gb) f64."""
    ka_keep, ka_args = _poly2(a_xy, a_nv)
    kb_keep, kb_args = _poly2(b_xy, b_nv)
    n, ka = ka_keep[0].shape[:2]
    kb = kb_keep[0].shape[1]
    g = np.ascontiguousarray(g, np.float64)
    ga = np.zeros((n, ka, 2), np.float64)
    gb = np.zeros((n, kb, 2), np.float64)
    L = lib()
    _run(lambda lo, hi: L.oracle_simple_iou_pairs_grad(lo, hi, *ka_args, *kb_args, _p(g, _f64p),
                                                       _p(ga, _f64p), _p(gb, _f64p)), n, threads)
    return ga, gb


def simple_margins(a_xy, b_xy, a_nv=None, b_nv=None, threads=1):
    """[n, 3]: vertex-to-edge distance over the pair's size, smallest |sin| of
    a crossing, intersection area over the smaller polygon's (1 if
    disjoint)."""
    ka_keep, ka_args = _poly2(a_xy, a_nv)
    kb_keep, kb_args = _poly2(b_xy, b_nv)
    n = ka_keep[0].shape[0]
    out = np.zeros((n, 3), np.float64)
    L = lib()
    _run(lambda lo, hi: L.oracle_simple_margins(lo, hi, *ka_args, *kb_args, _p(out, _f64p)),
         n, threads)
    return out


def simple_filtered_mask(margins, dist=1e-4, sin=1e-3, sliver=1e-4):
    """Pairs in general position: no vertex within dist * size of an edge of
    the other polygon, no crossing at |sin| below sin, and no intersection
    smaller than sliver times the smaller polygon (the convex filter's
    criteria)."""
    return (margins[:, 0] >= dist) & (margins[:, 1] >= sin) & (margins[:, 2] >= sliver)
