"""Batched, differentiable convex-polygon IoU on MI355X (gfx950).

Thin ctypes binding over the C ABI in include/dgal.h (libdgal.so, built by
paper_2011_11134_amd/build.py): argument marshalling only; every step of the
computation runs in the library's HIP kernels on torch's current stream.
There is no CPU fallback: without the built library the import fails.

Paper: Y. Zhong, "Differentiable Computational Geometry for 2D and 3D machine
learning", arXiv 2011.11134 (Sec. II-B listing: IoU with saved nx / xflags and
its gradient; Sec. III: convex CCW polygons in fixed-capacity arrays; Sec.
IV-A: rotated 2D/3D box IoU).
"""
import atexit
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgal.so")

DGAL_OK, DGAL_EINVAL, DGAL_ECAPACITY, DGAL_EHIP, DGAL_EIO = 0, -1, -2, -3, -4
DGAL_PAIRS, DGAL_MATRIX = 0, 1
MAX_SEGMENTS = 4096
TILE_PAIRS = 2048                 # pairs per matrix tile: rows x (TILE_PAIRS // rows)
TILE_ROWS_CHOICES = (4, 8, 16)    # tile shapes the matrix forward can use
TILE_ROWS_DEFAULT = 8
TILE_MASK_WORDS = TILE_PAIRS // 64 + 2  # survivor bits, tile origin, row length

_vp = ctypes.c_void_p


class Polys(ctypes.Structure):
    """dgal_polys"""
    _fields_ = [("xy", _vp), ("nv", _vp), ("zlo", _vp), ("zhi", _vp),
                ("count", ctypes.c_int64), ("kmax", ctypes.c_int32)]


class Saved(ctypes.Structure):
    """dgal_saved"""
    _fields_ = [("pair_id", _vp), ("nx", _vp), ("xflags", _vp),
                ("capacity", ctypes.c_int64), ("count", _vp),
                ("tile_start", _vp), ("tile_count", _vp), ("tile_capacity", ctypes.c_int64),
                ("tile_mask", _vp), ("tile_rows", ctypes.c_int32), ("seg_prefix", _vp)]


class Boxes(ctypes.Structure):
    """dgal_boxes"""
    _fields_ = [("p", _vp), ("count", ctypes.c_int64), ("dim", ctypes.c_int32)]


EXPORTS = ("dgal_create", "dgal_destroy", "dgal_status_string", "dgal_check",
           "dgal_iou_pairs", "dgal_iou_matrix", "dgal_iou_matrix_noalloc", "dgal_iou_backward",
           "dgal_intersect", "dgal_intersect_backward", "dgal_area", "dgal_area_backward",
           "dgal_iou_boxes", "dgal_iou_boxes_backward", "dgal_set_autotune",
           "dgal_autotune_report", "dgal_validate", "dgal_set_validate",
           "dgal_iou_simple_pairs", "dgal_iou_simple_backward", "dgal_validate_simple",
           "dgal_set_profiling", "dgal_profile_report", "dgal_set_path_stats",
           "dgal_path_stats", "dgal_tune_cache_load", "dgal_tune_cache_save",
           "dgal_tune_cache_report", "dgal_tune_cache_clear")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python {_HERE}/build.py` "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.dgal_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
    L.dgal_create.restype = ctypes.c_int
    L.dgal_destroy.argtypes = [_vp]
    L.dgal_destroy.restype = None
    L.dgal_status_string.argtypes = [ctypes.c_int]
    L.dgal_status_string.restype = ctypes.c_char_p
    L.dgal_check.argtypes = [_vp, _vp]
    L.dgal_check.restype = ctypes.c_int
    L.dgal_iou_pairs.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, _vp]
    L.dgal_iou_pairs.restype = ctypes.c_int
    L.dgal_iou_matrix.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, i32, i32, _vp, i64,
                                  ctypes.POINTER(Saved), _vp]
    L.dgal_iou_matrix.restype = ctypes.c_int
    L.dgal_iou_matrix_noalloc.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, i32, i32, _vp, i64,
                                          _vp]
    L.dgal_iou_matrix_noalloc.restype = ctypes.c_int
    L.dgal_iou_backward.argtypes = [_vp, i32, Polys, Polys, _vp, _vp, _vp, i32, i32, _vp, i64,
                                    _vp, _vp, ctypes.POINTER(Saved), _vp, _vp, _vp, _vp, _vp]
    L.dgal_iou_backward.restype = ctypes.c_int
    L.dgal_intersect.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, _vp]
    L.dgal_intersect.restype = ctypes.c_int
    L.dgal_intersect_backward.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, _vp, _vp, _vp]
    L.dgal_intersect_backward.restype = ctypes.c_int
    L.dgal_area.argtypes = [_vp, Polys, _vp, _vp]
    L.dgal_area.restype = ctypes.c_int
    L.dgal_area_backward.argtypes = [_vp, Polys, _vp, _vp, _vp]
    L.dgal_area_backward.restype = ctypes.c_int
    L.dgal_iou_boxes.argtypes = [_vp, Boxes, Boxes, _vp, _vp, _vp, _vp]
    L.dgal_iou_boxes.restype = ctypes.c_int
    L.dgal_iou_boxes_backward.argtypes = [_vp, Boxes, Boxes, _vp, _vp, _vp, _vp, _vp, _vp]
    L.dgal_iou_boxes_backward.restype = ctypes.c_int
    L.dgal_set_autotune.argtypes = [_vp, i32]
    L.dgal_set_autotune.restype = ctypes.c_int
    L.dgal_autotune_report.argtypes = [_vp, ctypes.c_char_p, i64]
    L.dgal_autotune_report.restype = ctypes.c_int
    L.dgal_tune_cache_load.argtypes = [ctypes.c_char_p]
    L.dgal_tune_cache_load.restype = ctypes.c_int
    L.dgal_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.dgal_tune_cache_save.restype = ctypes.c_int
    L.dgal_tune_cache_report.argtypes = [ctypes.c_char_p, i64]
    L.dgal_tune_cache_report.restype = ctypes.c_int
    L.dgal_tune_cache_clear.argtypes = []
    L.dgal_tune_cache_clear.restype = ctypes.c_int
    L.dgal_set_path_stats.argtypes = [_vp, i32]
    L.dgal_set_path_stats.restype = ctypes.c_int
    L.dgal_path_stats.argtypes = [_vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(i64), _vp]
    L.dgal_path_stats.restype = ctypes.c_int
    L.dgal_set_profiling.argtypes = [_vp, i32]
    L.dgal_set_profiling.restype = ctypes.c_int
    L.dgal_profile_report.argtypes = [_vp, ctypes.c_char_p, i64]
    L.dgal_profile_report.restype = ctypes.c_int
    L.dgal_validate.argtypes = [_vp, Polys, _vp, _vp, _vp]
    L.dgal_validate.restype = ctypes.c_int
    L.dgal_validate_simple.argtypes = [_vp, Polys, _vp, _vp, _vp]
    L.dgal_validate_simple.restype = ctypes.c_int
    L.dgal_set_validate.argtypes = [_vp, i32]
    L.dgal_set_validate.restype = ctypes.c_int
    L.dgal_iou_simple_pairs.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, _vp, _vp]
    L.dgal_iou_simple_pairs.restype = ctypes.c_int
    L.dgal_iou_simple_backward.argtypes = [_vp, Polys, Polys, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.dgal_iou_simple_backward.restype = ctypes.c_int
    return L


lib = _load()
_ctx = {}


def _destroy_all():
    for c in _ctx.values():
        lib.dgal_destroy(c)
    _ctx.clear()


atexit.register(_destroy_all)


class DgalError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {lib.dgal_status_string(status).decode()}")
        self.status = status


def _ok(status, what):
    if status != DGAL_OK:
        raise DgalError(status, what)


def context(device=None):
    """The library context of a CUDA/HIP device (created once)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    c = _ctx.get(idx)
    if c is None:
        h = _vp()
        _ok(lib.dgal_create(ctypes.byref(h), idx), "dgal_create")
        c = h.value
        _ctx[idx] = c
    return c


def _stream(t):
    return torch.cuda.current_stream(t.device).cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _need(t, dtype, name, dev=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dev is not None and t.device != dev:
        raise ValueError(f"{name} is on {t.device}, expected {dev}")
    return t


def polys(xy, nv=None, z=None):
    """Describes [n, kmax, 2] fp32 polygons (+ optional [n] uint8 counts and a
    (zlo, zhi) pair of [n] fp32 tensors) as a dgal_polys; returns (struct, keep)."""
    _need(xy, torch.float32, "xy")
    if xy.dim() != 3 or xy.shape[2] != 2:
        raise ValueError("polygons must be [n, kmax, 2]")
    n, k = xy.shape[0], xy.shape[1]
    if nv is not None:
        _need(nv, torch.uint8, "nv", xy.device)
        if nv.shape != (n,):
            raise ValueError("nv must be [n]")
    zlo = zhi = None
    if z is not None:
        zlo, zhi = z
        _need(zlo, torch.float32, "zlo", xy.device)
        _need(zhi, torch.float32, "zhi", xy.device)
        if zlo.shape != (n,) or zhi.shape != (n,):
            raise ValueError("zlo / zhi must be [n]")
    s = Polys(_ptr(xy), _ptr(nv), _ptr(zlo), _ptr(zhi), n, k)
    return s, (xy, nv, zlo, zhi)


# --------------------------------------------------------------------- pairs

def iou_pairs(a_xy, b_xy, a_nv=None, b_nv=None, a_z=None, b_z=None, save=True):
    """IoU of elementwise pairs (Sec. II-B listing, batched).

    Returns (iou [n] fp32, nx [n] uint8, xflags [n, ka+kb] uint8); nx and
    xflags are None when save is False."""
    pa, ka = polys(a_xy, a_nv, a_z)
    pb, kb = polys(b_xy, b_nv, b_z)
    n = a_xy.shape[0]
    dev = a_xy.device
    iou = torch.empty(n, dtype=torch.float32, device=dev)
    nx = xf = None
    if save:
        nx = torch.empty(n, dtype=torch.uint8, device=dev)
        xf = torch.empty((n, a_xy.shape[1] + b_xy.shape[1]), dtype=torch.uint8, device=dev)
    _ok(lib.dgal_iou_pairs(context(dev), pa, pb, _ptr(iou), _ptr(nx), _ptr(xf), _stream(a_xy)),
        "dgal_iou_pairs")
    return iou, nx, xf


def iou_pairs_backward(a_xy, b_xy, grad, nx, xflags, a_nv=None, b_nv=None, a_z=None, b_z=None):
    """Gradient of sum(grad * IoU) from the saved nx / xflags (Sec. II-B
    `iou_grad`).  Returns (grad_a [n,ka,2], grad_b [n,kb,2], grad_a_z [n,2] or
    None, grad_b_z [n,2] or None); z gradients are (d/dzlo, d/dzhi)."""
    pa, ka = polys(a_xy, a_nv, a_z)
    pb, kb = polys(b_xy, b_nv, b_z)
    dev = a_xy.device
    _need(grad, torch.float32, "grad", dev)
    _need(nx, torch.uint8, "nx", dev)
    _need(xflags, torch.uint8, "xflags", dev)
    ga = torch.empty_like(a_xy)
    gb = torch.empty_like(b_xy)
    gaz = gbz = None
    if a_z is not None:
        gaz = torch.empty((a_xy.shape[0], 2), dtype=torch.float32, device=dev)
        gbz = torch.empty((b_xy.shape[0], 2), dtype=torch.float32, device=dev)
    _ok(lib.dgal_iou_backward(context(dev), DGAL_PAIRS, pa, pb, None, None, None, 0, 0, _ptr(grad),
                              0, _ptr(nx), _ptr(xflags), None, _ptr(ga), _ptr(gb), _ptr(gaz),
                              _ptr(gbz), _stream(a_xy)),
        "dgal_iou_backward(pairs)")
    return ga, gb, gaz, gbz


# ------------------------------------------------------------ primitives

def intersect(a_xy, b_xy, a_nv=None, b_nv=None):
    """Intersection polygons of elementwise pairs (Sec. II-B / III).

    Returns (xy [n, ka+kb, 2] fp32 counter-clockwise from the smallest code,
    0 past nx; nx [n] uint8; xflags [n, ka+kb] uint8)."""
    pa, ka = polys(a_xy, a_nv)
    pb, kb = polys(b_xy, b_nv)
    n, cap = a_xy.shape[0], a_xy.shape[1] + b_xy.shape[1]
    dev = a_xy.device
    xy = torch.empty((n, cap, 2), dtype=torch.float32, device=dev)
    nx = torch.empty(n, dtype=torch.uint8, device=dev)
    xf = torch.empty((n, cap), dtype=torch.uint8, device=dev)
    _ok(lib.dgal_intersect(context(dev), pa, pb, _ptr(xy), _ptr(nx), _ptr(xf), _stream(a_xy)),
        "dgal_intersect")
    return xy, nx, xf


def intersect_backward(a_xy, b_xy, grad_xy, nx, xflags, a_nv=None, b_nv=None):
    """Gradient of sum(grad_xy * xy) with respect to both polygons, from the
    saved nx / xflags.  Returns (grad_a [n,ka,2], grad_b [n,kb,2])."""
    pa, ka = polys(a_xy, a_nv)
    pb, kb = polys(b_xy, b_nv)
    dev = a_xy.device
    _need(grad_xy, torch.float32, "grad_xy", dev)
    _need(nx, torch.uint8, "nx", dev)
    _need(xflags, torch.uint8, "xflags", dev)
    if grad_xy.shape != (a_xy.shape[0], a_xy.shape[1] + b_xy.shape[1], 2):
        raise ValueError("grad_xy must be [n, ka+kb, 2]")
    ga = torch.empty_like(a_xy)
    gb = torch.empty_like(b_xy)
    _ok(lib.dgal_intersect_backward(context(dev), pa, pb, _ptr(grad_xy), _ptr(nx), _ptr(xflags),
                                    _ptr(ga), _ptr(gb), _stream(a_xy)),
        "dgal_intersect_backward")
    return ga, gb


def area(xy, nv=None):
    """Shoelace areas (Sec. III) of [n, k, 2] fp32 polygons: [n] fp32."""
    p, keep = polys(xy, nv)
    out = torch.empty(xy.shape[0], dtype=torch.float32, device=xy.device)
    _ok(lib.dgal_area(context(xy.device), p, _ptr(out), _stream(xy)), "dgal_area")
    return out


def area_backward(xy, grad, nv=None):
    """Gradient of sum(grad * area) with respect to the vertices: [n, k, 2]."""
    p, keep = polys(xy, nv)
    _need(grad, torch.float32, "grad", xy.device)
    out = torch.empty_like(xy)
    _ok(lib.dgal_area_backward(context(xy.device), p, _ptr(grad), _ptr(out), _stream(xy)),
        "dgal_area_backward")
    return out


# ------------------------------------------------------------- boxes

def _boxes(p, name):
    _need(p, torch.float32, name)
    if p.dim() != 2 or p.shape[1] not in (5, 7):
        raise ValueError(f"{name} must be [n, 5] (cx, cy, w, l, yaw) or [n, 7] (+ z, h)")
    return Boxes(_ptr(p), p.shape[0], p.shape[1])


def iou_boxes(a, b, save=True):
    """IoU of box pairs given as parameter rows (Sec. IV-A), corners formed
    in-kernel.  Returns (iou [n], nx [n] or None, xflags [n, 8] or None)."""
    ba, bb = _boxes(a, "a"), _boxes(b, "b")
    dev = a.device
    n = a.shape[0]
    iou = torch.empty(n, dtype=torch.float32, device=dev)
    nx = xf = None
    if save:
        nx = torch.empty(n, dtype=torch.uint8, device=dev)
        xf = torch.empty((n, 8), dtype=torch.uint8, device=dev)
    _ok(lib.dgal_iou_boxes(context(dev), ba, bb, _ptr(iou), _ptr(nx), _ptr(xf), _stream(a)),
        "dgal_iou_boxes")
    return iou, nx, xf


def iou_boxes_backward(a, b, grad, nx, xflags):
    """Gradient of sum(grad * IoU) with respect to the box parameters:
    (grad_a [n, dim], grad_b [n, dim])."""
    ba, bb = _boxes(a, "a"), _boxes(b, "b")
    dev = a.device
    _need(grad, torch.float32, "grad", dev)
    _need(nx, torch.uint8, "nx", dev)
    _need(xflags, torch.uint8, "xflags", dev)
    ga = torch.empty_like(a)
    gb = torch.empty_like(b)
    _ok(lib.dgal_iou_boxes_backward(context(dev), ba, bb, _ptr(grad), _ptr(nx), _ptr(xflags),
                                    _ptr(ga), _ptr(gb), _stream(a)),
        "dgal_iou_boxes_backward")
    return ga, gb


# --------------------------------------------------------------------- matrix

class SavedPairs:
    """Device buffers of a dgal_saved work list (pairs that survived the cull
    of a matrix forward, with their nx / xflags) and its per-tile table."""

    def __init__(self, capacity, cap, tiles, device, tile_rows=0):
        self.pair_id = torch.empty(capacity, dtype=torch.int64, device=device)
        self.nx = torch.empty(capacity, dtype=torch.uint8, device=device)
        self.xflags = torch.empty((capacity, cap), dtype=torch.uint8, device=device)
        # reset by the forward's own kernel (graph replays included)
        self.count = torch.empty(1, dtype=torch.int64, device=device)
        self.tile_start = torch.empty(max(tiles, 1), dtype=torch.int64, device=device)
        self.tile_count = torch.empty(max(tiles, 1), dtype=torch.int32, device=device)
        self.tile_mask = torch.empty((max(tiles, 1), TILE_MASK_WORDS), dtype=torch.int64,
                                     device=device)
        # the segments' prefixes, written by the forward and reused by the backward
        self.seg_prefix = torch.empty(2 * (MAX_SEGMENTS + 1), dtype=torch.int64, device=device)
        self.capacity = capacity
        self.tiles = tiles
        self.tiles_used = 0  # tiles of the last forward (set by iou_matrix)
        # 0: the forward picks the tile shape (autotuned, else the default)
        # and records it here for the backward
        self.tile_rows = tile_rows

    def struct(self):
        return Saved(_ptr(self.pair_id), _ptr(self.nx), _ptr(self.xflags), self.capacity,
                     _ptr(self.count), _ptr(self.tile_start), _ptr(self.tile_count), self.tiles,
                     _ptr(self.tile_mask), self.tile_rows, _ptr(self.seg_prefix))


def segments(n_a, n_b, a_off, b_off=None, self_pairs=False, device=None):
    """Device segment table for iou_matrix: (a_off, b_off, out_off, nseg,
    total output size, tile capacity (the most tiles over the tile shapes),
    {tile rows: tile count}).  Build it before a HIP-graph capture and pass it as
    `seg=` (the table itself needs host-to-device copies)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    return _segments(n_a, n_b, a_off, b_off, self_pairs, dev)


def _segments(n_a, n_b, a_off, b_off, self_pairs, dev):
    """Device offsets (a_off, b_off, out_off) and total output size."""
    if a_off is None:
        by = {r: ((-(-n_a // r)) * (-(-n_b // (TILE_PAIRS // r))) if n_a and n_b else 0)
              for r in TILE_ROWS_CHOICES}
        return None, None, None, 0, n_a * n_b, max(by.values()), by
    a_off = torch.as_tensor(a_off, dtype=torch.int64)
    b_off = a_off if (self_pairs or b_off is None) else torch.as_tensor(b_off, dtype=torch.int64)
    a_cpu, b_cpu = a_off.cpu(), b_off.cpu()
    sizes = (a_cpu[1:] - a_cpu[:-1]) * (b_cpu[1:] - b_cpu[:-1])
    out_off = torch.cat([torch.zeros(1, dtype=torch.int64), torch.cumsum(sizes, 0)[:-1]])
    total = int(sizes.sum())
    nseg = int(a_cpu.numel() - 1)
    if not 1 <= nseg <= MAX_SEGMENTS:
        raise ValueError(f"1..{MAX_SEGMENTS} segments supported, got {nseg}")
    na = a_cpu[1:] - a_cpu[:-1]
    nb = b_cpu[1:] - b_cpu[:-1]
    by = {r: int(torch.where(sizes > 0, ((na + r - 1) // r) *
                             ((nb + TILE_PAIRS // r - 1) // (TILE_PAIRS // r)), 0).sum())
          for r in TILE_ROWS_CHOICES}
    return (a_off.to(dev).contiguous(), b_off.to(dev).contiguous(), out_off.to(dev).contiguous(),
            nseg, total, max(by.values()), by)


def iou_matrix(a_xy, b_xy=None, a_nv=None, b_nv=None, a_z=None, b_z=None, a_off=None, b_off=None,
               self_pairs=False, save=False, capacity=None, check=True, seg=None, saved=None):
    """IoU matrix (one a x b block, or segments such as per-scene self pairs).

    Returns (iou, saved, seg): iou is [na, nb] for one block or flat
    (blocks concatenated row-major) with segments; saved is the SavedPairs
    work list (the backward's state; None when save=False); seg is the tuple
    of device offsets.  capacity bounds the survivors of the cull; exceeding
    a given one raises (check=True).  By default it is max(65536, pairs / 16),
    and (check=True) a call that finds more survivors is repeated once with
    room for all of them.

    Capturable use (a HIP graph, or a loop that must not synchronise): pass
    `seg` from segments() and a SavedPairs as `saved` (reused, nothing is
    allocated for it), with check=False; an overflow is then reported by the
    next check_errors()."""
    if self_pairs:
        b_xy, b_nv, b_z, b_off = a_xy, a_nv, a_z, a_off
    pa, ka = polys(a_xy, a_nv, a_z)
    pb, kb = polys(b_xy, b_nv, b_z)
    dev = a_xy.device
    if seg is None:
        seg = _segments(a_xy.shape[0], b_xy.shape[0], a_off, b_off, self_pairs, dev)
    d_a, d_b, d_o, nseg, total, tiles, tiles_by = seg
    iou = torch.empty(total, dtype=torch.float32, device=dev)
    given = saved
    sized = capacity is not None or given is not None
    if capacity is None:
        capacity = given.capacity if given is not None else max(1 << 16, total // 16)
    cap_codes = a_xy.shape[1] + b_xy.shape[1]
    if given is not None and (given.tiles < tiles or given.xflags.shape[1] != cap_codes):
        raise ValueError(f"saved holds {given.tiles} tiles of {given.xflags.shape[1]} codes; "
                         f"this call needs {tiles} tiles of {cap_codes}")

    def run(cap):
        sv = given if given is not None else SavedPairs(cap, cap_codes, tiles, dev)
        st = sv.struct()
        _ok(lib.dgal_iou_matrix(context(dev), pa, pb, _ptr(d_a), _ptr(d_b), _ptr(d_o), nseg,
                                int(bool(self_pairs)), _ptr(iou), total, ctypes.byref(st),
                                _stream(a_xy)),
            "dgal_iou_matrix")
        sv.tile_rows = st.tile_rows  # the shape the forward used, for the backward
        sv.tiles_used = tiles_by[sv.tile_rows]
        return sv

    if check:
        check_errors(dev)  # an earlier call's deferred error is its own, raised here
    saved = run(capacity)
    if check:
        try:
            check_errors(dev)
        except DgalError as e:
            # a default capacity too small for this input: the count holds how
            # many pairs survived the cull, so the call is repeated once with
            # room for all of them.  Any other error (an intersection over its
            # capacity, rejected offsets) is raised.
            if sized or e.status != DGAL_ECAPACITY:
                raise
            cnt = int(saved.count.item())
            if cnt <= saved.capacity:
                raise
            saved = run(cnt)
            check_errors(dev)
    if d_a is None:
        iou = iou.view(a_xy.shape[0], b_xy.shape[0])
    return iou, (saved if save else None), (d_a, d_b, d_o, nseg)


def iou_matrix_backward(grad, saved, seg, a_xy, b_xy=None, a_nv=None, b_nv=None, a_z=None,
                        b_z=None, self_pairs=False):
    """Gradient of sum(grad * IoU-matrix) from the saved list.  Returns
    (grad_a, grad_b, grad_a_z, grad_b_z); with self_pairs everything is in
    grad_a / grad_a_z and the b entries are None."""
    if self_pairs:
        b_xy, b_nv, b_z = a_xy, a_nv, a_z
    pa, ka = polys(a_xy, a_nv, a_z)
    pb, kb = polys(b_xy, b_nv, b_z)
    dev = a_xy.device
    grad = _need(grad.contiguous(), torch.float32, "grad", dev)
    d_a, d_b, d_o, nseg = seg
    ga = torch.empty_like(a_xy)
    gb = None if self_pairs else torch.empty_like(b_xy)
    gaz = gbz = None
    if a_z is not None:
        gaz = torch.empty((a_xy.shape[0], 2), dtype=torch.float32, device=dev)
        gbz = None if self_pairs else torch.empty((b_xy.shape[0], 2), dtype=torch.float32,
                                                  device=dev)
    st = saved.struct()
    _ok(lib.dgal_iou_backward(context(dev), DGAL_MATRIX, pa, pb, _ptr(d_a), _ptr(d_b), _ptr(d_o),
                              nseg, int(bool(self_pairs)), _ptr(grad), grad.numel(), None, None,
                              ctypes.byref(st), _ptr(ga), _ptr(gb), _ptr(gaz), _ptr(gbz),
                              _stream(a_xy)),
        "dgal_iou_backward(matrix)")
    return ga, gb, gaz, gbz


def iou_simple_pairs(a_xy, b_xy, a_nv=None, b_nv=None, save=True):
    """IoU of elementwise pairs of simple (not necessarily convex) polygons.
    Returns (iou [n], xmask, smask, inside): the saved state as int64 [n]
    tensors holding the uint64 masks, and uint8 [n]; None when save=False."""
    pa, _ = polys(a_xy, a_nv)
    pb, _ = polys(b_xy, b_nv)
    n, dev = a_xy.shape[0], a_xy.device
    iou = torch.empty(n, dtype=torch.float32, device=dev)
    xm = sm = ins = None
    if save:
        xm = torch.empty(n, dtype=torch.int64, device=dev)
        sm = torch.empty(n, dtype=torch.int64, device=dev)
        ins = torch.empty(n, dtype=torch.uint8, device=dev)
    _ok(lib.dgal_iou_simple_pairs(context(dev), pa, pb, _ptr(iou), _ptr(xm), _ptr(sm), _ptr(ins),
                                  _stream(a_xy)), "dgal_iou_simple_pairs")
    return iou, xm, sm, ins


def iou_simple_backward(a_xy, b_xy, grad, xmask, smask, inside, a_nv=None, b_nv=None):
    """Gradient of sum(grad * IoU) for simple polygon pairs from the saved
    state: (grad_a [n, ka, 2], grad_b [n, kb, 2])."""
    pa, _ = polys(a_xy, a_nv)
    pb, _ = polys(b_xy, b_nv)
    dev = a_xy.device
    _need(grad, torch.float32, "grad", dev)
    _need(xmask, torch.int64, "xmask", dev)
    _need(smask, torch.int64, "smask", dev)
    _need(inside, torch.uint8, "inside", dev)
    ga = torch.empty_like(a_xy)
    gb = torch.empty_like(b_xy)
    _ok(lib.dgal_iou_simple_backward(context(dev), pa, pb, _ptr(grad), _ptr(xmask), _ptr(smask),
                                     _ptr(inside), _ptr(ga), _ptr(gb), _stream(a_xy)),
        "dgal_iou_simple_backward")
    return ga, gb


def validate(xy, nv=None):
    """Input-contract status of each polygon (Sec. III), checked on the GPU:
    (status uint8 [n]: 0 valid, 1 vertex count outside [3, kmax], 2 a turn
    not strictly left, 3 winds more than once; number of invalid polygons)."""
    p, keep = polys(xy, nv)
    n = xy.shape[0]
    status = torch.empty(n, dtype=torch.uint8, device=xy.device)
    n_bad = torch.empty(1, dtype=torch.int64, device=xy.device)
    _ok(lib.dgal_validate(context(xy.device), p, _ptr(status), _ptr(n_bad), _stream(xy)),
        "dgal_validate")
    return status, int(n_bad.item())


def validate_simple(xy, nv=None):
    """Simple-polygon contract status of each polygon, checked on the GPU:
    (status uint8 [n]: 0 valid, 1 vertex count outside [3, kmax], 2 edges
    meet or overlap, 3 area not positive; number of invalid polygons)."""
    p, keep = polys(xy, nv)
    n = xy.shape[0]
    status = torch.empty(n, dtype=torch.uint8, device=xy.device)
    n_bad = torch.empty(1, dtype=torch.int64, device=xy.device)
    _ok(lib.dgal_validate_simple(context(xy.device), p, _ptr(status), _ptr(n_bad), _stream(xy)),
        "dgal_validate_simple")
    return status, int(n_bad.item())


def set_validate(enable=True, device=None):
    """Turns the input check before every call on (or off) for a device's
    context; while on, a call with an invalid polygon raises DgalError
    (DGAL_EINVAL) and enqueues nothing."""
    _ok(lib.dgal_set_validate(context(device), int(bool(enable))), "dgal_set_validate")


def set_autotune(enable=True, device=None):
    """Enables (or disables) launch-shape autotuning on a device's context:
    the next call of each kind times its candidate grids once (synchronising)
    and keeps the fastest."""
    _ok(lib.dgal_set_autotune(context(device), int(bool(enable))), "dgal_set_autotune")


def tune_cache_load(path):
    """Merges a tune-cache JSON file into the process-wide store of tuned
    launch shapes; returns the number of entries read."""
    n = lib.dgal_tune_cache_load(os.fsencode(path))
    if n < 0:
        raise DgalError(n, "dgal_tune_cache_load")
    return n


def tune_cache_save(path):
    """Writes the process-wide store of tuned launch shapes to a JSON file."""
    _ok(lib.dgal_tune_cache_save(os.fsencode(path)), "dgal_tune_cache_save")


def tune_cache_report():
    """The store's entries, one line each (key, shape, timed milliseconds)."""
    need = 1 << 16
    while True:
        buf = ctypes.create_string_buffer(need)
        n = lib.dgal_tune_cache_report(buf, need)
        if n < 0:
            raise DgalError(n, "dgal_tune_cache_report")
        text = buf.value.decode()
        if text.count("\n") >= n or need >= 1 << 26:
            return text
        need *= 4


def tune_cache_clear():
    lib.dgal_tune_cache_clear()


def autotune_report(device=None):
    """(number of tuned kinds, text with one line per kind)."""
    buf = ctypes.create_string_buffer(8192)
    n = lib.dgal_autotune_report(context(device), buf, len(buf))
    if n < 0:
        raise DgalError(n, "dgal_autotune_report")
    return n, buf.value.decode()


def set_profiling(enable=True, device=None):
    """Per-kernel timing on a device's context (every launch waited for: a
    measuring aid, not for graph capture); enabling resets the totals."""
    _ok(lib.dgal_set_profiling(context(device), int(bool(enable))), "dgal_set_profiling")


def profile_report(device=None):
    """{kernel: (launches, total ms)} timed since profiling was enabled."""
    buf = ctypes.create_string_buffer(8192)
    n = lib.dgal_profile_report(context(device), buf, len(buf))
    if n < 0:
        raise DgalError(n, "dgal_profile_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, launches, ms = line.split()
        out[name] = (int(launches), float(ms))
    return out


def set_path_stats(enable=True, device=None):
    """Counting, on the device, of the pairs the forward kernels evaluate, of
    those whose orientation signs took the fp64 path, and of those whose
    areas were rebuilt in fp64 (thin pairs)."""
    _ok(lib.dgal_set_path_stats(context(device), int(bool(enable))), "dgal_set_path_stats")


def path_stats(device=None):
    """(pairs evaluated, pairs with fp64 signs, pairs with fp64 areas) since
    the last read; clears them."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    n, k, t = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _ok(lib.dgal_path_stats(context(dev), ctypes.byref(n), ctypes.byref(k), ctypes.byref(t),
                            torch.cuda.current_stream(dev).cuda_stream), "dgal_path_stats")
    return int(n.value), int(k.value), int(t.value)


def check_errors(device=None):
    """Synchronises torch's current stream and raises on a deferred device error."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    st = lib.dgal_check(context(dev), torch.cuda.current_stream(dev).cuda_stream)
    _ok(st, "deferred device error")


# --------------------------------------------------------------------- autograd

class IoUPairs(torch.autograd.Function):
    """IoU of elementwise polygon pairs; backward by the library's kernel from
    the saved nx / xflags (no re-intersection)."""

    @staticmethod
    def forward(ctx, a_xy, b_xy, a_nv=None, b_nv=None):
        iou, nx, xf = iou_pairs(a_xy, b_xy, a_nv, b_nv, save=True)
        ctx.save_for_backward(a_xy, b_xy, nx, xf)
        ctx.nvs = (a_nv, b_nv)
        ctx.mark_non_differentiable(nx, xf)
        return iou

    @staticmethod
    def backward(ctx, g):
        a_xy, b_xy, nx, xf = ctx.saved_tensors
        a_nv, b_nv = ctx.nvs
        ga, gb, _, _ = iou_pairs_backward(a_xy, b_xy, g.contiguous().float(), nx, xf, a_nv, b_nv)
        return ga, gb, None, None


class IoUSimplePairs(torch.autograd.Function):
    """IoU of elementwise pairs of simple (not necessarily convex) polygons;
    backward by the library's kernel from the saved crossing state."""

    @staticmethod
    def forward(ctx, a_xy, b_xy, a_nv=None, b_nv=None):
        iou, xm, sm, ins = iou_simple_pairs(a_xy, b_xy, a_nv, b_nv, save=True)
        ctx.save_for_backward(a_xy, b_xy, xm, sm, ins)
        ctx.nvs = (a_nv, b_nv)
        return iou

    @staticmethod
    def backward(ctx, g):
        a_xy, b_xy, xm, sm, ins = ctx.saved_tensors
        a_nv, b_nv = ctx.nvs
        ga, gb = iou_simple_backward(a_xy, b_xy, g.contiguous().float(), xm, sm, ins, a_nv, b_nv)
        return ga, gb, None, None


class Intersect(torch.autograd.Function):
    """Intersection polygons of elementwise pairs; returns (xy, nx, xflags),
    differentiable in xy (backward from the saved codes)."""

    @staticmethod
    def forward(ctx, a_xy, b_xy, a_nv=None, b_nv=None):
        xy, nx, xf = intersect(a_xy, b_xy, a_nv, b_nv)
        ctx.save_for_backward(a_xy, b_xy, nx, xf)
        ctx.nvs = (a_nv, b_nv)
        ctx.mark_non_differentiable(nx, xf)
        return xy, nx, xf

    @staticmethod
    def backward(ctx, g, _gnx=None, _gxf=None):
        a_xy, b_xy, nx, xf = ctx.saved_tensors
        a_nv, b_nv = ctx.nvs
        ga, gb = intersect_backward(a_xy, b_xy, g.contiguous().float(), nx, xf, a_nv, b_nv)
        return ga, gb, None, None


class Area(torch.autograd.Function):
    """Polygon areas, differentiable in the vertices."""

    @staticmethod
    def forward(ctx, xy, nv=None):
        ctx.save_for_backward(xy)
        ctx.nv = nv
        return area(xy, nv)

    @staticmethod
    def backward(ctx, g):
        (xy,) = ctx.saved_tensors
        return area_backward(xy, g.contiguous().float(), ctx.nv), None


class IoUBoxes(torch.autograd.Function):
    """IoU of box pairs from their parameters (2D [n, 5] or 3D [n, 7]);
    backward down to the parameters."""

    @staticmethod
    def forward(ctx, a, b):
        iou, nx, xf = iou_boxes(a, b, save=True)
        ctx.save_for_backward(a, b, nx, xf)
        return iou

    @staticmethod
    def backward(ctx, g):
        a, b, nx, xf = ctx.saved_tensors
        ga, gb = iou_boxes_backward(a, b, g.contiguous().float(), nx, xf)
        return ga, gb


class IoU3DPairs(torch.autograd.Function):
    """3D IoU (BEV polygon intersection x z-overlap) of elementwise pairs."""

    @staticmethod
    def forward(ctx, a_xy, a_zlo, a_zhi, b_xy, b_zlo, b_zhi):
        iou, nx, xf = iou_pairs(a_xy, b_xy, a_z=(a_zlo, a_zhi), b_z=(b_zlo, b_zhi), save=True)
        ctx.save_for_backward(a_xy, a_zlo, a_zhi, b_xy, b_zlo, b_zhi, nx, xf)
        return iou

    @staticmethod
    def backward(ctx, g):
        a_xy, a_zlo, a_zhi, b_xy, b_zlo, b_zhi, nx, xf = ctx.saved_tensors
        ga, gb, gaz, gbz = iou_pairs_backward(a_xy, b_xy, g.contiguous().float(), nx, xf,
                                              a_z=(a_zlo, a_zhi), b_z=(b_zlo, b_zhi))
        return ga, gaz[:, 0], gaz[:, 1], gb, gbz[:, 0], gbz[:, 1]


class IoUMatrix(torch.autograd.Function):
    """IoU matrix of two polygon sets; backward from the saved non-empty pairs.

    apply(a_xy, b_xy, capacity=None, work=None): `work` = (seg, saved) from
    segments() and a SavedPairs makes the forward capturable (no allocation
    for the work list, no synchronisation; overflows are reported by
    check_errors())."""

    @staticmethod
    def forward(ctx, a_xy, b_xy, capacity=None, work=None):
        seg, sv = (None, None) if work is None else work
        iou, saved, seg = iou_matrix(a_xy, b_xy, save=True, capacity=capacity,
                                     check=work is None, seg=seg, saved=sv)
        ctx.saved_list = saved
        ctx.seg = seg
        ctx.save_for_backward(a_xy, b_xy)
        return iou

    @staticmethod
    def backward(ctx, g):
        a_xy, b_xy = ctx.saved_tensors
        ga, gb, _, _ = iou_matrix_backward(g.contiguous().float().reshape(-1), ctx.saved_list,
                                           ctx.seg, a_xy, b_xy)
        return ga, gb, None, None


class IoU3DScenes(torch.autograd.Function):
    """Per-scene self-pairwise 3D IoU of boxes (BEV polygons with z-extents);
    scene s holds boxes off[s]..off[s+1] and owns a block of the flat output
    (its diagonal is 1 with zero gradient; entries (r, c) and (c, r) are one
    unordered pair, the lower index evaluated first).

    apply(xy, zlo, zhi, off, capacity=None, work=None): `work` = (seg, saved)
    from segments(..., self_pairs=True) and a SavedPairs makes the forward
    capturable in a HIP graph (no allocation for the work list, no
    synchronisation; overflows are reported by check_errors())."""

    @staticmethod
    def forward(ctx, xy, zlo, zhi, off, capacity=None, work=None):
        seg, sv = (None, None) if work is None else work
        iou, saved, seg = iou_matrix(xy, a_z=(zlo, zhi), a_off=off, self_pairs=True, save=True,
                                     capacity=capacity, check=work is None, seg=seg, saved=sv)
        ctx.saved_list = saved
        ctx.seg = seg
        ctx.save_for_backward(xy, zlo, zhi)
        return iou

    @staticmethod
    def backward(ctx, g):
        xy, zlo, zhi = ctx.saved_tensors
        ga, _, gaz, _ = iou_matrix_backward(g.contiguous().float(), ctx.saved_list, ctx.seg, xy,
                                            a_z=(zlo, zhi), self_pairs=True)
        return ga, gaz[:, 0], gaz[:, 1], None, None, None
