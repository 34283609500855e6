#!/usr/bin/env python3
"""Throughput benchmark of the batched differentiable convex-polygon IoU path
on one MI355X.

A step is one pass of the whole path over one batch of synthetic inputs that
are resident in HBM before timing starts:
  c5 (default): 64 scenes of U{50..2000} 3D boxes, per-scene self-pair IoU
                (~94 M pairs), forward (cull, work list, exact pairs) and
                backward from the saved work list: the largest workload, and
                the one the pairs/s metric is quoted on;
  c3:           1,048,576 rotated-rectangle pairs, forward (IoU + saved nx /
                xflags) and backward (gradients for both boxes) kernels;
  c1 / c4:      the same on 1,024 rectangle pairs / 262,144 mixed 3..8-gon pairs;
  c2:           4096 x 4096 IoU matrix, forward;
  c3b:          c3's pairs as box-parameter rows (corners formed in-kernel),
                forward and backward to the parameters;
  c3i:          the exported intersection primitive on c3's pairs (ordered
                polygons, nx, xflags) and its backward;
  c4n:          262,144 pairs of simple, generally non-convex 3..8-gons,
                forward and backward.
Prints one JSON line (rank 0, one GPU).  The timed region is `steps` steps
back to back: replays of one captured HIP graph of the step (--eager: the
library's calls launched one by one).  Kernel durations for the roofline come
from the library's per-kernel timing mode (HIP events on the launch stream
around each kernel), run after the timed region.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "IoU pairs/s fwd+bwd fp32 (≤1e-5 vs FP64 oracle), fused batched vs plain"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3

# Algorithmic bytes per pair (inputs read + outputs written, nothing else):
#   rectangles, forward:  2 x 32 B vertices + 4 B IoU + 1 B nx + 8 B flags  = 77
#   rectangles, backward: 2 x 32 B vertices + 4 B grad + 1 B nx + 8 B flags
#                         + 2 x 32 B gradients                                = 141
#   8-slot polygons:      2 x (64 + 1) B vertices and counts; flags 16 B
#   boxes by parameters:  2 x 20 B (cx, cy, w, l, yaw) + 13 B  /  + 4 + 9 + 2 x 20 B
#   intersection primitive (rectangles), forward: 2 x 32 B vertices + 8 x 8 B
#                         ordered vertices + 1 B nx + 8 B flags              = 137
#                         backward: 2 x 32 B vertices + 8 x 8 B vertex
#                         gradients + 9 B saved + 2 x 32 B gradients         = 201
#   simple polygons:      2 x (64 + 1) B + 4 B IoU + 17 B saved (two uint64
#                         masks, one inclusion byte)  /  + 4 + 17 + 2 x 64 B
BYTES = {
    ("rect", "fwd"): 77, ("rect", "bwd"): 141,
    ("simple", "fwd"): 130 + 4 + 17, ("simple", "bwd"): 130 + 4 + 17 + 128,
    ("box", "fwd"): 53, ("box", "bwd"): 93,
    ("isect", "fwd"): 137, ("isect", "bwd"): 201,
    ("poly", "fwd"): 130 + 4 + 1 + 16, ("poly", "bwd"): 130 + 4 + 1 + 16 + 128,
}
# Algorithmic fp32 operations per rectangle pair (FMA = 2), counted from the
# method's arithmetic: forward 128 for the 32 orientations, 16 for the edges,
# ~28 for ~4 crossings, ~100 for the centroid, angle keys and shoelace of ~6
# vertices, ~30 for the areas and the IoU (~320); backward ~420 (rebuild of
# ~6 vertices, shoelace gradient, chain rule of ~4 crossings, areas).
FLOPS = {("rect", "fwd"): 320, ("rect", "bwd"): 420}


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c4", "c5", "c3b", "c3i", "c4n"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true", help="skip the plain per-op GPU form")
    p.add_argument("--copy-calib-mib", type=int, default=0,
                   help="also run a plain device copy of this size (HBM counter calibration)")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the built-in launch shapes (default: the library's autotuner "
                        "picks them during the warm-up)")
    p.add_argument("--eager", action="store_true",
                   help="launch the step's calls one by one instead of replaying a captured "
                        "HIP graph of the step")
    p.add_argument("--graph", action="store_true", help="(the default) replay a HIP graph")
    return p.parse_args()


def source_digest():
    """Digest of the kernel sources, to tell whether stored counter readings
    still describe the kernels being timed."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2011_11134_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's reading), or
    None when the kernel sources have changed since the counters were read."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    ent = rec.get("launches", {}).get(f"{workload}/{kernel}")
    return None if ent is None else int(ent["bytes"])


def _elementwise_bytes(kind, kernel, pairs):
    """(bound, algorithmic bytes per launch, basis) of an elementwise kernel:
    its inputs read once and its outputs written once (the BYTES table)."""
    direction = kernel.rsplit("_", 1)[-1]
    per = BYTES.get((kind, direction))
    if per is None:
        return "hbm", 0, f"{kernel}: not priced"
    return "hbm", per * pairs, f"{per} B per pair x {pairs} pairs"


class PairsStep:
    """Forward + backward of elementwise pairs with fixed device buffers."""

    def __init__(self, dg, torch, d):
        self.dg = dg
        self.a = torch.from_numpy(d["a_xy"]).cuda()
        self.b = torch.from_numpy(d["b_xy"]).cuda()
        self.anv = None if d.get("a_nv") is None else torch.from_numpy(d["a_nv"]).cuda()
        self.bnv = None if d.get("b_nv") is None else torch.from_numpy(d["b_nv"]).cuda()
        self.g = torch.from_numpy(d["grad"]).cuda()
        n, ka = self.a.shape[:2]
        kb = self.b.shape[1]
        self.n = n
        self.iou = torch.empty(n, device="cuda")
        self.nx = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.xf = torch.empty((n, ka + kb), dtype=torch.uint8, device="cuda")
        self.ga = torch.empty_like(self.a)
        self.gb = torch.empty_like(self.b)
        self.pa, _ = dg.polys(self.a, self.anv)
        self.pb, _ = dg.polys(self.b, self.bnv)
        self.ctx = dg.context()
        self.kind = "rect" if ka == 4 and self.anv is None else "poly"
        self.pairs = n

    def algorithmic_bytes(self, kernel):
        return _elementwise_bytes(self.kind, kernel, self.pairs)

    def fwd(self, stream):
        st = self.dg.lib.dgal_iou_pairs(self.ctx, self.pa, self.pb, self.iou.data_ptr(),
                                        self.nx.data_ptr(), self.xf.data_ptr(), stream)
        assert st == 0, st

    def bwd(self, stream):
        dg = self.dg
        st = dg.lib.dgal_iou_backward(self.ctx, dg.DGAL_PAIRS, self.pa, self.pb, None, None, None, 0,
                                      0, self.g.data_ptr(), 0, self.nx.data_ptr(),
                                      self.xf.data_ptr(), None, self.ga.data_ptr(),
                                      self.gb.data_ptr(), None, None, stream)
        assert st == 0, st


class BoxesStep:
    """Forward + backward of box pairs given by their parameters (corners
    formed in-kernel), fixed device buffers."""

    def __init__(self, dg, torch, d):
        self.dg = dg
        self.a = torch.from_numpy(d["a_box"]).cuda()
        self.b = torch.from_numpy(d["b_box"]).cuda()
        self.g = torch.from_numpy(d["grad"]).cuda()
        n, dim = self.a.shape
        self.n = self.pairs = n
        self.iou = torch.empty(n, device="cuda")
        self.nx = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.xf = torch.empty((n, 8), dtype=torch.uint8, device="cuda")
        self.ga = torch.empty_like(self.a)
        self.gb = torch.empty_like(self.b)
        self.ba = dg.Boxes(self.a.data_ptr(), n, dim)
        self.bb = dg.Boxes(self.b.data_ptr(), n, dim)
        self.ctx = dg.context()
        self.kind = "box"

    def algorithmic_bytes(self, kernel):
        return _elementwise_bytes(self.kind, kernel, self.pairs)

    def fwd(self, stream):
        st = self.dg.lib.dgal_iou_boxes(self.ctx, self.ba, self.bb, self.iou.data_ptr(),
                                        self.nx.data_ptr(), self.xf.data_ptr(), stream)
        assert st == 0, st

    def bwd(self, stream):
        st = self.dg.lib.dgal_iou_boxes_backward(self.ctx, self.ba, self.bb, self.g.data_ptr(),
                                                 self.nx.data_ptr(), self.xf.data_ptr(),
                                                 self.ga.data_ptr(), self.gb.data_ptr(), stream)
        assert st == 0, st


class IntersectStep:
    """The exported intersection primitive on rectangle pairs: ordered
    intersection polygons with nx / xflags, then the gradient of
    sum <grad_xy, polygon> back to both inputs, fixed device buffers."""

    def __init__(self, dg, torch, d):
        self.dg = dg
        self.a = torch.from_numpy(d["a_xy"]).cuda()
        self.b = torch.from_numpy(d["b_xy"]).cuda()
        self.g = torch.from_numpy(d["grad_xy"]).cuda()
        n, ka = self.a.shape[:2]
        cap = ka + self.b.shape[1]
        self.n = self.pairs = n
        self.xy = torch.empty((n, cap, 2), device="cuda")
        self.nx = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.xf = torch.empty((n, cap), dtype=torch.uint8, device="cuda")
        self.ga = torch.empty_like(self.a)
        self.gb = torch.empty_like(self.b)
        self.pa, _ = dg.polys(self.a)
        self.pb, _ = dg.polys(self.b)
        self.ctx = dg.context()
        self.kind = "isect"

    def algorithmic_bytes(self, kernel):
        return _elementwise_bytes(self.kind, kernel, self.pairs)

    def fwd(self, stream):
        st = self.dg.lib.dgal_intersect(self.ctx, self.pa, self.pb, self.xy.data_ptr(),
                                        self.nx.data_ptr(), self.xf.data_ptr(), stream)
        assert st == 0, st

    def bwd(self, stream):
        st = self.dg.lib.dgal_intersect_backward(self.ctx, self.pa, self.pb, self.g.data_ptr(),
                                                 self.nx.data_ptr(), self.xf.data_ptr(),
                                                 self.ga.data_ptr(), self.gb.data_ptr(), stream)
        assert st == 0, st


class SimpleStep:
    """Forward + backward of simple (not necessarily convex) polygon pairs
    with fixed device buffers."""

    def __init__(self, dg, torch, d):
        self.dg = dg
        self.a = torch.from_numpy(d["a_xy"]).cuda()
        self.b = torch.from_numpy(d["b_xy"]).cuda()
        self.anv = torch.from_numpy(d["a_nv"]).cuda()
        self.bnv = torch.from_numpy(d["b_nv"]).cuda()
        self.g = torch.from_numpy(d["grad"]).cuda()
        n = self.a.shape[0]
        self.n = self.pairs = n
        self.iou = torch.empty(n, device="cuda")
        self.xm = torch.empty(n, dtype=torch.int64, device="cuda")
        self.sm = torch.empty(n, dtype=torch.int64, device="cuda")
        self.ins = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.ga = torch.empty_like(self.a)
        self.gb = torch.empty_like(self.b)
        self.pa, _ = dg.polys(self.a, self.anv)
        self.pb, _ = dg.polys(self.b, self.bnv)
        self.ctx = dg.context()
        self.kind = "simple"

    def algorithmic_bytes(self, kernel):
        return _elementwise_bytes(self.kind, kernel, self.pairs)

    def fwd(self, stream):
        st = self.dg.lib.dgal_iou_simple_pairs(self.ctx, self.pa, self.pb, self.iou.data_ptr(),
                                               self.xm.data_ptr(), self.sm.data_ptr(),
                                               self.ins.data_ptr(), stream)
        assert st == 0, st

    def bwd(self, stream):
        st = self.dg.lib.dgal_iou_simple_backward(self.ctx, self.pa, self.pb, self.g.data_ptr(),
                                                  self.xm.data_ptr(), self.sm.data_ptr(),
                                                  self.ins.data_ptr(), self.ga.data_ptr(),
                                                  self.gb.data_ptr(), stream)
        assert st == 0, st


class MatrixStep:
    """4096 x 4096 IoU matrix (forward only) or per-scene 3D self pairs
    (forward + backward) with fixed device buffers."""

    def __init__(self, dg, torch, d, wl):
        self.dg = dg
        self.wl = wl
        self.a = torch.from_numpy(d["a_xy"]).cuda()
        self.ctx = dg.context()
        if wl == "c2":
            self.b = torch.from_numpy(d["b_xy"]).cuda()
            self.pa, _ = dg.polys(self.a)
            self.pb, _ = dg.polys(self.b)
            self.total = self.a.shape[0] * self.b.shape[0]
            self.seg = (None, None, None, 0)
            tiles = dg.segments(len(self.a), len(self.b), None)[5]
            # the forward's work list (survivors of the cull)
            self.saved = dg.SavedPairs(max(1 << 16, self.total // 16), 8, tiles, self.a.device)
            self.self_pairs = 0
        else:
            self.lo = torch.from_numpy(d["a_zlo"]).cuda()
            self.hi = torch.from_numpy(d["a_zhi"]).cuda()
            self.pa, _ = dg.polys(self.a, None, (self.lo, self.hi))
            self.pb = self.pa
            d_a, d_b, d_o, nseg, total, tiles, _ = dg.segments(len(self.a), len(self.a), d["off"],
                                                               self_pairs=True)
            self.seg = (d_a, d_b, d_o, nseg)
            self.total = total
            self.saved = dg.SavedPairs(max(1 << 16, total // 16), 8, tiles, self.a.device)
            self.g = torch.from_numpy(d["grad"]).cuda()
            self.ga = torch.empty_like(self.a)
            self.gz = torch.empty((len(self.a), 2), device="cuda")
            self.self_pairs = 1
        self.iou = torch.empty(self.total, device="cuda")
        self.pairs = self.total
        self.kind = "matrix"
        self.has_bwd = wl == "c5"

    def _p(self, t):
        return None if t is None else t.data_ptr()

    def algorithmic_bytes(self, kernel):
        """(bound, bytes per launch, basis): what each kernel of the matrix
        path must read and write at least, every input once.  A box is
        32 B of corners (+ 8 B of z-extent in 3D); a saved work-list entry is
        an 8 B pair id, 1 B nx and 8 B of flags."""
        box = 32 + (8 if self.self_pairs else 0)
        boxes = len(self.a) + (0 if self.self_pairs else len(self.b))
        surv = int(self.saved.count.item())
        g_reads = 8 if self.self_pairs else 4  # the entry's g (and its transpose's)
        if kernel == "k_matrix_cull":
            return ("hbm", 4 * self.pairs + box * boxes,
                    f"4 B of output per pair x {self.pairs} pairs + {box} B x {boxes} boxes")
        if kernel == "k_matrix_exact":
            return ("hbm", 21 * surv + box * boxes,
                    f"21 B per survivor (8 id + 4 IoU + 1 nx + 8 flags) x {surv} + "
                    f"{box} B x {boxes} boxes")
        if kernel == "k_matrix_fill":
            return "hbm", 8 * surv, f"8 B pair id per survivor x {surv}"
        if kernel == "k_matrix_bwd":
            per = 17 + g_reads
            return ("hbm", per * surv + 2 * box * boxes,
                    f"{per} B per survivor (17 saved + {g_reads} upstream) x {surv} + "
                    f"2 x {box} B (read, written) x {boxes} boxes")
        return "hbm", 0, f"{kernel}: not priced"

    def fwd(self, stream):
        dg = self.dg
        d_a, d_b, d_o, nseg = self.seg
        st_s = self.saved.struct()
        st = dg.lib.dgal_iou_matrix(self.ctx, self.pa, self.pb, self._p(d_a), self._p(d_b),
                                    self._p(d_o), nseg, self.self_pairs, self.iou.data_ptr(),
                                    self.total, dg.ctypes.byref(st_s), stream)
        assert st == 0, st
        self.saved.tile_rows = st_s.tile_rows  # the tile shape used, for the backward

    def bwd(self, stream):
        dg = self.dg
        d_a, d_b, d_o, nseg = self.seg
        st_s = self.saved.struct()
        st = dg.lib.dgal_iou_backward(self.ctx, dg.DGAL_MATRIX, self.pa, self.pb, d_a.data_ptr(),
                                      d_b.data_ptr(), d_o.data_ptr(), nseg, 1, self.g.data_ptr(),
                                      self.total, None, None, dg.ctypes.byref(st_s),
                                      self.ga.data_ptr(), None, self.gz.data_ptr(), None, stream)
        assert st == 0, st


def plain_baseline(torch, d, wl, steps=5, warmup=2):
    """The plain per-op GPU form (torch ops + autograd) on the same workload:
    forward + backward pairs/s.  Scenes: each scene's pairs formed by
    broadcasting, one scene at a time (bench_plain.iou3d_scenes_plain)."""
    from bench_plain import iou3d_scenes_plain, iou_pairs_plain
    if wl == "c5":
        xy = torch.from_numpy(d["a_xy"]).cuda().requires_grad_(True)
        lo = torch.from_numpy(d["a_zlo"]).cuda().requires_grad_(True)
        hi = torch.from_numpy(d["a_zhi"]).cuda().requires_grad_(True)
        g = torch.from_numpy(d["grad"]).cuda()
        off = d["off"]
        pairs = int(d["out_off"][-1])

        def step():
            for t in (xy, lo, hi):
                t.grad = None
            iou3d_scenes_plain(xy, lo, hi, off).backward(g)
    else:
        a = torch.from_numpy(d["a_xy"]).cuda().requires_grad_(True)
        b = torch.from_numpy(d["b_xy"]).cuda().requires_grad_(True)
        anv = None if d.get("a_nv") is None else torch.from_numpy(d["a_nv"]).cuda()
        bnv = None if d.get("b_nv") is None else torch.from_numpy(d["b_nv"]).cuda()
        g = torch.from_numpy(d["grad"]).cuda()
        pairs = len(d["a_xy"])

        def step():
            a.grad = None
            b.grad = None
            iou = iou_pairs_plain(a, b, anv, bnv)
            iou.backward(g)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    form = "torch ops + autograd on the GPU (bench_plain.py)"
    if wl == "c5":
        form += ", every ordered pair of a scene by broadcasting, scene by scene"
    return {"value": round(pairs / (ms * 1e-3), 1), "unit": "pairs/s",
            "ms_per_step": round(ms, 4), "steps": steps, "form": form}


def _timed_runs(fn, min_s=1.0):
    """Median wall time of fn() over at least 3 runs and min_s seconds."""
    times = []
    start = time.perf_counter()
    while len(times) < 3 or time.perf_counter() - start < min_s:
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return statistics.median(times), len(times)


def cpu_baseline(d, wl, kind):
    """The FP64 oracle, as it stands, on the host cores, on the workload or a
    bounded sample of it: forward + analytic backward (forward only for the
    c2 matrix), repeated for at least 1 s of wall time (at least 3 runs),
    median run, as pairs/s; on the host's cores (up to 16 threads, the
    batch split in contiguous ranges) and on one thread."""
    import oracle
    cores = max(1, min(16, os.cpu_count() or 1))
    if kind in ("rect", "poly"):
        a, b, g = d["a_xy"], d["b_xy"], d["grad"]
        anv, bnv = d.get("a_nv"), d.get("b_nv")

        def run(threads):
            iou, nx, xf, _ = oracle.iou_pairs(a, b, anv, bnv, threads=threads)
            oracle.iou_pairs_grad(a, b, g, nx, xf, anv, bnv, threads=threads)
        pairs, what = len(a), f"whole workload ({len(a)} pairs, forward + backward)"
    elif kind == "box":
        a, b, g = d["a_box"], d["b_box"], d["grad"]

        def run(threads):
            iou, nx, xf, _ = oracle.iou_boxes(a, b, threads=threads)
            oracle.iou_boxes_grad(a, b, g, nx, xf, threads=threads)
        pairs, what = len(a), f"whole workload ({len(a)} box pairs, forward + backward)"
    elif kind == "simple":
        a, b, g, anv, bnv = d["a_xy"], d["b_xy"], d["grad"], d["a_nv"], d["b_nv"]

        def run(threads):
            oracle.simple_iou_pairs(a, b, anv, bnv, threads=threads)
            oracle.simple_iou_pairs_grad(a, b, g, anv, bnv, threads=threads)
        pairs, what = len(a), f"whole workload ({len(a)} simple polygon pairs, forward + backward)"
    elif kind == "isect":
        a, b, g = d["a_xy"], d["b_xy"], d["grad_xy"]

        def run(threads):
            xy, nx, xf, _ = oracle.intersect_pairs(a, b, threads=threads)
            oracle.intersect_pairs_grad(a, b, g, nx, xf, threads=threads)
        pairs, what = len(a), f"whole workload ({len(a)} pairs, intersection + backward)"
    elif wl == "c2":
        # the oracle's matrix routine runs on one thread: the first 128 rows
        # against all 4096 columns
        cores = 1
        a, b = d["a_xy"][:128], d["b_xy"]

        def run(threads):
            oracle.iou_matrix(a, b)
        pairs, what = len(a) * len(b), f"rows 0..127 x {len(b)} columns of the matrix, forward"
    else:
        return _cpu_baseline_scenes(d)
    t, runs = _timed_runs(lambda: run(cores))
    out = {"value": round(pairs / t, 1), "unit": "pairs/s", "cores": cores, "kind": "oracle",
           "sample": f"{what} x {runs} runs, median {t:.4f} s per run",
           "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}
    if cores > 1:
        t1, r1 = _timed_runs(lambda: run(1))
        out["value_1_thread"] = round(pairs / t1, 1)
        out["sample_1_thread"] = f"the same on one thread x {r1} runs, median {t1:.4f} s"
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _cpu_baseline_scenes(d, frac=0.1, seed=2011):
    """The oracle's per-scene self-pair matrix, forward + analytic backward,
    on a seeded sample of the scenes (10% of them, or one per host thread up
    to 16 if that is more; every pair of each sampled scene), run on one
    thread and on the host's cores (the sampled scenes in parallel, one per
    thread; ctypes releases the GIL), at least 3 runs each, median; pairs/s
    scales linearly to the whole workload (each pair costs the same on
    average, independent of its scene)."""
    import numpy as np

    import oracle
    from concurrent.futures import ThreadPoolExecutor
    off, xy, lo, hi, g = d["off"], d["a_xy"], d["a_zlo"], d["a_zhi"], d["grad"]
    out_off = d["out_off"]
    nsc = len(off) - 1
    host = max(1, min(os.cpu_count() or 1, 16))
    pick = np.sort(np.random.default_rng(seed).choice(
        nsc, min(nsc, max(1, round(frac * nsc), host)), replace=False))
    jobs = []
    for s in pick:
        o0, o1 = int(off[s]), int(off[s + 1])
        jobs.append((xy[o0:o1], (lo[o0:o1], hi[o0:o1]), np.array([0, o1 - o0], np.int64),
                     g[out_off[s]:out_off[s + 1]]))
    pairs = int(sum((off[s + 1] - off[s]) ** 2 for s in pick))

    def one(job):
        x, z, o, gg = job
        oracle.iou_matrix(x, a_z=z, a_off=o, self_pairs=True)
        oracle.iou_matrix_grad(gg, x, a_z=z, a_off=o, self_pairs=True)

    def serial():
        for j in jobs:
            one(j)

    threads = max(1, min(len(jobs), host))

    def parallel():
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, jobs))

    t1, r1 = _timed_runs(serial, min_s=0.0)
    tn, rn = _timed_runs(parallel, min_s=0.0)
    return {"value": round(pairs / tn, 1), "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": (f"seeded {len(pick)} of the {nsc} scenes ({pairs} self pairs), "
                       f"forward + backward, one scene per thread, x {rn} runs, median "
                       f"{tn:.3f} s per run; scales to the whole workload by pairs"),
            "value_1_thread": round(pairs / t1, 1),
            "sample_1_thread": f"the same sample on one thread x {r1} runs, median {t1:.3f} s",
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def filter_stats(d, wl, step, sample=65536, seed=2012):
    """Rejection rate of the degeneracy filter that defines the parity set (the
    oracle's five margins: vertex-to-edge distance, crossing angle, polygon
    turn, angular gap of the intersection's vertices, sliver ratio) on a
    seeded sample of the workload's pairs; for the matrices, of the pairs
    that survived the cull (every other pair is disjoint).  Host-side, after
    the timed region."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(seed)
    anv = bnv = None
    if wl in ("c2", "c5"):
        pid = step.saved.pair_id[:int(step.saved.count.item())].cpu().numpy()
        pid = np.sort(rng.choice(pid, min(sample, len(pid)), replace=False))
        if wl == "c2":
            nb = len(d["b_xy"])
            a, b = d["a_xy"][pid // nb], d["b_xy"][pid % nb]
        else:
            out_off, off = d["out_off"], d["off"]
            s_ = np.searchsorted(out_off, pid, side="right") - 1
            n = off[s_ + 1] - off[s_]
            loc = pid - out_off[s_]
            r, c = loc // n, loc % n
            ia, ib = off[s_] + np.minimum(r, c), off[s_] + np.maximum(r, c)
            a, b = d["a_xy"][ia], d["a_xy"][ib]
        what = f"{len(pid)} sampled cull survivors"
    else:
        if wl == "c3b":
            a_all, b_all = synth_corners(d["a_box"]), synth_corners(d["b_box"])
        else:
            a_all, b_all = d["a_xy"], d["b_xy"]
        n = len(a_all)
        idx = np.sort(rng.choice(n, min(sample, n), replace=False))
        a, b = a_all[idx], b_all[idx]
        if d.get("a_nv") is not None:
            anv, bnv = d["a_nv"][idx], d["b_nv"][idx]
        what = f"{len(idx)} sampled pairs"
    threads = max(1, min(16, os.cpu_count() or 1))
    if wl == "c4n":
        m = oracle.simple_margins(a, b, anv, bnv, threads=threads)
        keep = oracle.simple_filtered_mask(m)
    else:
        m = oracle.pair_margins(a, b, anv, bnv, threads=threads)
        keep = oracle.filtered_mask(m)
    out = {"sample": what, "rejected": round(float(1.0 - keep.mean()), 5)}
    if "redrawn" in d:  # polygons the generator redrew (broken convexity after rounding)
        out["generator_redrawn"] = int(d["redrawn"])
    return out


def synth_corners(box):
    import numpy as np

    import synth
    b = np.asarray(box, np.float64)
    return synth.boxes_to_quads(b[:, 0], b[:, 1], b[:, 2], b[:, 3], b[:, 4])


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the path shards "
              "by independent pairs / scenes, with no exchange in the forward and one column-"
              "gradient reduction for two-set matrices in the backward",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2011_11134_amd as dg
    import synth

    torch.cuda.set_device(0)
    wl = args.workload
    d = synth.get(wl)
    if wl in ("c1", "c3", "c4"):
        step = PairsStep(dg, torch, d)
    elif wl == "c3b":
        step = BoxesStep(dg, torch, d)
    elif wl == "c3i":
        step = IntersectStep(dg, torch, d)
    elif wl == "c4n":
        step = SimpleStep(dg, torch, d)
    else:
        step = MatrixStep(dg, torch, d, wl)
    has_bwd = getattr(step, "has_bwd", True)
    stream = torch.cuda.current_stream().cuda_stream

    # warm-up; with the autotuner on, the first forward and backward time their
    # candidate launch shapes here (synchronising) and keep the fastest
    if not args.no_autotune:
        dg.set_autotune(True)
    for _ in range(max(1, args.warmup)):
        step.fwd(stream)
        if has_bwd:
            step.bwd(stream)
    torch.cuda.synchronize()
    dg.set_autotune(False)
    dg.check_errors()
    tuned = dg.autotune_report()[1].strip().splitlines()

    # path statistics of one forward (before the timed region, so that a
    # profile's last steps are the timed ones and the per-kernel timing): the
    # pairs the exact kernels evaluated and those whose signs took the fp64
    # path
    path = None
    if wl not in ("c4n",):
        dg.set_path_stats(True)
        dg.path_stats()
        step.fwd(stream)
        n_eval, n_fp64, n_thin = dg.path_stats()
        dg.set_path_stats(False)
        path = {"pairs_evaluated": n_eval, "fp64_signs": n_fp64,
                "rate": round(n_fp64 / max(n_eval, 1), 6), "fp64_areas": n_thin}
    torch.cuda.synchronize()
    dg.check_errors()

    # The step is captured once into a HIP graph (the library allocates
    # nothing per call and needs no host synchronisation) and replayed;
    # --eager launches the calls one by one instead.
    use_graph = not args.eager
    if use_graph:
        g_step = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_step):
            cs = torch.cuda.current_stream().cuda_stream
            step.fwd(cs)
            if has_bwd:
                step.bwd(cs)
        torch.cuda.synchronize()
        run_step = g_step.replay
    else:
        def run_step():
            step.fwd(stream)
            if has_bwd:
                step.bwd(stream)
    for _ in range(2):
        run_step()
    torch.cuda.synchronize()
    dg.check_errors()

    # Timed region: exactly `steps` steps, bracketed by synchronize, with one
    # event pair on the launch stream around it (an event between kernels
    # would add queue work to every step).
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_start.record()
    for _ in range(args.steps):
        run_step()
    e_end.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dg.check_errors()
    step_ms_events = e_start.elapsed_time(e_end) / args.steps

    # Kernel durations: the library's per-kernel timing mode brackets every
    # kernel it launches with two HIP events on the launch stream (and waits
    # for each), over `steps` more steps launched one by one.
    dg.set_profiling(True)
    for _ in range(args.steps):
        step.fwd(stream)
        if has_bwd:
            step.bwd(stream)
    torch.cuda.synchronize()
    prof = dg.profile_report()
    dg.set_profiling(False)
    dg.check_errors()
    per_launch = {k: ms / n for k, (n, ms) in prof.items()}
    per_step = {k: ms / args.steps for k, (n, ms) in prof.items()}
    kname = max(per_step, key=per_step.get)  # the dominant kernel of a step
    dur_s = per_launch[kname] * 1e-3
    bound, bytes_launch, basis = step.algorithmic_bytes(kname)
    hbm_gbs = bytes_launch / dur_s / 1e9
    roof = {"bound": bound, "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(hbm_gbs / HBM_PEAK_GBS, 4), "traffic": stored_traffic(wl, kname),
            "kernel": kname, "kernel_ms": round(per_launch[kname], 4),
            "bytes_per_launch": int(bytes_launch), "bytes_basis": basis}
    flops = FLOPS.get((step.kind, kname[-3:]))
    if flops is not None:
        tf = flops * step.pairs / dur_s / 1e12
        roof["alu"] = {"achieved": round(tf, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(tf / FP32_PEAK_TFLOPS, 4), "flops_per_pair": flops}
    kernels = {k: {"ms_per_launch": round(per_launch[k], 4),
                   "launches_per_step": round(prof[k][0] / args.steps, 2)} for k in prof}

    filt = filter_stats(d, wl, step)

    if args.copy_calib_mib:
        src = torch.empty(args.copy_calib_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d, wl, step.kind)
    plain = None
    if not args.no_plain and (step.kind in ("rect", "poly") or wl == "c5"):
        plain = plain_baseline(torch, d, wl)

    value = step.pairs * args.steps / elapsed
    names = {"c1": "c1: 1,024 rotated-rectangle pairs, forward + backward",
             "c2": "c2: 4096 x 4096 rotated BEV box IoU matrix, forward",
             "c3": "c3: 1,048,576 rotated-rectangle pairs, forward + backward",
             "c4": "c4: 262,144 convex 3..8-gon pairs, forward + backward",
             "c5": "c5: 64 scenes (U{50..2000} boxes), per-scene 3D self-pair IoU, forward + backward",
             "c3b": "c3 boxes: 1,048,576 rotated-box pairs as (cx, cy, w, l, yaw) rows, corners "
                    "formed in-kernel, forward + backward to the parameters",
             "c3i": "c3 intersection primitive: 1,048,576 rotated-rectangle pairs, ordered "
                    "intersection polygons + nx + xflags, backward from per-vertex gradients",
             "c4n": "c4 simple: 262,144 pairs of simple (about half non-convex) 3..8-gons, "
                    "forward + backward"}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": names[wl], "pairs": int(step.pairs),
                   ("box_dim" if step.kind == "box" else "kmax"): int(step.a.shape[1]),
                   "parallelism": "single GPU",
                   "launch": "HIP graph replay" if use_graph else "eager",
                   "launch_shapes": tuned or "built-in"},
        "kernels": kernels,
        "step_ms_events": round(step_ms_events, 4),
        "roofline": roof,
        "fp64_fallback": path,
        "filter": filt,
        "cpu_baseline": cpu,
        "plain": plain,
        "vs_plain": None if plain is None else round(value / plain["value"], 2),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
