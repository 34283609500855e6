"""GPU input-contract check (Sec. III: convex, counter-clockwise, at most kmax
vertices) through the C ABI against the oracle's status of each polygon, and
the check-before-every-call mode."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev_t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


def _say(msg):
    print(msg, flush=True)


def _mixed(n=20000, seed=131):
    """Valid 3..8-gons and broken variants of them, [n, 8, 2] + counts."""
    rng = np.random.default_rng(seed)
    d = synth.c4_polygons(n=n, seed=seed)
    xy, nv = d["a_xy"].copy(), d["a_nv"].copy()
    kind = rng.integers(0, 7, n)
    for i in range(n):
        k = int(nv[i])
        v = xy[i, :k].copy()
        if kind[i] == 1:            # clockwise
            v = v[::-1]
        elif kind[i] == 2 and k >= 4:  # two neighbours swapped: a bow tie
            j = int(rng.integers(0, k - 1))
            v[[j, j + 1]] = v[[j + 1, j]]
        elif kind[i] == 3:          # star polygon {p/q}, q >= 2, rotated and scaled
            p = int(rng.choice([5, 7, 7, 8]))
            q = {5: 2, 7: int(rng.choice([2, 3])), 8: 3}[p]
            ph, r = rng.uniform(0, 2 * math.pi), rng.uniform(0.5, 2.0)
            c = rng.uniform(-1, 1, 2)
            v = np.array([[c[0] + r * math.cos(ph + 2 * math.pi * q * t / p),
                           c[1] + r * math.sin(ph + 2 * math.pi * q * t / p)] for t in range(p)],
                         np.float32)
            k = p
        elif kind[i] == 4 and k < 8:  # a vertex repeated
            j = int(rng.integers(0, k))
            v = np.concatenate([v[:j + 1], v[j:j + 1], v[j + 1:]])
            k += 1
        elif kind[i] == 5:          # vertex count out of range
            nv[i] = rng.choice([0, 1, 2, 9, 200])
            continue
        xy[i, :k] = v
        xy[i, k:] = v[0]
        nv[i] = k
    return xy, nv


def test_status_matches_oracle(dg):
    xy, nv = _mixed()
    _say(f"case: validate mixed {len(xy)} polygons")
    st, n_bad = dg.validate(dev_t(xy), dev_t(nv))
    st = st.cpu().numpy()
    ref = oracle.polygon_status(xy, nv)
    assert np.array_equal(st, ref), np.flatnonzero(st != ref)[:10]
    assert n_bad == int(np.count_nonzero(ref))
    counts = np.bincount(ref, minlength=4)
    _say(str({"status_counts": counts.tolist()}))
    assert np.all(counts > 100)  # every outcome is exercised


def test_full_size_rectangles_are_valid(dg):
    d = synth.c3_pairs()
    _say(f"case: validate c3 rectangles {len(d['a_xy'])} x 2")
    for key in ("a_xy", "b_xy"):
        st, n_bad = dg.validate(dev_t(d[key]))
        assert n_bad == 0
        assert int(st.max().item()) == 0


def test_check_before_every_call(dg):
    d = synth.c1_pairs(n=4096, seed=132)
    a, b = dev_t(d["a_xy"]), dev_t(d["b_xy"])
    iou0, nx0, xf0 = dg.iou_pairs(a, b)
    bad = d["b_xy"].copy()
    bad[17] = bad[17, ::-1]  # one clockwise polygon
    tb_bad = dev_t(bad)
    dg.set_validate(True)
    try:
        i2, n2, x2 = dg.iou_pairs(a, b)
        assert torch.equal(i2, iou0) and torch.equal(n2, nx0) and torch.equal(x2, xf0)
        with pytest.raises(dg.DgalError) as e:
            dg.iou_pairs(a, tb_bad)
        assert e.value.status == dg.DGAL_EINVAL
        with pytest.raises(dg.DgalError):
            dg.intersect(a, tb_bad)
        with pytest.raises(dg.DgalError):
            dg.iou_matrix(a[:64], tb_bad[:64])
        # the area accepts any simple polygon and is not checked
        dg.area(tb_bad)
    finally:
        dg.set_validate(False)
    # off again: the clockwise polygon goes through unchecked
    iou1, _, _ = dg.iou_pairs(a, tb_bad)
    try:  # a clockwise polygon may overflow its pair's capacity (a sticky error)
        dg.check_errors()
    except dg.DgalError as e:
        assert e.status == dg.DGAL_ECAPACITY
    keep = np.ones(len(bad), bool)
    keep[17] = False
    assert torch.equal(iou1.cpu()[keep], iou0.cpu()[keep])


def _mixed_simple(n=20000, seed=133):
    """Simple polygons and broken variants of them (clockwise, swapped
    neighbours, repeated vertices, stars, counts out of range, integer
    rectilinear shapes whose edges touch exactly)."""
    rng = np.random.default_rng(seed)
    d = synth.c4_simple(n=n, seed=seed)
    xy, nv = d["a_xy"].copy(), d["a_nv"].copy()
    kind = rng.integers(0, 8, n)
    for i in range(n):
        k = int(nv[i])
        v = xy[i, :k].copy()
        if kind[i] == 1:
            v = v[::-1]
        elif kind[i] == 2 and k >= 4:
            j = int(rng.integers(0, k - 1))
            v[[j, j + 1]] = v[[j + 1, j]]
        elif kind[i] == 3 and k < 8:
            j = int(rng.integers(0, k))
            v = np.concatenate([v[:j + 1], v[j:j + 1], v[j + 1:]])
            k += 1
        elif kind[i] == 4:
            v = np.array([[math.cos(0.3 + 4 * math.pi * t / 5), math.sin(0.3 + 4 * math.pi * t / 5)]
                          for t in range(5)], np.float32)
            k = 5
        elif kind[i] == 5:
            nv[i] = rng.choice([0, 2, 9, 77])
            continue
        elif kind[i] == 6:
            w, h = int(rng.integers(3, 7)), int(rng.integers(3, 7))
            a1 = int(rng.integers(1, w - 1))
            a2 = int(rng.integers(a1 + 1, w))
            b = int(rng.integers(0, h + 1))  # b = 0 or h: edges touch or fold
            v = np.array([(0, 0), (w, 0), (w, h), (a2, h), (a2, b), (a1, b), (a1, h), (0, h)],
                         np.float32)
            k = 8
        xy[i, :k] = v
        xy[i, k:] = v[0]
        nv[i] = k
    return xy, nv


def test_simple_status_matches_oracle(dg):
    xy, nv = _mixed_simple()
    _say(f"case: validate_simple mixed {len(xy)} polygons")
    st, n_bad = dg.validate_simple(dev_t(xy), dev_t(nv))
    st = st.cpu().numpy()
    ref = oracle.simple_status(xy, nv)
    assert np.array_equal(st, ref), np.flatnonzero(st != ref)[:10]
    assert n_bad == int(np.count_nonzero(ref))
    counts = np.bincount(ref, minlength=4)
    _say(str({"status_counts": counts.tolist()}))
    assert np.all(counts > 100)


def test_simple_check_before_every_call(dg):
    d = synth.c4_simple(n=2048, seed=134)
    a, b = dev_t(d["a_xy"]), dev_t(d["b_xy"])
    an, bn = dev_t(d["a_nv"]), dev_t(d["b_nv"])
    iou0, _, _, _ = dg.iou_simple_pairs(a, b, an, bn)
    bad = d["b_xy"].copy()
    bad[5, :d["b_nv"][5]] = bad[5, :d["b_nv"][5]][::-1]  # clockwise
    dg.set_validate(True)
    try:
        i1, _, _, _ = dg.iou_simple_pairs(a, b, an, bn)
        assert torch.equal(i1, iou0)
        with pytest.raises(dg.DgalError) as e:
            dg.iou_simple_pairs(a, dev_t(bad), an, bn)
        assert e.value.status == dg.DGAL_EINVAL
    finally:
        dg.set_validate(False)
