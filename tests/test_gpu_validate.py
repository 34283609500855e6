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
