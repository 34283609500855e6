"""Launch-shape autotuning: tuned calls compute exactly what the built-in
shapes compute, and every kind of call used is recorded once."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev_t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_2011_11134_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


def _pairs(dg, d):
    a, b, g = dev_t(d["a_xy"]), dev_t(d["b_xy"]), dev_t(d["grad"])
    iou, nx, xf = dg.iou_pairs(a, b)
    ga, gb, _, _ = dg.iou_pairs_backward(a, b, g, nx, xf)
    return [t.cpu().numpy() for t in (iou, nx, xf, ga, gb)]


def _scenes(dg, d):
    xy = dev_t(d["a_xy"])
    z = (dev_t(d["a_zlo"]), dev_t(d["a_zhi"]))
    iou, saved, seg = dg.iou_matrix(xy, a_z=z, a_off=d["off"], self_pairs=True, save=True)
    g = dev_t(d["grad"])
    ga, _, gz, _ = dg.iou_matrix_backward(g, saved, seg, xy, a_z=z, self_pairs=True)
    return [t.cpu().numpy() for t in (iou, ga, gz)]


def test_autotuned_calls_match_builtin_shapes(dg):
    print("case: autotune pairs 20000 + scenes 6", flush=True)
    dp = synth.c3_pairs(n=20000, seed=121)
    ds = synth.c5_scenes(scenes=6, nmin=50, nmax=400, seed=122)
    ref_p, ref_s = _pairs(dg, dp), _scenes(dg, ds)
    dg.set_autotune(True)
    try:
        tuned_p, tuned_s = _pairs(dg, dp), _scenes(dg, ds)
        n, text = dg.autotune_report()
        print(text, flush=True)
        assert n >= 4 and "pairs_fwd" in text and "matrix_bwd" in text
        again_p, again_s = _pairs(dg, dp), _scenes(dg, ds)   # now with the stored shapes
    finally:
        dg.set_autotune(False)
    for r, t, a in zip(ref_p, tuned_p, again_p):
        assert np.array_equal(r, t) and np.array_equal(r, a)
    # the matrix backward sums rows in LDS in an order that may vary: values agree to rounding
    for r, t, a in zip(ref_s, tuned_s, again_s):
        assert np.allclose(r, t, rtol=1e-5, atol=1e-6) and np.allclose(r, a, rtol=1e-5, atol=1e-6)
    dg.check_errors()
