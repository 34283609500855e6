"""Launch-shape autotuning: tuned calls compute exactly what the built-in
shapes compute, every kind of call used is recorded once, and the choices
persist through the tune cache into a fresh context."""
import ctypes

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


def test_tuned_shapes_persist_into_a_fresh_context(dg, tmp_path):
    """A tuned matrix forward (tile shape included) is saved to a cache file,
    loaded back into the process-wide store, and taken by a context created
    afterwards without tuning; its outputs equal the built-in shape's."""
    print("case: tune cache, scenes 5", flush=True)
    ds = synth.c5_scenes(scenes=5, nmin=40, nmax=900, seed=131)
    xy = dev_t(ds["a_xy"])
    z = (dev_t(ds["a_zlo"]), dev_t(ds["a_zhi"]))
    ref, _, _ = dg.iou_matrix(xy, a_z=z, a_off=ds["off"], self_pairs=True)
    dg.set_autotune(True)
    try:
        tuned, saved, _ = dg.iou_matrix(xy, a_z=z, a_off=ds["off"], self_pairs=True, save=True)
    finally:
        dg.set_autotune(False)
    assert saved.tile_rows in dg.TILE_ROWS_CHOICES
    assert torch.equal(ref, tuned)
    _, text = dg.autotune_report()
    line = [ln for ln in text.splitlines() if "matrix_fwd" in ln and "seg1" in ln
            and f"/b{len(ds['a_xy']).bit_length()}.{(5).bit_length()}:" in ln]
    assert len(line) == 1, text
    assert f"rows={saved.tile_rows}" in line[0]
    key = line[0].split(":")[0]
    path = tmp_path / "tune.json"
    dg.tune_cache_save(str(path))
    dg.tune_cache_clear()
    assert dg.tune_cache_load(str(path)) >= 1
    assert key in dg.tune_cache_report()
    # a fresh context, tuning off: the forward takes the stored shape
    ctx = ctypes.c_void_p()
    assert dg.lib.dgal_create(ctypes.byref(ctx), torch.cuda.current_device()) == dg.DGAL_OK
    try:
        pa, _ = dg.polys(xy, None, z)
        seg = dg.segments(len(ds["a_xy"]), len(ds["a_xy"]), ds["off"], self_pairs=True)
        sv = dg.SavedPairs(1 << 20, 8, seg[5], xy.device)
        st = sv.struct()
        out = torch.full((seg[4],), -1.0, device="cuda")
        rc = dg.lib.dgal_iou_matrix(ctx, pa, pa, seg[0].data_ptr(), seg[1].data_ptr(),
                                    seg[2].data_ptr(), seg[3], 1, out.data_ptr(), seg[4],
                                    ctypes.byref(st), torch.cuda.current_stream().cuda_stream)
        assert rc == dg.DGAL_OK
        assert dg.lib.dgal_check(ctx, torch.cuda.current_stream().cuda_stream) == dg.DGAL_OK
        assert st.tile_rows == saved.tile_rows
        buf = ctypes.create_string_buffer(1 << 14)
        assert dg.lib.dgal_autotune_report(ctx, buf, len(buf)) == 1
        assert buf.value.decode().split(":")[0] == key
        assert torch.equal(out, ref)
    finally:
        torch.cuda.synchronize()
        dg.lib.dgal_destroy(ctx)
