"""Helpers for the GPU parity tests: run the HIP path through the binding and
the FP64 oracle on the same seeded fp32 inputs, and compare.

Parity bar: nx and xflags bit-exact on every pair (the signs that select the
intersection's vertices and order its boundary are exact on both sides, so
the sequences agree also on degenerate input); |IoU - IoU_oracle| <= 1e-5 on
every pair; per-pair gradient relative error ||g - g_ref|| / max(||g_ref||,
1e-8) <= 1e-3 against the oracle's analytic gradient on every pair whose
crossing edges meet at |sin| >= 1e-3 (a crossing's chain rule carries 1/sin,
so fp32 rounding reaches it as u/sin^2).  Thin polygons and tiny (sliver)
intersections are compared like every other pair: the library rebuilds
their areas, and the elementwise backward their gradient, in fp64.
"""
import numpy as np
import torch

import oracle

IOU_TOL = 1e-5
GRAD_TOL = 1e-3


def dev_t(x, dtype=None):
    if x is None:
        return None
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def conditioned_mask(margins):
    """Pairs whose gradient fp32 can carry to 1e-3: no two crossing edges
    meet at |sin| below 1e-3 (a crossing's chain rule carries 1/sin, so fp32
    rounding reaches it as u/sin^2; margin [1] of the oracle's degeneracy
    margins).  The structure and the IoU are compared on every pair."""
    m = np.asarray(margins)
    return m[:, 1] >= oracle.FILTER_SIN


def grad_rel_err(g, ref):
    g = g.reshape(g.shape[0], -1).astype(np.float64)
    ref = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(g - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-8)


def run_pairs(dg, a, b, a_nv=None, b_nv=None, a_z=None, b_z=None, grad=None):
    """GPU forward (+ backward if grad is given); returns numpy arrays."""
    ta, tb = dev_t(a), dev_t(b)
    tan, tbn = dev_t(a_nv), dev_t(b_nv)
    taz = None if a_z is None else (dev_t(a_z[0]), dev_t(a_z[1]))
    tbz = None if b_z is None else (dev_t(b_z[0]), dev_t(b_z[1]))
    iou, nx, xf = dg.iou_pairs(ta, tb, tan, tbn, taz, tbz)
    out = {"iou": iou.cpu().numpy(), "nx": nx.cpu().numpy(), "xflags": xf.cpu().numpy()}
    if grad is not None:
        tg = dev_t(grad)
        ga, gb, gaz, gbz = dg.iou_pairs_backward(ta, tb, tg, nx, xf, tan, tbn, taz, tbz)
        out.update(ga=ga.cpu().numpy(), gb=gb.cpu().numpy(),
                   gaz=None if gaz is None else gaz.cpu().numpy(),
                   gbz=None if gbz is None else gbz.cpu().numpy())
        # the backward kernel alone, driven by the oracle's saved state
        out["_tensors"] = (ta, tb, tg, tan, tbn, taz, tbz)
    dg.check_errors()
    return out


def compare_pairs(dg, a, b, a_nv=None, b_nv=None, a_z=None, b_z=None, grad=None,
                  require_filtered_frac=0.5, threads=8):
    """Full parity check of the elementwise path; returns a summary dict."""
    gpu = run_pairs(dg, a, b, a_nv, b_nv, a_z, b_z, grad)
    ref_iou, ref_nx, ref_xf, bad = oracle.iou_pairs(a, b, a_nv, b_nv, a_z, b_z, threads=threads)
    assert bad == 0
    margins = oracle.pair_margins(a, b, a_nv, b_nv, threads=threads)
    keep = oracle.filtered_mask(margins)
    assert keep.mean() >= require_filtered_frac, keep.mean()
    # integer state: bit-exact on every pair
    assert np.array_equal(gpu["nx"], ref_nx), np.nonzero(gpu["nx"] != ref_nx)[0][:5]
    mism = np.nonzero(np.any(gpu["xflags"] != ref_xf, axis=1))[0]
    assert mism.size == 0, (mism[:5], gpu["xflags"][mism[:3]], ref_xf[mism[:3]])
    # IoU everywhere
    d = np.abs(gpu["iou"].astype(np.float64) - ref_iou)
    assert d.max() <= IOU_TOL, (d.max(), int(d.argmax()))
    summary = {"n": len(a), "filtered": float(keep.mean()), "max_iou_err": float(d.max()),
               "nx_agree_all": float(np.mean(gpu["nx"] == ref_nx))}
    if grad is not None:
        ga, gb, gaz, gbz = oracle.iou_pairs_grad(a, b, grad, ref_nx, ref_xf, a_nv, b_nv, a_z, b_z,
                                                 threads=threads)
        parts_gpu = [gpu["ga"], gpu["gb"]] + ([gpu["gaz"], gpu["gbz"]] if a_z is not None else [])
        parts_ref = [ga, gb] + ([gaz, gbz] if a_z is not None else [])
        n = len(a)
        g_gpu = np.concatenate([p.reshape(n, -1) for p in parts_gpu], 1)
        g_ref = np.concatenate([p.reshape(n, -1) for p in parts_ref], 1)
        err = grad_rel_err(g_gpu, g_ref)
        cond = conditioned_mask(margins)
        if cond.any():
            assert err[cond].max() <= GRAD_TOL, (err[cond].max(),
                                                 int(np.argmax(np.where(cond, err, 0))))
            summary["max_grad_err"] = float(err[cond].max())
        summary["max_grad_err_all"] = float(err.max())
        if keep.any():
            summary["max_grad_err_filtered"] = float(err[keep].max())
        # the backward kernel on the oracle's own saved state, every pair
        ta, tb, tg, tan, tbn, taz, tbz = gpu["_tensors"]
        o_ga, o_gb, o_gaz, o_gbz = dg.iou_pairs_backward(ta, tb, tg, dev_t(ref_nx), dev_t(ref_xf),
                                                         tan, tbn, taz, tbz)
        parts = [o_ga.cpu().numpy(), o_gb.cpu().numpy()]
        if a_z is not None:
            parts += [o_gaz.cpu().numpy(), o_gbz.cpu().numpy()]
        g2 = np.concatenate([p.reshape(n, -1) for p in parts], 1)
        err2 = grad_rel_err(g2, g_ref)
        summary["max_grad_err_oracle_state_all"] = float(err2.max())
        summary["p999_grad_err_oracle_state_all"] = float(np.quantile(err2, 0.999))
    return summary
