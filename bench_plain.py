"""The plain per-op GPU form of the same geometry, used as the "vs plain"
denominator of the benchmark: convex-polygon intersection, shoelace area and
IoU written as a chain of ordinary torch tensor ops on the GPU, differentiated
by torch autograd (loops and branches become masks and padded tensors, which is
what an autograd framework needs when a geometry routine has data-dependent
control flow).  It is a measurement baseline, not part of the library: nothing
in the library calls it.

Steps per pair, vectorised over the batch (K slots per polygon):
  orientation of every vertex against every edge of the other polygon;
  inside vertices and straddling edge pairs (crossings) as masks;
  all 2K + K^2 candidate points with a validity mask;
  counter-clockwise order by atan2 about the centroid of the valid points
  (invalid candidates sort last);
  shoelace of the valid prefix (padded with the first point), IoU.
"""
import torch


def _cross(ax, ay, bx, by):
    return ax * by - ay * bx


def iou_pairs_plain(a, b, a_nv=None, b_nv=None):
    """a, b: [n, K, 2] fp32 CUDA tensors (requires_grad allowed); a_nv/b_nv:
    optional [n] vertex counts.  Returns IoU [n] fp32 (autograd-able)."""
    inter, a1, a2, m = inter_areas_plain(a, b, a_nv, b_nv)
    u = a1 + a2 - inter
    ok = (m > 0) & (u > 0)
    u_safe = torch.where(ok, u, torch.ones_like(u))
    return torch.where(ok, inter / u_safe, torch.zeros_like(u))


def iou3d_scenes_plain(xy, zlo, zhi, off):
    """Per-scene self-pair 3D IoU, the plain way: every ordered pair of a
    scene's boxes formed by broadcasting, the 2D geometry above, times the
    z-overlap over the union volume; the diagonal is 1.  xy [n, 4, 2], zlo,
    zhi [n] (requires_grad allowed), off: host offsets [scenes + 1].  Returns
    the flat blocks, row-major per scene, concatenated (autograd-able)."""
    out = []
    for s in range(len(off) - 1):
        o0, o1 = int(off[s]), int(off[s + 1])
        n = o1 - o0
        if n == 0:
            continue
        A = xy[o0:o1]
        a = A[:, None].expand(n, n, *A.shape[1:]).reshape(n * n, *A.shape[1:])
        b = A[None, :].expand(n, n, *A.shape[1:]).reshape(n * n, *A.shape[1:])
        inter, a1, a2, m = inter_areas_plain(a, b)
        lo, hi = zlo[o0:o1], zhi[o0:o1]
        lo1, hi1 = lo[:, None].expand(n, n).reshape(-1), hi[:, None].expand(n, n).reshape(-1)
        lo2, hi2 = lo[None, :].expand(n, n).reshape(-1), hi[None, :].expand(n, n).reshape(-1)
        hz = torch.minimum(hi1, hi2) - torch.maximum(lo1, lo2)
        v = inter * hz
        u = a1 * (hi1 - lo1) + a2 * (hi2 - lo2) - v
        ok = (m > 0) & (hz > 0) & (u > 0)
        u_safe = torch.where(ok, u, torch.ones_like(u))
        iou = torch.where(ok, v / u_safe, torch.zeros_like(u))
        eye = torch.eye(n, dtype=torch.bool, device=xy.device).reshape(-1)
        out.append(torch.where(eye, torch.ones_like(iou), iou))
    return torch.cat(out)


def inter_areas_plain(a, b, a_nv=None, b_nv=None):
    """Intersection area, the two polygon areas and the intersection's vertex
    count of elementwise pairs (the steps in the module docstring)."""
    n, K = a.shape[0], a.shape[1]
    dev = a.device
    k_idx = torch.arange(K, device=dev)
    n1 = torch.full((n,), K, device=dev, dtype=torch.long) if a_nv is None else a_nv.long()
    n2 = torch.full((n,), K, device=dev, dtype=torch.long) if b_nv is None else b_nv.long()
    nxt1 = torch.where(k_idx[None, :] + 1 < n1[:, None], k_idx[None, :] + 1, 0)  # [n, K]
    nxt2 = torch.where(k_idx[None, :] + 1 < n2[:, None], k_idx[None, :] + 1, 0)
    v1 = k_idx[None, :] < n1[:, None]
    v2 = k_idx[None, :] < n2[:, None]
    px, py = a[..., 0], a[..., 1]
    qx, qy = b[..., 0], b[..., 1]
    epx = torch.gather(px, 1, nxt1) - px
    epy = torch.gather(py, 1, nxt1) - py
    eqx = torch.gather(qx, 1, nxt2) - qx
    eqy = torch.gather(qy, 1, nxt2) - qy
    # d[n, i, j] = P_i - Q_j
    dx = px[:, :, None] - qx[:, None, :]
    dy = py[:, :, None] - qy[:, None, :]
    oP = _cross(eqx[:, None, :], eqy[:, None, :], dx, dy)        # orient(Q_j, Q_j+1, P_i)
    oQ = _cross(epx[:, :, None], epy[:, :, None], -dx, -dy)      # orient(P_i, P_i+1, Q_j), [n,i,j]
    vij = v1[:, :, None] & v2[:, None, :]
    sP = (oP > 0) | ~vij
    sQ = (oQ > 0) | ~vij
    inP = sP.all(2) & v1                                        # P_i inside Q
    inQ = sQ.all(1) & v2                                        # Q_j inside P
    sP_next = torch.gather(oP > 0, 1, nxt1[:, :, None].expand(n, K, K))
    sQ_next = torch.gather(oQ > 0, 2, nxt2[:, None, :].expand(n, K, K))
    cross_ij = ((oP > 0) != sP_next) & ((oQ > 0) != sQ_next) & vij
    oP_next = torch.gather(oP, 1, nxt1[:, :, None].expand(n, K, K))
    den = oP - oP_next
    den = torch.where(cross_ij, den, torch.ones_like(den))
    t = torch.where(cross_ij, oP / den, torch.zeros_like(den))
    cx_ = px[:, :, None] + t * epx[:, :, None]
    cy_ = py[:, :, None] + t * epy[:, :, None]
    cand_x = torch.cat([px, qx, cx_.reshape(n, K * K)], 1)
    cand_y = torch.cat([py, qy, cy_.reshape(n, K * K)], 1)
    valid = torch.cat([inP, inQ, cross_ij.reshape(n, K * K)], 1)
    m = valid.sum(1)
    vf = valid.to(a.dtype)
    cnt = torch.clamp(m, min=1).to(a.dtype)
    cxm = (cand_x * vf).sum(1) / cnt
    cym = (cand_y * vf).sum(1) / cnt
    ang = torch.atan2((cand_y - cym[:, None]).detach(), (cand_x - cxm[:, None]).detach())
    ang = torch.where(valid, ang, torch.full_like(ang, float("inf")))
    order = torch.argsort(ang, dim=1)
    sx = torch.gather(cand_x, 1, order)
    sy = torch.gather(cand_y, 1, order)
    pos = torch.arange(sx.shape[1], device=dev)[None, :]
    keep = pos < m[:, None]
    sx = torch.where(keep, sx, sx[:, :1])
    sy = torch.where(keep, sy, sy[:, :1])
    inter = 0.5 * _cross(sx, sy, torch.roll(sx, -1, 1), torch.roll(sy, -1, 1)).sum(1)

    def area(x, y, nn, nx_idx):
        xn = torch.gather(x, 1, nx_idx)
        yn = torch.gather(y, 1, nx_idx)
        vv = k_idx[None, :] < nn[:, None]
        return 0.5 * torch.where(vv, _cross(x, y, xn, yn), torch.zeros_like(x)).sum(1)

    a1 = area(px, py, n1, nxt1)
    a2 = area(qx, qy, n2, nxt2)
    return inter, a1, a2, m
