/*
 * simple_oracle.c -- plain, slow FP64 CPU oracle for the IoU of two SIMPLE
 * polygons (counter-clockwise, not necessarily convex) and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY, like dgal_oracle.c: used by the tests, the smoke
 * check and the benchmark's CPU baseline; shares nothing with the GPU
 * library.
 *
 * Paper: Y. Zhong, "Differentiable Computational Geometry for 2D and 3D machine
 * learning", arXiv 2011.11134.  Sec. III keeps polygons convex and plans
 * support for arbitrary polygons; Sec. V lists arbitrary shapes as future
 * work.  This file computes, for simple polygons P and Q, the plain
 * definitions:
 *
 *   area(P n Q)  by a vertical slab decomposition: between consecutive
 *                x-coordinates of all vertices and of all edge crossings, the
 *                edges that span the slab keep their vertical order, so the
 *                length of (P n Q) on a vertical line is linear in x and the
 *                slab's area is its width times that length at mid-slab (the
 *                cross-sections of P and Q are the even-odd intervals of the
 *                edges' ordinates there);
 *   IoU          = area(P n Q) / (area(P) + area(Q) - area(P n Q)), polygon
 *                areas by the shoelace formula;
 *   gradient     the derivative of area(P n Q) when vertex v moves: only the
 *                parts of the two edges at v that lie inside the other
 *                polygon move the boundary of the intersection, with the
 *                edge's outward normal (dy, -dx) weighted by how far along
 *                the edge the point moves with v (1 - t on the edge leaving
 *                v, t on the edge arriving at v).  The inside parts of an
 *                edge are found by cutting it at its crossings with the
 *                other polygon, sorting the cuts, and testing the midpoint of
 *                each piece for inclusion (crossing number).
 *
 * The state the GPU path saves (edge crossing mask, entering-edge mask, the
 * inclusion of each polygon's vertex 0 in the other) is also produced here,
 * for the configuration in which Q is moved by (eps, eps^2), eps -> 0+: the
 * tie rule that resolves contacts for convex input, so that a contact
 * (a vertex on an edge, collinear overlapping edges, shared vertices) gives
 * one definite state.  The area is exact without it; the gradient assumes
 * general position (the tests compare it on pairs whose margins exclude
 * contact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SMP_MAXV 8
#define SMP_MAXX (2 * SMP_MAXV + SMP_MAXV * SMP_MAXV)

typedef struct { double x, y; } spt;

static double s_orient(spt a, spt b, spt c) {
  return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

static int s_sign(double v) { return (v > 0) - (v < 0); }

/* Proper crossing of segments ab and cd (interiors meet at one point). */
static int s_cross(spt a, spt b, spt c, spt d, double *t, double *s) {
  const double o1 = s_orient(c, d, a), o2 = s_orient(c, d, b);
  const double o3 = s_orient(a, b, c), o4 = s_orient(a, b, d);
  if (s_sign(o1) * s_sign(o2) >= 0 || s_sign(o3) * s_sign(o4) >= 0) return 0;
  *t = o1 / (o1 - o2); /* along ab */
  *s = o3 / (o3 - o4); /* along cd */
  return 1;
}

/* Signs under the tie rule, Q moved by d = (eps, eps^2):
 *   side of P's point p of Q's moved edge c->d:
 *     orient(c + d, e + d, p) = o + f.y eps - f.x eps^2,  f = e - c;
 *   side of Q's moved point q of P's edge a->b:
 *     orient(a, b, q + d) = o - e.y eps + e.x eps^2,  e = b - a.
 * The first non-zero coefficient decides; neither is zero for an edge of
 * non-zero length. */
static int s_tie_pq(spt c, spt e, spt p) {
  const double o = s_orient(c, e, p);
  if (o != 0.0) return s_sign(o);
  if (e.y != c.y) return s_sign(e.y - c.y);
  return s_sign(c.x - e.x);
}

static int s_tie_qp(spt a, spt b, spt q) {
  const double o = s_orient(a, b, q);
  if (o != 0.0) return s_sign(o);
  if (b.y != a.y) return s_sign(a.y - b.y);
  return s_sign(b.x - a.x);
}

/* P's point p inside Q moved by d (even-odd, ray towards +x): a vertex of
 * the moved Q is above p when its y is >= p's (eps^2 > 0); an edge that
 * straddles the ray meets it right of p when p is left of the edge going
 * up, right of it going down. */
static int s_tie_inside_pq(spt p, const spt *Q, int n) {
  int c = 0;
  for (int k = 0; k < n; ++k) {
    spt a = Q[k], b = Q[(k + 1) % n];
    const int ua = a.y >= p.y, ub = b.y >= p.y;
    if (ua != ub) {
      const int s = s_tie_pq(a, b, p);
      if (ub ? s > 0 : s < 0) c ^= 1;
    }
  }
  return c;
}

/* Q's moved point q + d inside P: a vertex of P is above q + d when its y
 * is > q's; the side test is the moved point's. */
static int s_tie_inside_qp(spt q, const spt *P, int n) {
  int c = 0;
  for (int k = 0; k < n; ++k) {
    spt a = P[k], b = P[(k + 1) % n];
    const int ua = a.y > q.y, ub = b.y > q.y;
    if (ua != ub) {
      const int s = s_tie_qp(a, b, q);
      if (ub ? s > 0 : s < 0) c ^= 1;
    }
  }
  return c;
}

/* Crossing-number inclusion of p in polygon v (even-odd). */
static int s_inside(spt p, const spt *v, int n) {
  int c = 0;
  for (int k = 0; k < n; ++k) {
    spt a = v[k], b = v[(k + 1) % n];
    if ((a.y > p.y) != (b.y > p.y)) {
      const double x = a.x + (p.y - a.y) * (b.x - a.x) / (b.y - a.y);
      if (x > p.x) c ^= 1;
    }
  }
  return c;
}

static double s_shoelace(const spt *v, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += v[k].x * v[(k + 1) % n].y - v[(k + 1) % n].x * v[k].y;
  return 0.5 * s;
}

static int s_cmp(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Sorted ordinates where the vertical line at x meets the polygon's edges. */
static int s_cut(const spt *v, int n, double x, double *ys) {
  int m = 0;
  for (int k = 0; k < n; ++k) {
    spt a = v[k], b = v[(k + 1) % n];
    const double lo = a.x < b.x ? a.x : b.x, hi = a.x < b.x ? b.x : a.x;
    if (lo < x && x < hi) ys[m++] = a.y + (x - a.x) * (b.y - a.y) / (b.x - a.x);
  }
  qsort(ys, (size_t)m, sizeof(double), s_cmp);
  return m;
}

/* Length of the common part of two unions of intervals [y0,y1],[y2,y3],... */
static double s_common(const double *a, int na, const double *b, int nb) {
  double len = 0.0;
  for (int i = 0; i + 1 < na; i += 2)
    for (int j = 0; j + 1 < nb; j += 2) {
      const double lo = a[i] > b[j] ? a[i] : b[j];
      const double hi = a[i + 1] < b[j + 1] ? a[i + 1] : b[j + 1];
      if (hi > lo) len += hi - lo;
    }
  return len;
}

static double s_slab_area(const spt *P, int n1, const spt *Q, int n2) {
  double xs[SMP_MAXX];
  int m = 0;
  for (int k = 0; k < n1; ++k) xs[m++] = P[k].x;
  for (int k = 0; k < n2; ++k) xs[m++] = Q[k].x;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j) {
      double t, s;
      spt a = P[i], b = P[(i + 1) % n1];
      if (s_cross(a, b, Q[j], Q[(j + 1) % n2], &t, &s)) xs[m++] = a.x + t * (b.x - a.x);
    }
  qsort(xs, (size_t)m, sizeof(double), s_cmp);
  double area = 0.0;
  for (int k = 0; k + 1 < m; ++k) {
    if (!(xs[k + 1] > xs[k])) continue;
    const double xm = 0.5 * (xs[k] + xs[k + 1]);
    double ya[SMP_MAXV], yb[SMP_MAXV];
    const int na = s_cut(P, n1, xm, ya), nb = s_cut(Q, n2, xm, yb);
    area += (xs[k + 1] - xs[k]) * s_common(ya, na, yb, nb);
  }
  return area;
}

/* Inside parts of edge a->b with respect to polygon v: W1 = integral of
 * (1 - t), W2 = integral of t over the parameters t in [0, 1] whose point is
 * inside. */
static void s_edge_weights(spt a, spt b, const spt *v, int n, double *w1, double *w2) {
  double ts[SMP_MAXV + 2];
  int m = 0;
  ts[m++] = 0.0;
  ts[m++] = 1.0;
  for (int j = 0; j < n; ++j) {
    double t, s;
    if (s_cross(a, b, v[j], v[(j + 1) % n], &t, &s)) ts[m++] = t;
  }
  qsort(ts, (size_t)m, sizeof(double), s_cmp);
  *w1 = 0.0;
  *w2 = 0.0;
  for (int k = 0; k + 1 < m; ++k) {
    const double t0 = ts[k], t1 = ts[k + 1];
    if (!(t1 > t0)) continue;
    const double tm = 0.5 * (t0 + t1);
    spt p = {a.x + tm * (b.x - a.x), a.y + tm * (b.y - a.y)};
    if (!s_inside(p, v, n)) continue;
    *w1 += 0.5 * ((1.0 - t0) * (1.0 - t0) - (1.0 - t1) * (1.0 - t1));
    *w2 += 0.5 * (t1 * t1 - t0 * t0);
  }
}

/* d area(P n Q) / d P_k into g[2k], g[2k+1]. */
static void s_inter_grad(const spt *P, int n1, const spt *Q, int n2, double *g) {
  for (int k = 0; k < n1; ++k) g[2 * k] = g[2 * k + 1] = 0.0;
  for (int i = 0; i < n1; ++i) {
    const int in = (i + 1) % n1;
    spt a = P[i], b = P[in];
    double w1, w2;
    s_edge_weights(a, b, Q, n2, &w1, &w2);
    const double nx = b.y - a.y, ny = -(b.x - a.x); /* outward normal x |edge| */
    g[2 * i] += nx * w1;
    g[2 * i + 1] += ny * w1;
    g[2 * in] += nx * w2;
    g[2 * in + 1] += ny * w2;
  }
}

static int s_load(const float *xy, const uint8_t *nv, int64_t i, int k, spt *v) {
  int n = nv ? (int)nv[i] : k;
  if (n < 3 || n > k || n > SMP_MAXV) return -1;
  const float *r = xy + i * (int64_t)k * 2;
  for (int t = 0; t < n; ++t) {
    v[t].x = (double)r[2 * t];
    v[t].y = (double)r[2 * t + 1];
  }
  return n;
}

static double s_iou(double I, double A1, double A2) {
  const double U = A1 + A2 - I;
  return (I > 0.0 && U > 0.0) ? I / U : 0.0;
}

/* Exported for a single pair: intersection area by slabs. */
double oracle_simple_inter_area(const double *p, int n1, const double *q, int n2) {
  spt P[SMP_MAXV], Q[SMP_MAXV];
  if (n1 < 3 || n1 > SMP_MAXV || n2 < 3 || n2 > SMP_MAXV) return -1.0;
  for (int k = 0; k < n1; ++k) P[k] = (spt){p[2 * k], p[2 * k + 1]};
  for (int k = 0; k < n2; ++k) Q[k] = (spt){q[2 * k], q[2 * k + 1]};
  return s_slab_area(P, n1, Q, n2);
}

/* Batched forward over pairs [lo, hi): IoU, and the saved state, all with b
 * moved by the tie rule's (eps, eps^2): xmask bit i*8+j when edge i of a
 * crosses edge j of b (the ends of each lie on opposite sides of the
 * other's line); smask bit i*8+j when, in addition, a's vertex i is right
 * of b's edge j (edge i enters b there); inside bit 0 when a's vertex 0 is
 * inside b, bit 1 when b's vertex 0 is inside a.  Returns the number of
 * pairs with invalid counts. */
int64_t oracle_simple_iou_pairs(int64_t lo, int64_t hi, const float *a_xy, const uint8_t *a_nv,
                                int ka, const float *b_xy, const uint8_t *b_nv, int kb,
                                double *iou, uint64_t *xmask, uint64_t *smask, uint8_t *inside) {
  int64_t bad = 0;
  for (int64_t i = lo; i < hi; ++i) {
    spt P[SMP_MAXV], Q[SMP_MAXV];
    const int n1 = s_load(a_xy, a_nv, i, ka, P), n2 = s_load(b_xy, b_nv, i, kb, Q);
    if (n1 < 0 || n2 < 0) {
      ++bad;
      iou[i] = 0.0;
      if (xmask) xmask[i] = smask[i] = 0;
      if (inside) inside[i] = 0;
      continue;
    }
    const double I = s_slab_area(P, n1, Q, n2);
    iou[i] = s_iou(I, s_shoelace(P, n1), s_shoelace(Q, n2));
    if (xmask) {
      uint64_t xm = 0, sm = 0;
      for (int e = 0; e < n1; ++e)
        for (int f = 0; f < n2; ++f) {
          spt a = P[e], b = P[(e + 1) % n1], c = Q[f], d = Q[(f + 1) % n2];
          const int sa = s_tie_pq(c, d, a), sb = s_tie_pq(c, d, b);
          const int sc = s_tie_qp(a, b, c), sd = s_tie_qp(a, b, d);
          if (sa != sb && sc != sd) {
            xm |= 1ull << (e * 8 + f);
            if (sa < 0) sm |= 1ull << (e * 8 + f);
          }
        }
      xmask[i] = xm;
      smask[i] = sm;
    }
    if (inside)
      inside[i] = (uint8_t)(s_tie_inside_pq(P[0], Q, n2) | (s_tie_inside_qp(Q[0], P, n1) << 1));
  }
  return bad;
}

/* Gradient of sum g * IoU over pairs [lo, hi) with respect to the vertices
 * (rows [i][ka][2] and [i][kb][2], padded slots 0). */
void oracle_simple_iou_pairs_grad(int64_t lo, int64_t hi, const float *a_xy, const uint8_t *a_nv,
                                  int ka, const float *b_xy, const uint8_t *b_nv, int kb,
                                  const double *g, double *ga, double *gb) {
  for (int64_t i = lo; i < hi; ++i) {
    double *oa = ga + i * (int64_t)ka * 2, *ob = gb + i * (int64_t)kb * 2;
    memset(oa, 0, sizeof(double) * 2 * (size_t)ka);
    memset(ob, 0, sizeof(double) * 2 * (size_t)kb);
    spt P[SMP_MAXV], Q[SMP_MAXV];
    const int n1 = s_load(a_xy, a_nv, i, ka, P), n2 = s_load(b_xy, b_nv, i, kb, Q);
    if (n1 < 0 || n2 < 0) continue;
    const double I = s_slab_area(P, n1, Q, n2);
    const double A1 = s_shoelace(P, n1), A2 = s_shoelace(Q, n2);
    const double U = A1 + A2 - I;
    if (!(I > 0.0 && U > 0.0)) continue;
    /* IoU = I / U:  d IoU = (A1 + A2) / U^2 dI - I / U^2 (dA1 + dA2) */
    const double cI = g[i] * (A1 + A2) / (U * U), cA = -g[i] * I / (U * U);
    double dIp[2 * SMP_MAXV], dIq[2 * SMP_MAXV];
    s_inter_grad(P, n1, Q, n2, dIp);
    s_inter_grad(Q, n2, P, n1, dIq);
    for (int k = 0; k < n1; ++k) {
      spt pv = P[(k + n1 - 1) % n1], nx = P[(k + 1) % n1];
      oa[2 * k] = cI * dIp[2 * k] + cA * 0.5 * (nx.y - pv.y);
      oa[2 * k + 1] = cI * dIp[2 * k + 1] + cA * 0.5 * (pv.x - nx.x);
    }
    for (int k = 0; k < n2; ++k) {
      spt pv = Q[(k + n2 - 1) % n2], nx = Q[(k + 1) % n2];
      ob[2 * k] = cI * dIq[2 * k] + cA * 0.5 * (nx.y - pv.y);
      ob[2 * k + 1] = cI * dIq[2 * k + 1] + cA * 0.5 * (pv.x - nx.x);
    }
  }
}

/* Degeneracy margins of simple-polygon pairs [lo, hi): out[i][0] = smallest
 * distance from a vertex of either polygon to an edge of the other, over the
 * pair's size L (diagonal of the joint bounding box); out[i][1] = smallest
 * |sin| of the angle between two crossing edges (1 if none); out[i][2] = the
 * intersection area over the smaller polygon's area (1 if they do not meet):
 * a sliver has an IoU whose fp32 evaluation is all rounding. */
void oracle_simple_margins(int64_t lo, int64_t hi, const float *a_xy, const uint8_t *a_nv, int ka,
                           const float *b_xy, const uint8_t *b_nv, int kb, double *out) {
  for (int64_t i = lo; i < hi; ++i) {
    spt P[SMP_MAXV], Q[SMP_MAXV];
    const int n1 = s_load(a_xy, a_nv, i, ka, P), n2 = s_load(b_xy, b_nv, i, kb, Q);
    out[3 * i] = 0.0;
    out[3 * i + 1] = 0.0;
    out[3 * i + 2] = 0.0;
    if (n1 < 0 || n2 < 0) continue;
    double x0 = P[0].x, x1 = P[0].x, y0 = P[0].y, y1 = P[0].y;
    for (int k = 0; k < n1; ++k) {
      x0 = fmin(x0, P[k].x); x1 = fmax(x1, P[k].x); y0 = fmin(y0, P[k].y); y1 = fmax(y1, P[k].y);
    }
    for (int k = 0; k < n2; ++k) {
      x0 = fmin(x0, Q[k].x); x1 = fmax(x1, Q[k].x); y0 = fmin(y0, Q[k].y); y1 = fmax(y1, Q[k].y);
    }
    const double L = hypot(x1 - x0, y1 - y0);
    double dmin = INFINITY, smin = 1.0;
    for (int side = 0; side < 2; ++side) {
      const spt *V = side ? Q : P, *W = side ? P : Q;
      const int nv = side ? n2 : n1, nw = side ? n1 : n2;
      for (int k = 0; k < nv; ++k)
        for (int j = 0; j < nw; ++j) {
          spt a = W[j], b = W[(j + 1) % nw], p = V[k];
          const double dx = b.x - a.x, dy = b.y - a.y, len2 = dx * dx + dy * dy;
          double t = len2 > 0 ? ((p.x - a.x) * dx + (p.y - a.y) * dy) / len2 : 0.0;
          t = t < 0 ? 0 : (t > 1 ? 1 : t);
          dmin = fmin(dmin, hypot(p.x - (a.x + t * dx), p.y - (a.y + t * dy)));
        }
    }
    for (int e = 0; e < n1; ++e)
      for (int f = 0; f < n2; ++f) {
        double t, s;
        spt a = P[e], b = P[(e + 1) % n1], c = Q[f], d = Q[(f + 1) % n2];
        if (s_cross(a, b, c, d, &t, &s)) {
          const double ux = b.x - a.x, uy = b.y - a.y, vx = d.x - c.x, vy = d.y - c.y;
          smin = fmin(smin, fabs(ux * vy - uy * vx) / (hypot(ux, uy) * hypot(vx, vy)));
        }
      }
    out[3 * i] = L > 0 ? dmin / L : 0.0;
    out[3 * i + 1] = smin;
    const double I = s_slab_area(P, n1, Q, n2);
    const double amin = fmin(s_shoelace(P, n1), s_shoelace(Q, n2));
    out[3 * i + 2] = I > 0.0 ? (amin > 0 ? I / amin : 0.0) : 1.0;
  }
}

/* Input check for simple polygons: 0 if the polygon has 3..8 vertices, no
 * two non-adjacent edges meet, no two adjacent edges overlap, and its
 * shoelace area is positive (counter-clockwise); else 1 (vertex count),
 * 2 (edges meet or overlap) or 3 (area not positive). */
static int s_status(const spt *v, int n);

int oracle_simple_valid(const double *xy, int n) {
  if (n < 3 || n > SMP_MAXV) return 0;
  spt v[SMP_MAXV];
  for (int k = 0; k < n; ++k) v[k] = (spt){xy[2 * k], xy[2 * k + 1]};
  return s_status(v, n) == 0;
}

/* Status of polygons [lo, hi) of a [count][kmax][2] fp32 array. */
void oracle_simple_statuses(int64_t lo, int64_t hi, const float *xy, const uint8_t *nv, int kmax,
                            uint8_t *status) {
  for (int64_t i = lo; i < hi; ++i) {
    const int n = nv ? (int)nv[i] : kmax;
    if (n < 3 || n > kmax || n > SMP_MAXV) {
      status[i] = 1;
      continue;
    }
    spt v[SMP_MAXV];
    const float *r = xy + i * (int64_t)kmax * 2;
    for (int k = 0; k < n; ++k) v[k] = (spt){(double)r[2 * k], (double)r[2 * k + 1]};
    status[i] = (uint8_t)s_status(v, n);
  }
}

static int s_status(const spt *v, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      spt a = v[i], b = v[(i + 1) % n], c = v[j], d = v[(j + 1) % n];
      const int adjacent = (j == i + 1) || (i == 0 && j == n - 1);
      const double o1 = s_orient(c, d, a), o2 = s_orient(c, d, b);
      const double o3 = s_orient(a, b, c), o4 = s_orient(a, b, d);
      if (adjacent) {
        /* the shared vertex only: the edges must not fold back onto each other */
        spt s = (j == i + 1) ? b : a;               /* shared vertex */
        spt u = (j == i + 1) ? a : b;               /* far end of edge i */
        spt w = (j == i + 1) ? d : c;               /* far end of edge j */
        if (s_orient(u, s, w) == 0.0 &&
            ((u.x - s.x) * (w.x - s.x) + (u.y - s.y) * (w.y - s.y)) > 0)
          return 2;
        continue;
      }
      const int s1 = s_sign(o1), s2 = s_sign(o2), s3 = s_sign(o3), s4 = s_sign(o4);
      if (s1 * s2 <= 0 && s3 * s4 <= 0) {
        /* touching or crossing, unless collinear and disjoint */
        if (s1 == 0 && s2 == 0 && s3 == 0 && s4 == 0) {
          const double lo1 = fmin(a.x, b.x), hi1 = fmax(a.x, b.x);
          const double lo2 = fmin(c.x, d.x), hi2 = fmax(c.x, d.x);
          const double ly1 = fmin(a.y, b.y), hy1 = fmax(a.y, b.y);
          const double ly2 = fmin(c.y, d.y), hy2 = fmax(c.y, d.y);
          if (hi1 < lo2 || hi2 < lo1 || hy1 < ly2 || hy2 < ly1) continue;
        }
        return 2;
      }
    }
  return s_shoelace(v, n) > 0.0 ? 0 : 3;
}
