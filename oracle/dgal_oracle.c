/*
 * dgal_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for batched
 * convex-polygon intersection, shoelace area, IoU (2D, and BEV x z-overlap 3D)
 * and the analytic IoU gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only users of this library.  It shares
 * no source, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Paper: Y. Zhong, "Differentiable Computational Geometry for 2D and 3D machine
 * learning", arXiv 2011.11134.
 *   Sec. II-B (listing)  IoU of two convex polygons is area(intersection) over
 *                        area(p1) + area(p2) - area(intersection); the forward
 *                        keeps the intersection's vertex count nx and one
 *                        provenance flag per intersection vertex (xflags), and
 *                        the gradient is computed from p1, p2, the upstream
 *                        gradient, nx and xflags alone.
 *   Sec. II-C            results live in fixed-capacity storage; two
 *                        quadrilaterals meet in at most 8 vertices.
 *   Sec. III             points are coordinate pairs; a line is kept as the
 *                        coefficients of its equation and is built from two
 *                        points in a differentiable way; a polygon is convex,
 *                        counter-clockwise, and holds at most `capacity`
 *                        vertices; the same polygon type carries the per-vertex
 *                        gradient.
 *   Sec. IV-A            rotated 2D and 3D IoU of bounding boxes.
 *
 * The intersection is computed from its plain definition: the vertices of
 * P n Q are the vertices of P inside Q, the vertices of Q inside P and the
 * points where an edge of P crosses an edge of Q; ordered counter-clockwise
 * they give the area by the shoelace formula.
 *
 * Readings where the paper is silent:
 *   R1 flag encoding: P vertex i -> i; Q vertex j -> 0x10|j; crossing of P edge
 *      i with Q edge j -> 0x40|(i<<3)|j; unused slot -> 0xFF.  Edge i runs from
 *      vertex i to vertex (i+1) mod n.
 *   R2 vertex order: counter-clockwise along the boundary, starting at the
 *      smallest code.  On distinct points this is the order by angle about
 *      any interior point; where points coincide (contacts resolved by R3)
 *      it is the boundary order of the moved pair, found by walking the
 *      boundary from edge to edge (see intersect).
 *   R3 degeneracies: symbolic perturbation, Q translated by (eps, eps^2) with
 *      eps -> 0+.  An exactly-zero orientation takes the sign of the leading
 *      eps term (see side_of_q_edge / side_of_p_edge).
 *   R4 empty intersection: IoU = 0, gradient 0.
 *   R5 a non-positive union (reached by flat 3D boxes): IoU = 0, gradient 0.
 *   R6 capacity of an intersection: n1 + n2.
 *   R9 gradient at a change of combinatorial type: the one-sided gradient of
 *      the structure recorded in the flags.
 *   R12 3D IoU: BEV intersection area times z-overlap over the union volume.
 *   R15 self-pair matrices: the diagonal is exactly 1 (the IoU of a polygon
 *      with itself), with zero gradient.
 *   R25 self-pair matrices (one set against itself, as in the per-scene 3D
 *      IoU of Sec. IV-A): entries (r, c) and (c, r) hold the IoU of one
 *      unordered pair, evaluated once with the lower-indexed polygon as P and
 *      the higher-indexed one as Q (the polygon the tie rule R3 moves, and the
 *      second argument of the z-overlap ties).  The matrix is then symmetric
 *      and each unordered pair has one derivative structure, so the summed
 *      gradient of a pair keeps the translation and rotation invariances also
 *      where the tie rule decides.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define ORC_MAXV 8             /* most vertices of an input polygon */
#define ORC_CAP (2 * ORC_MAXV) /* most vertices of an intersection (R6) */

typedef struct { double x, y; } point;
typedef struct { double v[3]; } hvec;     /* homogeneous 3-vector */
typedef struct {
  int n;
  point v[ORC_CAP];
  uint8_t code[ORC_CAP];
} polygon;

static point mkpt(double x, double y) {
  point p;
  p.x = x;
  p.y = y;
  return p;
}
static point psub(point a, point b) { return mkpt(a.x - b.x, a.y - b.y); }
static double cross2(point u, point v) { return u.x * v.y - u.y * v.x; }

/* orient(a, b, c) = (b - a) x (c - a); positive iff c is left of a -> b. */
static double orient(point a, point b, point c) {
  return cross2(psub(b, a), psub(c, a));
}

static hvec hcross(hvec u, hvec w) {
  hvec r;
  r.v[0] = u.v[1] * w.v[2] - u.v[2] * w.v[1];
  r.v[1] = u.v[2] * w.v[0] - u.v[0] * w.v[2];
  r.v[2] = u.v[0] * w.v[1] - u.v[1] * w.v[0];
  return r;
}
static hvec hpoint(point p) {
  hvec r;
  r.v[0] = p.x;
  r.v[1] = p.y;
  r.v[2] = 1.0;
  return r;
}

/* Meeting point of P's edge a->b with the line of Q's edge c->d (the meet of
 * the two lines of Sec. III), placed along a->b at t = o(a) / (o(a) - o(b)),
 * o = orient(c, d, .).  For fp32-valued points each orientation is exact up
 * to its last rounding, and at a crossing the two have opposite signs (or one
 * is zero), so t keeps full precision at any angle between the edges.  The
 * dehomogenised cross product of the two lines' coefficients gives the same
 * point in exact arithmetic but divides by the cross product of the edge
 * directions, which loses about 1/sin(angle) ulps: near-parallel edges that
 * share an end then meet visibly off the segment. */
static point edge_meet(point a, point b, point c, point d) {
  const double oa = orient(c, d, a), ob = orient(c, d, b);
  const double t = oa / (oa - ob);
  return mkpt(a.x + t * (b.x - a.x), a.y + t * (b.y - a.y));
}

/* R3.  Sign of orient(Q_j, Q_j1, p) with Q moved by (eps, eps^2):
 * orient - (f x (eps, eps^2)) with f = Q_j1 - Q_j, i.e. o + f.y*eps - f.x*eps^2. */
static int side_of_q_edge(point qj, point qj1, point p) {
  double o = orient(qj, qj1, p);
  if (o > 0) return 1;
  if (o < 0) return -1;
  if (qj1.y != qj.y) return qj1.y > qj.y ? 1 : -1;
  return qj.x > qj1.x ? 1 : -1;
}

/* R3.  Sign of orient(P_i, P_i1, q) with q moved by (eps, eps^2):
 * o + e x (eps, eps^2) with e = P_i1 - P_i, i.e. o - e.y*eps + e.x*eps^2. */
static int side_of_p_edge(point pi, point pi1, point q) {
  double o = orient(pi, pi1, q);
  if (o > 0) return 1;
  if (o < 0) return -1;
  if (pi.y != pi1.y) return pi.y > pi1.y ? 1 : -1;
  return pi1.x > pi.x ? 1 : -1;
}

/* Sec. II-B `intersect`, Sec. III convex CCW polygon.  Returns the vertex
 * count m (0 for an empty intersection) or -1 if more than the capacity would
 * be produced or the boundary walk does not close over the m vertices (both
 * possible only for invalid, non-convex input). */
static int intersect(const point *P, int n1, const point *Q, int n2,
                     polygon *out) {
  int sp[ORC_MAXV][ORC_MAXV]; /* sp[i][j]: side of P_i w.r.t. Q edge j */
  int sq[ORC_MAXV][ORC_MAXV]; /* sq[j][i]: side of Q_j w.r.t. P edge i */
  point cand[ORC_MAXV * ORC_MAXV + 2 * ORC_MAXV];
  uint8_t ccode[ORC_MAXV * ORC_MAXV + 2 * ORC_MAXV];
  int m = 0;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j) {
      sp[i][j] = side_of_q_edge(Q[j], Q[(j + 1) % n2], P[i]);
      sq[j][i] = side_of_p_edge(P[i], P[(i + 1) % n1], Q[j]);
    }
  /* vertices of P strictly inside Q */
  for (int i = 0; i < n1; ++i) {
    int in = 1;
    for (int j = 0; j < n2; ++j) in &= sp[i][j] > 0;
    if (in) {
      cand[m] = P[i];
      ccode[m] = (uint8_t)i;
      ++m;
    }
  }
  /* vertices of Q strictly inside P */
  for (int j = 0; j < n2; ++j) {
    int in = 1;
    for (int i = 0; i < n1; ++i) in &= sq[j][i] > 0;
    if (in) {
      cand[m] = Q[j];
      ccode[m] = (uint8_t)(0x10 | j);
      ++m;
    }
  }
  /* edge crossings: P edge i straddles the line of Q edge j and vice versa */
  for (int i = 0; i < n1; ++i) {
    int i1 = (i + 1) % n1;
    for (int j = 0; j < n2; ++j) {
      int j1 = (j + 1) % n2;
      if (sp[i][j] != sp[i1][j] && sq[j][i] != sq[j1][i]) {
        cand[m] = edge_meet(P[i], P[i1], Q[j], Q[j1]);
        ccode[m] = (uint8_t)(0x40 | (i << 3) | j);
        ++m;
      }
    }
  }
  if (m > n1 + n2) return -1;
  out->n = m;
  if (m == 0) return 0;

  /* R2: the boundary of P n Q walked counter-clockwise from the smallest
   * code (the candidates were collected in ascending code, so that is the
   * first one).  Each vertex leaves along one edge that runs inside the other
   * polygon: a vertex of P (of Q) along its own edge; a crossing of P edge i
   * with Q edge j along P edge i when that edge enters Q there (P_i outside
   * the line of Q edge j), else along Q edge j (which then enters P).  The
   * next vertex on an edge is its end vertex when that end is inside the
   * other polygon, else the crossing where the edge leaves it (a convex
   * polygon is left once).  The signs are those of the pair moved by the tie
   * rule (R3), whose intersection has distinct vertices in a definite
   * boundary order; this walk finds that order also where the unmoved points
   * coincide, which no angle about a centre can tell apart. */
  int order[ORC_MAXV * ORC_MAXV + 2 * ORC_MAXV];
  int seen[ORC_MAXV * ORC_MAXV + 2 * ORC_MAXV];
  for (int k = 0; k < m; ++k) seen[k] = 0;
  int cur = 0;
  for (int k = 0; k < m; ++k) {
    if (seen[cur]) return -1; /* a closed walk shorter than m: invalid input */
    seen[cur] = 1;
    order[k] = cur;
    const int code = ccode[cur];
    int along_p, e; /* the edge the boundary leaves on: P edge e or Q edge e */
    if (code < 0x10) {
      along_p = 1;
      e = code;
    } else if (code < 0x40) {
      along_p = 0;
      e = code & 0x0F;
    } else {
      const int i = (code >> 3) & 7, j = code & 7;
      along_p = sp[i][j] < 0;
      e = along_p ? i : j;
    }
    int want = -1; /* code of the next vertex */
    if (along_p) {
      const int e1 = (e + 1) % n1;
      int in = 1;
      for (int j = 0; j < n2; ++j) in &= sp[e1][j] > 0;
      if (in) {
        want = e1;
      } else {
        for (int j = 0; j < n2; ++j) {
          const int j1 = (j + 1) % n2;
          const int leaves = sp[e][j] > 0 && sp[e1][j] < 0 && sq[j][e] != sq[j1][e];
          if (leaves) {
            if (want >= 0) return -1; /* left twice: not convex */
            want = 0x40 | (e << 3) | j;
          }
        }
      }
    } else {
      const int e1 = (e + 1) % n2;
      int in = 1;
      for (int i = 0; i < n1; ++i) in &= sq[e1][i] > 0;
      if (in) {
        want = 0x10 | e1;
      } else {
        for (int i = 0; i < n1; ++i) {
          const int i1 = (i + 1) % n1;
          const int leaves = sq[e][i] > 0 && sq[e1][i] < 0 && sp[i][e] != sp[i1][e];
          if (leaves) {
            if (want >= 0) return -1;
            want = 0x40 | (i << 3) | e;
          }
        }
      }
    }
    int next = -1;
    for (int t = 0; t < m; ++t)
      if (ccode[t] == want) next = t;
    if (next < 0) return -1; /* the boundary leads to no collected vertex */
    cur = next;
  }
  if (cur != 0) return -1; /* the walk must close on its first vertex */
  for (int k = 0; k < m; ++k) {
    out->v[k] = cand[order[k]];
    out->code[k] = ccode[order[k]];
  }
  return m;
}

/* Shoelace area, written about the first vertex. */
static double area(const point *v, int n) {
  double s = 0.0;
  for (int k = 1; k + 1 < n; ++k) s += cross2(psub(v[k], v[0]), psub(v[k + 1], v[0]));
  return 0.5 * s;
}

/* Rebuild one intersection vertex from its provenance code (R1). */
static point vertex_from_code(const point *P, int n1, const point *Q, int n2,
                              uint8_t code) {
  if (code < 0x10) return P[code];
  if (code < 0x40) return Q[code & 0x0F];
  int i = (code >> 3) & 7, j = code & 7;
  return edge_meet(P[i], P[(i + 1) % n1], Q[j], Q[(j + 1) % n2]);
}

/* R12: z-overlap of two extents. */
static double z_overlap(double lo1, double hi1, double lo2, double hi2) {
  double top = hi1 < hi2 ? hi1 : hi2;
  double bot = lo1 > lo2 ? lo1 : lo2;
  double h = top - bot;
  return h > 0 ? h : 0.0;
}

/* IoU of one pair (Sec. II-B).  z1/z2 are (lo, hi) or NULL for 2D. */
static double iou_pair(const point *P, int n1, const point *Q, int n2,
                       const double *z1, const double *z2, uint8_t *nx,
                       uint8_t *flags, int cap, int *err) {
  polygon X;
  int m = intersect(P, n1, Q, n2, &X);
  if (flags)
    for (int k = 0; k < cap; ++k) flags[k] = 0xFF;
  if (m < 0) {
    *err = 1;
    if (nx) *nx = 0;
    return 0.0;
  }
  if (nx) *nx = (uint8_t)m;
  if (flags)
    for (int k = 0; k < m; ++k) flags[k] = X.code[k];
  double ai = m >= 3 ? area(X.v, m) : 0.0;
  double a1 = area(P, n1), a2 = area(Q, n2);
  if (m == 0) return 0.0; /* R4 */
  if (!z1) {
    double u = a1 + a2 - ai;
    return u > 0 ? ai / u : 0.0;
  }
  double hz = z_overlap(z1[0], z1[1], z2[0], z2[1]);
  double v = ai * hz, v1 = a1 * (z1[1] - z1[0]), v2 = a2 * (z2[1] - z2[0]);
  double u = v1 + v2 - v;
  return u > 0 ? v / u : 0.0;
}

/* Adds, into gv[0..n-1], gA * dA/dv for the shoelace area of v. */
static void area_grad(const point *v, int n, double gA, point *gv) {
  for (int k = 0; k < n; ++k) {
    point nxt = v[(k + 1) % n], prv = v[(k + n - 1) % n];
    gv[k].x += gA * 0.5 * (nxt.y - prv.y);
    gv[k].y += gA * 0.5 * (prv.x - nxt.x);
  }
}

/* Chain rule of X = meet(line(a,b), line(c,d)) through the homogeneous form
 * (Sec. III: a line's coefficients are the cross product (p,1) x (q,1) of
 * two of its points, and two lines meet at the dehomogenised cross product
 * of their coefficients).  G = dL/dX; adds dL/da.. into ga..gd. */
static void line_meet_grad(point a, point b, point c, point d, point G,
                           point *ga, point *gb, point *gc, point *gd) {
  hvec ah = hpoint(a), bh = hpoint(b), ch = hpoint(c), dh = hpoint(d);
  hvec l1 = hcross(ah, bh), l2 = hcross(ch, dh), h = hcross(l1, l2);
  hvec gh;
  gh.v[0] = G.x / h.v[2];
  gh.v[1] = G.y / h.v[2];
  gh.v[2] = -(G.x * h.v[0] + G.y * h.v[1]) / (h.v[2] * h.v[2]);
  /* h = l1 x l2  =>  dL/dl1 = l2 x gh,  dL/dl2 = gh x l1 */
  hvec gl1 = hcross(l2, gh), gl2 = hcross(gh, l1);
  /* l1 = a x b  =>  dL/da = b x gl1,  dL/db = gl1 x a  (same for l2) */
  hvec t;
  t = hcross(bh, gl1);
  ga->x += t.v[0];
  ga->y += t.v[1];
  t = hcross(gl1, ah);
  gb->x += t.v[0];
  gb->y += t.v[1];
  t = hcross(dh, gl2);
  gc->x += t.v[0];
  gc->y += t.v[1];
  t = hcross(gl2, ch);
  gd->x += t.v[0];
  gd->y += t.v[1];
}

/* Adds the gradient with respect to P and Q of sum_k <gX[k], X_k>, X_k the
 * intersection vertices named by their provenance codes: a polygon vertex
 * passes its gradient through, a crossing takes the chain rule of the meeting
 * point of two lines. */
static void route_vertex_grads(const point *P, int n1, const point *Q, int n2, int nx,
                               const uint8_t *flags, const point *gX, point *gP,
                               point *gQ) {
  for (int k = 0; k < nx; ++k) {
    uint8_t code = flags[k];
    if (code < 0x10) {
      gP[code].x += gX[k].x;
      gP[code].y += gX[k].y;
    } else if (code < 0x40) {
      gQ[code & 0x0F].x += gX[k].x;
      gQ[code & 0x0F].y += gX[k].y;
    } else {
      int i = (code >> 3) & 7, j = code & 7;
      int i1 = (i + 1) % n1, j1 = (j + 1) % n2;
      line_meet_grad(P[i], P[i1], Q[j], Q[j1], gX[k], &gP[i], &gP[i1], &gQ[j],
                     &gQ[j1]);
    }
  }
}

/* Sec. II-B `iou_grad`: gradient of one pair from the saved nx and flags.
 * Overwrites gP[0..n1-1], gQ[0..n2-1] (and gz1/gz2 = d/d(lo,hi) if 3D). */
static void iou_grad_pair(const point *P, int n1, const point *Q, int n2,
                          const double *z1, const double *z2, double g, int nx,
                          const uint8_t *flags, point *gP, point *gQ,
                          double *gz1, double *gz2) {
  for (int k = 0; k < n1; ++k) gP[k] = mkpt(0, 0);
  for (int k = 0; k < n2; ++k) gQ[k] = mkpt(0, 0);
  if (gz1) gz1[0] = gz1[1] = gz2[0] = gz2[1] = 0.0;
  if (nx < 3) return; /* R4 */
  point X[ORC_CAP];
  for (int k = 0; k < nx; ++k) X[k] = vertex_from_code(P, n1, Q, n2, flags[k]);
  double ai = area(X, nx), a1 = area(P, n1), a2 = area(Q, n2);
  double gI, gA1, gA2;
  if (!z1) {
    double u = a1 + a2 - ai;
    if (!(u > 0)) return;
    gI = g * (a1 + a2) / (u * u);
    gA1 = gA2 = -g * ai / (u * u);
  } else {
    double h1 = z1[1] - z1[0], h2 = z2[1] - z2[0];
    double hz = z_overlap(z1[0], z1[1], z2[0], z2[1]);
    double v = ai * hz, v1 = a1 * h1, v2 = a2 * h2, u = v1 + v2 - v;
    if (!(u > 0) || !(hz > 0)) return;
    double gV = g * (v1 + v2) / (u * u);
    double gV1 = -g * v / (u * u), gV2 = gV1;
    gI = gV * hz;
    double ghz = gV * ai;
    gA1 = gV1 * h1;
    gA2 = gV2 * h2;
    double gh1 = gV1 * a1, gh2 = gV2 * a2;
    gz1[1] += gh1;
    gz1[0] -= gh1;
    gz2[1] += gh2;
    gz2[0] -= gh2;
    /* hz = min(hi1, hi2) - max(lo1, lo2); ties go to the first argument */
    if (z1[1] <= z2[1]) gz1[1] += ghz; else gz2[1] += ghz;
    if (z1[0] >= z2[0]) gz1[0] -= ghz; else gz2[0] -= ghz;
  }
  /* dI/dX over the ordered intersection, routed by provenance code */
  point gX[ORC_CAP];
  for (int k = 0; k < nx; ++k) gX[k] = mkpt(0, 0);
  area_grad(X, nx, gI, gX);
  route_vertex_grads(P, n1, Q, n2, nx, flags, gX, gP, gQ);
  area_grad(P, n1, gA1, gP);
  area_grad(Q, n2, gA2, gQ);
}

/* Sutherland-Hodgman clipping of P by the half-planes of Q (textbook; an
 * algorithm independent of `intersect`, used only as a cross-check). */
static double clip_area(const point *P, int n1, const point *Q, int n2) {
  point buf[2][ORC_MAXV * 4 + 8];
  int n = n1;
  for (int k = 0; k < n1; ++k) buf[0][k] = P[k];
  int cur = 0;
  for (int j = 0; j < n2 && n > 0; ++j) {
    point a = Q[j], b = Q[(j + 1) % n2];
    int nn = 0;
    for (int k = 0; k < n; ++k) {
      point s = buf[cur][k], e = buf[cur][(k + 1) % n];
      double ds = orient(a, b, s), de = orient(a, b, e);
      if (ds >= 0) buf[1 - cur][nn++] = s;
      if ((ds >= 0) != (de >= 0)) {
        double t = ds / (ds - de);
        buf[1 - cur][nn++] = mkpt(s.x + t * (e.x - s.x), s.y + t * (e.y - s.y));
      }
    }
    n = nn;
    cur = 1 - cur;
  }
  return n >= 3 ? area(buf[cur], n) : 0.0;
}

/* ---- batched entry points (fp32 inputs upcast to fp64) ---- */

static int load_poly(const float *xy, const uint8_t *nv, int kmax, int64_t i,
                     point *out) {
  int n = nv ? nv[i] : kmax;
  if (n < 3 || n > kmax) return -1;
  for (int k = 0; k < n; ++k)
    out[k] = mkpt((double)xy[(i * kmax + k) * 2], (double)xy[(i * kmax + k) * 2 + 1]);
  return n;
}

static void load_z(const float *lo, const float *hi, int64_t i, double *z) {
  z[0] = (double)lo[i];
  z[1] = (double)hi[i];
}

/* Input contract of Sec. III for one polygon given by its fp32 coordinates
 * (read as doubles): returns 0 if valid, 1 if the vertex count is outside
 * [3, kmax] (kmax <= 8), 2 if some turn v_k-1 -> v_k -> v_k+1 is not strictly
 * left (clockwise order, a reflex or straight vertex, a repeated vertex),
 * 3 if every turn is left but the boundary turns around more than once (a
 * star polygon such as the pentagram).  The total turning is the sum of the
 * exterior angles, atan2 of each pair of consecutive edges; with every turn
 * left it is 2 pi times the number of times the boundary winds. */
static int polygon_status(const point *v, int n) {
  double turning = 0.0;
  for (int k = 0; k < n; ++k) {
    point a = v[(k + n - 1) % n], b = v[k], c = v[(k + 1) % n];
    if (!(orient(a, b, c) > 0)) return 2;
    point u = psub(b, a), w = psub(c, b);
    turning += atan2(cross2(u, w), u.x * w.x + u.y * w.y);
  }
  const double turns = turning / (2.0 * acos(-1.0));
  return fabs(turns - 1.0) < 0.5 ? 0 : 3;
}

int oracle_polygon_status(const float *xy, int n, int kmax) {
  if (kmax < 3 || kmax > ORC_MAXV || n < 3 || n > kmax) return 1;
  point v[ORC_MAXV];
  for (int k = 0; k < n; ++k) v[k] = mkpt((double)xy[2 * k], (double)xy[2 * k + 1]);
  return polygon_status(v, n);
}

/* Returns 1 iff the polygon (fp64 coordinates) is valid (Sec. III): 3..8
 * vertices, strictly convex, counter-clockwise, winding once. */
int oracle_polygon_valid(const double *xy, int n) {
  if (n < 3 || n > ORC_MAXV) return 0;
  point v[ORC_MAXV];
  for (int k = 0; k < n; ++k) v[k] = mkpt(xy[2 * k], xy[2 * k + 1]);
  return polygon_status(v, n) == 0;
}

/* Status of polygons [lo, hi) of a [count][kmax][2] fp32 array. */
void oracle_polygon_statuses(int64_t lo, int64_t hi, const float *xy, const uint8_t *nv, int kmax,
                             uint8_t *status) {
  for (int64_t i = lo; i < hi; ++i) {
    const int n = nv ? (int)nv[i] : kmax;
    status[i] = (uint8_t)oracle_polygon_status(xy + i * (int64_t)kmax * 2, n, kmax);
  }
}

/* Intersection polygon of one pair; writes m vertices and codes, returns m
 * (or -1 past capacity). */
int oracle_intersect(const double *p, int n1, const double *q, int n2,
                     double *out_xy, uint8_t *out_codes) {
  point P[ORC_MAXV], Q[ORC_MAXV];
  polygon X;
  if (n1 < 3 || n1 > ORC_MAXV || n2 < 3 || n2 > ORC_MAXV) return -1;
  for (int k = 0; k < n1; ++k) P[k] = mkpt(p[2 * k], p[2 * k + 1]);
  for (int k = 0; k < n2; ++k) Q[k] = mkpt(q[2 * k], q[2 * k + 1]);
  int m = intersect(P, n1, Q, n2, &X);
  for (int k = 0; k < m; ++k) {
    out_xy[2 * k] = X.v[k].x;
    out_xy[2 * k + 1] = X.v[k].y;
    out_codes[k] = X.code[k];
  }
  return m;
}

double oracle_area(const double *xy, int n) {
  point v[ORC_CAP];
  if (n < 0 || n > ORC_CAP) return 0.0;
  for (int k = 0; k < n; ++k) v[k] = mkpt(xy[2 * k], xy[2 * k + 1]);
  return area(v, n);
}

double oracle_clip_area(const double *p, int n1, const double *q, int n2) {
  point P[ORC_MAXV], Q[ORC_MAXV];
  if (n1 < 3 || n1 > ORC_MAXV || n2 < 3 || n2 > ORC_MAXV) return -1.0;
  for (int k = 0; k < n1; ++k) P[k] = mkpt(p[2 * k], p[2 * k + 1]);
  for (int k = 0; k < n2; ++k) Q[k] = mkpt(q[2 * k], q[2 * k + 1]);
  return clip_area(P, n1, Q, n2);
}

/* IoU of pairs (a[i], b[i]) for i in [lo, hi).  a_zlo == NULL => 2D.
 * xflags is [n][ka+kb] (0xFF padded).  Returns the number of pairs whose
 * input was invalid or overflowed the capacity. */
int64_t oracle_iou_pairs(int64_t lo, int64_t hi, const float *a_xy,
                         const uint8_t *a_nv, int ka, const float *a_zlo,
                         const float *a_zhi, const float *b_xy,
                         const uint8_t *b_nv, int kb, const float *b_zlo,
                         const float *b_zhi, double *iou, uint8_t *nx,
                         uint8_t *xflags) {
  int64_t bad = 0;
  int cap = ka + kb;
  for (int64_t i = lo; i < hi; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV];
    double z1[2], z2[2];
    int n1 = load_poly(a_xy, a_nv, ka, i, P), n2 = load_poly(b_xy, b_nv, kb, i, Q);
    int err = 0;
    if (n1 < 0 || n2 < 0) {
      iou[i] = 0.0;
      if (nx) nx[i] = 0;
      if (xflags) memset(xflags + i * cap, 0xFF, (size_t)cap);
      ++bad;
      continue;
    }
    if (a_zlo) {
      load_z(a_zlo, a_zhi, i, z1);
      load_z(b_zlo, b_zhi, i, z2);
    }
    iou[i] = iou_pair(P, n1, Q, n2, a_zlo ? z1 : NULL, a_zlo ? z2 : NULL,
                      nx ? nx + i : NULL, xflags ? xflags + i * cap : NULL, cap, &err);
    bad += err;
  }
  return bad;
}

/* Gradient of sum_i g[i] * IoU(a[i], b[i]) for i in [lo, hi), from the saved
 * nx / xflags.  ga_xy, gb_xy are [n][k][2] (padded slots written 0);
 * ga_z, gb_z are [n][2] = (d/dzlo, d/dzhi), or NULL for 2D. */
void oracle_iou_pairs_grad(int64_t lo, int64_t hi, const float *a_xy,
                           const uint8_t *a_nv, int ka, const float *a_zlo,
                           const float *a_zhi, const float *b_xy,
                           const uint8_t *b_nv, int kb, const float *b_zlo,
                           const float *b_zhi, const double *g,
                           const uint8_t *nx, const uint8_t *xflags,
                           double *ga_xy, double *gb_xy, double *ga_z,
                           double *gb_z) {
  int cap = ka + kb;
  for (int64_t i = lo; i < hi; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV], gP[ORC_MAXV], gQ[ORC_MAXV];
    double z1[2], z2[2], gz1[2], gz2[2];
    for (int k = 0; k < ka * 2; ++k) ga_xy[i * ka * 2 + k] = 0.0;
    for (int k = 0; k < kb * 2; ++k) gb_xy[i * kb * 2 + k] = 0.0;
    if (ga_z) ga_z[2 * i] = ga_z[2 * i + 1] = gb_z[2 * i] = gb_z[2 * i + 1] = 0.0;
    int n1 = load_poly(a_xy, a_nv, ka, i, P), n2 = load_poly(b_xy, b_nv, kb, i, Q);
    if (n1 < 0 || n2 < 0 || nx[i] > n1 + n2) continue;
    if (a_zlo) {
      load_z(a_zlo, a_zhi, i, z1);
      load_z(b_zlo, b_zhi, i, z2);
    }
    iou_grad_pair(P, n1, Q, n2, a_zlo ? z1 : NULL, a_zlo ? z2 : NULL, g[i], nx[i],
                  xflags + i * cap, gP, gQ, gz1, gz2);
    for (int k = 0; k < n1; ++k) {
      ga_xy[(i * ka + k) * 2] = gP[k].x;
      ga_xy[(i * ka + k) * 2 + 1] = gP[k].y;
    }
    for (int k = 0; k < n2; ++k) {
      gb_xy[(i * kb + k) * 2] = gQ[k].x;
      gb_xy[(i * kb + k) * 2 + 1] = gQ[k].y;
    }
    if (ga_z) {
      ga_z[2 * i] = gz1[0];
      ga_z[2 * i + 1] = gz1[1];
      gb_z[2 * i] = gz2[0];
      gb_z[2 * i + 1] = gz2[1];
    }
  }
}

/* Intersection polygons of pairs (a[i], b[i]) for i in [lo, hi) (Sec. III:
 * the convex intersection in a fixed-capacity buffer, with the vertex count
 * and provenance flags of Sec. II-B).  out_xy is [n][ka+kb][2] with slots at
 * and past nx written 0; xflags is 0xFF padded.  Returns the number of pairs
 * whose input was invalid or overflowed the capacity (written empty). */
int64_t oracle_intersect_pairs(int64_t lo, int64_t hi, const float *a_xy,
                               const uint8_t *a_nv, int ka, const float *b_xy,
                               const uint8_t *b_nv, int kb, double *out_xy,
                               uint8_t *nx, uint8_t *xflags) {
  int64_t bad = 0;
  int cap = ka + kb;
  for (int64_t i = lo; i < hi; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV];
    polygon X;
    double *row = out_xy + i * cap * 2;
    for (int k = 0; k < 2 * cap; ++k) row[k] = 0.0;
    memset(xflags + i * cap, 0xFF, (size_t)cap);
    nx[i] = 0;
    int n1 = load_poly(a_xy, a_nv, ka, i, P), n2 = load_poly(b_xy, b_nv, kb, i, Q);
    int m = (n1 < 0 || n2 < 0) ? -1 : intersect(P, n1, Q, n2, &X);
    if (m < 0 || m > cap) {
      ++bad;
      continue;
    }
    nx[i] = (uint8_t)m;
    for (int k = 0; k < m; ++k) {
      row[2 * k] = X.v[k].x;
      row[2 * k + 1] = X.v[k].y;
      xflags[i * cap + k] = X.code[k];
    }
  }
  return bad;
}

/* Gradient, with respect to both polygons of every pair, of
 * sum_i sum_k <g_xy[i][k], X_k(a[i], b[i])> for k < nx[i], the intersection
 * vertices rebuilt from the saved flags.  ga_xy, gb_xy are [n][k][2]
 * (padded slots written 0). */
void oracle_intersect_pairs_grad(int64_t lo, int64_t hi, const float *a_xy,
                                 const uint8_t *a_nv, int ka, const float *b_xy,
                                 const uint8_t *b_nv, int kb, const double *g_xy,
                                 const uint8_t *nx, const uint8_t *xflags,
                                 double *ga_xy, double *gb_xy) {
  int cap = ka + kb;
  for (int64_t i = lo; i < hi; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV], gP[ORC_MAXV], gQ[ORC_MAXV], gX[ORC_CAP];
    for (int k = 0; k < ka * 2; ++k) ga_xy[i * ka * 2 + k] = 0.0;
    for (int k = 0; k < kb * 2; ++k) gb_xy[i * kb * 2 + k] = 0.0;
    int n1 = load_poly(a_xy, a_nv, ka, i, P), n2 = load_poly(b_xy, b_nv, kb, i, Q);
    if (n1 < 0 || n2 < 0 || nx[i] > n1 + n2) continue;
    for (int k = 0; k < n1; ++k) gP[k] = mkpt(0, 0);
    for (int k = 0; k < n2; ++k) gQ[k] = mkpt(0, 0);
    for (int k = 0; k < nx[i]; ++k)
      gX[k] = mkpt(g_xy[(i * cap + k) * 2], g_xy[(i * cap + k) * 2 + 1]);
    route_vertex_grads(P, n1, Q, n2, nx[i], xflags + i * cap, gX, gP, gQ);
    for (int k = 0; k < n1; ++k) {
      ga_xy[(i * ka + k) * 2] = gP[k].x;
      ga_xy[(i * ka + k) * 2 + 1] = gP[k].y;
    }
    for (int k = 0; k < n2; ++k) {
      gb_xy[(i * kb + k) * 2] = gQ[k].x;
      gb_xy[(i * kb + k) * 2 + 1] = gQ[k].y;
    }
  }
}

/* Shoelace areas of polygons i in [lo, hi) (Sec. III), up to 16 vertices
 * (an intersection polygon's capacity), 0 for an invalid vertex count. */
void oracle_areas(int64_t lo, int64_t hi, const float *xy, const uint8_t *nv, int k,
                  double *out) {
  for (int64_t i = lo; i < hi; ++i) {
    point V[ORC_CAP];
    int n = k > ORC_CAP ? -1 : load_poly(xy, nv, k, i, V);
    out[i] = n < 0 ? 0.0 : area(V, n);
  }
}

/* Gradient of sum_i g[i] * area(p[i]); gxy is [n][k][2] (padded slots 0). */
void oracle_areas_grad(int64_t lo, int64_t hi, const float *xy, const uint8_t *nv, int k,
                       const double *g, double *gxy) {
  for (int64_t i = lo; i < hi; ++i) {
    point V[ORC_CAP], gV[ORC_CAP];
    for (int t = 0; t < 2 * k; ++t) gxy[i * k * 2 + t] = 0.0;
    int n = k > ORC_CAP ? -1 : load_poly(xy, nv, k, i, V);
    if (n < 0) continue;
    for (int t = 0; t < n; ++t) gV[t] = mkpt(0, 0);
    area_grad(V, n, g[i], gV);
    for (int t = 0; t < n; ++t) {
      gxy[(i * k + t) * 2] = gV[t].x;
      gxy[(i * k + t) * 2 + 1] = gV[t].y;
    }
  }
}

/* ---- rotated boxes (Sec. IV-A case study): box parameters -> corners ---- */

/* R11: the corners of box (cx, cy, w, l, yaw) are c + R(yaw) (+-l/2, +-w/2),
 * counter-clockwise from (+l/2, -w/2); the length runs along the heading. */
static const double BOX_SL[4] = {1.0, 1.0, -1.0, -1.0};
static const double BOX_SW[4] = {-1.0, 1.0, 1.0, -1.0};

static void box_corners(const float *bx, point *out) {
  double cx = bx[0], cy = bx[1], w = bx[2], l = bx[3], yaw = bx[4];
  double c = cos(yaw), s = sin(yaw);
  for (int k = 0; k < 4; ++k) {
    double dx = 0.5 * BOX_SL[k] * l, dy = 0.5 * BOX_SW[k] * w;
    out[k] = mkpt(cx + c * dx - s * dy, cy + s * dx + c * dy);
  }
}

/* Gradient of L with respect to (cx, cy, w, l, yaw) given dL/dcorner_k. */
static void box_param_grad(const float *bx, const point *gc, double *gp) {
  double w = bx[2], l = bx[3], yaw = bx[4];
  double c = cos(yaw), s = sin(yaw);
  for (int t = 0; t < 5; ++t) gp[t] = 0.0;
  for (int k = 0; k < 4; ++k) {
    double dx = 0.5 * BOX_SL[k] * l, dy = 0.5 * BOX_SW[k] * w;
    gp[0] += gc[k].x;
    gp[1] += gc[k].y;
    /* corner = c + (c dx - s dy, s dx + c dy) */
    gp[2] += 0.5 * BOX_SW[k] * (-s * gc[k].x + c * gc[k].y);
    gp[3] += 0.5 * BOX_SL[k] * (c * gc[k].x + s * gc[k].y);
    gp[4] += gc[k].x * (-s * dx - c * dy) + gc[k].y * (c * dx - s * dy);
  }
}

/* IoU of box pairs for i in [lo, hi); boxes are [n][dim] fp32 with dim 5
 * (cx, cy, w, l, yaw) for 2D or 7 (..., z, h; z the centre, R12) for 3D.
 * The corners are formed in fp64 from the fp32 parameters. */
int64_t oracle_iou_boxes(int64_t lo, int64_t hi, const float *a, const float *b, int dim,
                         double *iou, uint8_t *nx, uint8_t *xflags) {
  int64_t bad = 0;
  for (int64_t i = lo; i < hi; ++i) {
    point P[4], Q[4];
    double z1[2], z2[2];
    const float *ba = a + i * dim, *bb = b + i * dim;
    box_corners(ba, P);
    box_corners(bb, Q);
    if (dim == 7) {
      z1[0] = (double)ba[5] - 0.5 * ba[6];
      z1[1] = (double)ba[5] + 0.5 * ba[6];
      z2[0] = (double)bb[5] - 0.5 * bb[6];
      z2[1] = (double)bb[5] + 0.5 * bb[6];
    }
    int err = 0;
    iou[i] = iou_pair(P, 4, Q, 4, dim == 7 ? z1 : NULL, dim == 7 ? z2 : NULL,
                      nx ? nx + i : NULL, xflags ? xflags + i * 8 : NULL, 8, &err);
    bad += err;
  }
  return bad;
}

/* Gradient of sum_i g[i] * IoU(a[i], b[i]) with respect to the box
 * parameters, from the saved nx / xflags: the corner gradient of the IoU
 * backward, then the chain rule of the corner formula (and of
 * zlo = z - h/2, zhi = z + h/2 in 3D). */
void oracle_iou_boxes_grad(int64_t lo, int64_t hi, const float *a, const float *b, int dim,
                           const double *g, const uint8_t *nx, const uint8_t *xflags,
                           double *ga, double *gb) {
  for (int64_t i = lo; i < hi; ++i) {
    point P[4], Q[4], gP[4], gQ[4];
    double z1[2], z2[2], gz1[2], gz2[2], gpa[5], gpb[5];
    const float *ba = a + i * dim, *bb = b + i * dim;
    box_corners(ba, P);
    box_corners(bb, Q);
    if (dim == 7) {
      z1[0] = (double)ba[5] - 0.5 * ba[6];
      z1[1] = (double)ba[5] + 0.5 * ba[6];
      z2[0] = (double)bb[5] - 0.5 * bb[6];
      z2[1] = (double)bb[5] + 0.5 * bb[6];
    }
    for (int t = 0; t < dim; ++t) ga[i * dim + t] = gb[i * dim + t] = 0.0;
    if (nx[i] > 8) continue;
    iou_grad_pair(P, 4, Q, 4, dim == 7 ? z1 : NULL, dim == 7 ? z2 : NULL, g[i], nx[i],
                  xflags + i * 8, gP, gQ, gz1, gz2);
    box_param_grad(ba, gP, gpa);
    box_param_grad(bb, gQ, gpb);
    for (int t = 0; t < 5; ++t) {
      ga[i * dim + t] = gpa[t];
      gb[i * dim + t] = gpb[t];
    }
    if (dim == 7) {
      ga[i * dim + 5] = gz1[0] + gz1[1];
      ga[i * dim + 6] = 0.5 * (gz1[1] - gz1[0]);
      gb[i * dim + 5] = gz2[0] + gz2[1];
      gb[i * dim + 6] = 0.5 * (gz2[1] - gz2[0]);
    }
  }
}

/* IoU of index pairs (a[ia[t]], b[ib[t]]) for t in [lo, hi): the same
 * arithmetic as oracle_iou_pairs, for sampled entries of a matrix. */
int64_t oracle_iou_index_pairs(int64_t lo, int64_t hi, const int64_t *ia,
                               const int64_t *ib, const float *a_xy,
                               const uint8_t *a_nv, int ka, const float *a_zlo,
                               const float *a_zhi, const float *b_xy,
                               const uint8_t *b_nv, int kb, const float *b_zlo,
                               const float *b_zhi, double *iou, uint8_t *nx,
                               uint8_t *xflags) {
  int64_t bad = 0;
  int cap = ka + kb;
  for (int64_t t = lo; t < hi; ++t) {
    point P[ORC_MAXV], Q[ORC_MAXV];
    double z1[2], z2[2];
    int err = 0;
    int n1 = load_poly(a_xy, a_nv, ka, ia[t], P), n2 = load_poly(b_xy, b_nv, kb, ib[t], Q);
    if (n1 < 0 || n2 < 0) {
      iou[t] = 0.0;
      ++bad;
      continue;
    }
    if (a_zlo) {
      load_z(a_zlo, a_zhi, ia[t], z1);
      load_z(b_zlo, b_zhi, ib[t], z2);
    }
    iou[t] = iou_pair(P, n1, Q, n2, a_zlo ? z1 : NULL, a_zlo ? z2 : NULL,
                      nx ? nx + t : NULL, xflags ? xflags + t * cap : NULL, cap, &err);
    bad += err;
  }
  return bad;
}

/* Segmented IoU matrix: for each segment s, rows a[a_off[s]..a_off[s+1]) and
 * columns b[b_off[s]..b_off[s+1]) fill the row-major block that starts at
 * out_off[s].  self_pairs != 0 means b is a (same offsets) and the diagonal
 * of each block is 1 (the IoU of a polygon with itself); entry (r, c) is then
 * the pair evaluated with the lower index first (R25). */
void oracle_iou_matrix(int nseg, const int64_t *a_off, const int64_t *b_off,
                       const int64_t *out_off, int self_pairs, const float *a_xy,
                       const uint8_t *a_nv, int ka, const float *a_zlo,
                       const float *a_zhi, const float *b_xy,
                       const uint8_t *b_nv, int kb, const float *b_zlo,
                       const float *b_zhi, double *iou) {
  for (int s = 0; s < nseg; ++s) {
    int64_t na = a_off[s + 1] - a_off[s], nb = b_off[s + 1] - b_off[s];
    for (int64_t r = 0; r < na; ++r)
      for (int64_t c = 0; c < nb; ++c) {
        int64_t ia = a_off[s] + r, ib = b_off[s] + c;
        double *o = iou + out_off[s] + r * nb + c;
        if (self_pairs && r == c) {
          *o = 1.0;
          continue;
        }
        if (self_pairs && r > c) { /* R25: the unordered pair, lower index first */
          int64_t t = ia;
          ia = ib;
          ib = t;
        }
        oracle_iou_index_pairs(0, 1, &ia, &ib, a_xy, a_nv, ka, a_zlo, a_zhi, b_xy,
                               b_nv, kb, b_zlo, b_zhi, o, NULL, NULL);
      }
  }
}

/* Gradient of sum g * IoU over a segmented matrix (layout as above).  Rows
 * accumulate into ga, columns into gb (into ga as well when self_pairs, whose
 * diagonal is the constant 1 and contributes nothing; entry (r, c) with r > c
 * is the pair (c, r) of R25, so its P gradient goes to box c and its Q
 * gradient to box r).  Outputs are overwritten.  ga_z/gb_z may be NULL for
 * 2D. */
void oracle_iou_matrix_grad(int nseg, const int64_t *a_off, const int64_t *b_off,
                            const int64_t *out_off, int self_pairs,
                            const float *a_xy, const uint8_t *a_nv, int ka,
                            const float *a_zlo, const float *a_zhi,
                            const float *b_xy, const uint8_t *b_nv, int kb,
                            const float *b_zlo, const float *b_zhi,
                            const double *g, double *ga_xy, double *gb_xy,
                            double *ga_z, double *gb_z, int64_t n_a, int64_t n_b) {
  for (int64_t k = 0; k < n_a * ka * 2; ++k) ga_xy[k] = 0.0;
  if (!self_pairs)
    for (int64_t k = 0; k < n_b * kb * 2; ++k) gb_xy[k] = 0.0;
  if (ga_z) {
    for (int64_t k = 0; k < n_a * 2; ++k) ga_z[k] = 0.0;
    if (!self_pairs)
      for (int64_t k = 0; k < n_b * 2; ++k) gb_z[k] = 0.0;
  }
  double *gbx = self_pairs ? ga_xy : gb_xy;
  double *gbz = self_pairs ? ga_z : gb_z;
  int cap = ka + kb;
  for (int s = 0; s < nseg; ++s) {
    int64_t na = a_off[s + 1] - a_off[s], nb = b_off[s + 1] - b_off[s];
    for (int64_t r = 0; r < na; ++r)
      for (int64_t c = 0; c < nb; ++c) {
        if (self_pairs && r == c) continue;
        int64_t ia = a_off[s] + r, ib = b_off[s] + c;
        if (self_pairs && r > c) { /* R25 */
          int64_t t = ia;
          ia = ib;
          ib = t;
        }
        point P[ORC_MAXV], Q[ORC_MAXV], gP[ORC_MAXV], gQ[ORC_MAXV];
        double z1[2], z2[2], gz1[2], gz2[2];
        uint8_t nx, flags[ORC_CAP];
        int err = 0;
        int n1 = load_poly(a_xy, a_nv, ka, ia, P), n2 = load_poly(b_xy, b_nv, kb, ib, Q);
        if (n1 < 0 || n2 < 0) continue;
        if (a_zlo) {
          load_z(a_zlo, a_zhi, ia, z1);
          load_z(b_zlo, b_zhi, ib, z2);
        }
        const double *pz1 = a_zlo ? z1 : NULL, *pz2 = a_zlo ? z2 : NULL;
        iou_pair(P, n1, Q, n2, pz1, pz2, &nx, flags, cap, &err);
        if (err) continue;
        iou_grad_pair(P, n1, Q, n2, pz1, pz2, g[out_off[s] + r * nb + c], nx, flags,
                      gP, gQ, gz1, gz2);
        for (int k = 0; k < n1; ++k) {
          ga_xy[(ia * ka + k) * 2] += gP[k].x;
          ga_xy[(ia * ka + k) * 2 + 1] += gP[k].y;
        }
        for (int k = 0; k < n2; ++k) {
          gbx[(ib * kb + k) * 2] += gQ[k].x;
          gbx[(ib * kb + k) * 2 + 1] += gQ[k].y;
        }
        if (ga_z) {
          ga_z[2 * ia] += gz1[0];
          ga_z[2 * ia + 1] += gz1[1];
          gbz[2 * ib] += gz2[0];
          gbz[2 * ib + 1] += gz2[1];
        }
      }
  }
}

/* Degeneracy margins of pairs [lo, hi), five per pair (used to select the
 * generator-filtered parity set):
 *   [0] min |orient(e_s, e_e, v)| / (|e_e - e_s| * L) over all vertex/edge
 *       tests, L = bounding-box diagonal of P u Q;
 *   [1] min |sin| of the angle between two crossing edges (1 if none);
 *   [2] min normalised turn orient/(|u||w|) over the vertices of P and Q;
 *   [3] min normalised cross product between consecutive ordered intersection
 *       vertices seen from the centroid (1 if empty);
 *   [4] intersection area over the smaller polygon area (1 if empty): a
 *       sliver sits next to the change to an empty intersection. */
void oracle_pair_margins(int64_t lo, int64_t hi, const float *a_xy,
                         const uint8_t *a_nv, int ka, const float *b_xy,
                         const uint8_t *b_nv, int kb, double *out) {
  for (int64_t i = lo; i < hi; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV];
    double *o = out + 5 * i;
    int n1 = load_poly(a_xy, a_nv, ka, i, P), n2 = load_poly(b_xy, b_nv, kb, i, Q);
    if (n1 < 0 || n2 < 0) {
      o[0] = o[1] = o[2] = o[3] = o[4] = 0.0;
      continue;
    }
    double xmin = P[0].x, xmax = P[0].x, ymin = P[0].y, ymax = P[0].y;
    for (int k = 0; k < n1; ++k) {
      xmin = fmin(xmin, P[k].x); xmax = fmax(xmax, P[k].x);
      ymin = fmin(ymin, P[k].y); ymax = fmax(ymax, P[k].y);
    }
    for (int k = 0; k < n2; ++k) {
      xmin = fmin(xmin, Q[k].x); xmax = fmax(xmax, Q[k].x);
      ymin = fmin(ymin, Q[k].y); ymax = fmax(ymax, Q[k].y);
    }
    double L = hypot(xmax - xmin, ymax - ymin);
    double dmin = INFINITY, smin = 1.0, tmin = INFINITY, gmin = 1.0;
    for (int i2 = 0; i2 < n1; ++i2)
      for (int j = 0; j < n2; ++j) {
        point q0 = Q[j], q1 = Q[(j + 1) % n2], p0 = P[i2], p1 = P[(i2 + 1) % n1];
        double d1 = fabs(orient(q0, q1, p0)) / (hypot(q1.x - q0.x, q1.y - q0.y) * L);
        double d2 = fabs(orient(p0, p1, q0)) / (hypot(p1.x - p0.x, p1.y - p0.y) * L);
        dmin = fmin(dmin, fmin(d1, d2));
      }
    for (int k = 0; k < n1; ++k) {
      point a = P[(k + n1 - 1) % n1], b = P[k], c = P[(k + 1) % n1];
      point u = psub(b, a), w = psub(c, b);
      tmin = fmin(tmin, cross2(u, w) / (hypot(u.x, u.y) * hypot(w.x, w.y)));
    }
    for (int k = 0; k < n2; ++k) {
      point a = Q[(k + n2 - 1) % n2], b = Q[k], c = Q[(k + 1) % n2];
      point u = psub(b, a), w = psub(c, b);
      tmin = fmin(tmin, cross2(u, w) / (hypot(u.x, u.y) * hypot(w.x, w.y)));
    }
    polygon X;
    int m = intersect(P, n1, Q, n2, &X);
    for (int k = 0; k < m; ++k) {
      uint8_t code = X.code[k];
      if (code >= 0x40) {
        int a = (code >> 3) & 7, b = code & 7;
        point e = psub(P[(a + 1) % n1], P[a]), f = psub(Q[(b + 1) % n2], Q[b]);
        smin = fmin(smin, fabs(cross2(e, f)) / (hypot(e.x, e.y) * hypot(f.x, f.y)));
      }
    }
    if (m >= 3) {
      point c = mkpt(0, 0);
      for (int k = 0; k < m; ++k) { c.x += X.v[k].x; c.y += X.v[k].y; }
      c.x /= m;
      c.y /= m;
      for (int k = 0; k < m; ++k) {
        point u = psub(X.v[k], c), w = psub(X.v[(k + 1) % m], c);
        gmin = fmin(gmin, cross2(u, w) / (hypot(u.x, u.y) * hypot(w.x, w.y)));
      }
    } else if (m > 0) {
      gmin = 0.0;
    }
    double sliver = 1.0;
    if (m >= 3) {
      double a1 = area(P, n1), a2 = area(Q, n2);
      sliver = area(X.v, m) / (a1 < a2 ? a1 : a2);
    } else if (m > 0) {
      sliver = 0.0;
    }
    o[0] = dmin;
    o[1] = smin;
    o[2] = tmin;
    o[3] = gmin;
    o[4] = sliver;
  }
}

/* ---- fp64-input entry points (finite differences need steps that are not
 * rounded to fp32).  Polygons are [n][k][2] doubles with k vertices each. ---- */

void oracle_iou_pairs_f64(int64_t n, const double *a_xy, int ka,
                          const double *a_z, const double *b_xy, int kb,
                          const double *b_z, double *iou, uint8_t *nx,
                          uint8_t *xflags) {
  int cap = ka + kb;
  for (int64_t i = 0; i < n; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV];
    int err = 0;
    for (int k = 0; k < ka; ++k) P[k] = mkpt(a_xy[(i * ka + k) * 2], a_xy[(i * ka + k) * 2 + 1]);
    for (int k = 0; k < kb; ++k) Q[k] = mkpt(b_xy[(i * kb + k) * 2], b_xy[(i * kb + k) * 2 + 1]);
    iou[i] = iou_pair(P, ka, Q, kb, a_z ? a_z + 2 * i : NULL, a_z ? b_z + 2 * i : NULL,
                      nx + i, xflags + i * cap, cap, &err);
  }
}

void oracle_iou_pairs_grad_f64(int64_t n, const double *a_xy, int ka,
                               const double *a_z, const double *b_xy, int kb,
                               const double *b_z, const double *g,
                               const uint8_t *nx, const uint8_t *xflags,
                               double *ga_xy, double *gb_xy, double *ga_z,
                               double *gb_z) {
  int cap = ka + kb;
  for (int64_t i = 0; i < n; ++i) {
    point P[ORC_MAXV], Q[ORC_MAXV], gP[ORC_MAXV], gQ[ORC_MAXV];
    double gz1[2], gz2[2];
    for (int k = 0; k < ka; ++k) P[k] = mkpt(a_xy[(i * ka + k) * 2], a_xy[(i * ka + k) * 2 + 1]);
    for (int k = 0; k < kb; ++k) Q[k] = mkpt(b_xy[(i * kb + k) * 2], b_xy[(i * kb + k) * 2 + 1]);
    iou_grad_pair(P, ka, Q, kb, a_z ? a_z + 2 * i : NULL, a_z ? b_z + 2 * i : NULL, g[i],
                  nx[i], xflags + i * cap, gP, gQ, gz1, gz2);
    for (int k = 0; k < ka; ++k) {
      ga_xy[(i * ka + k) * 2] = gP[k].x;
      ga_xy[(i * ka + k) * 2 + 1] = gP[k].y;
    }
    for (int k = 0; k < kb; ++k) {
      gb_xy[(i * kb + k) * 2] = gQ[k].x;
      gb_xy[(i * kb + k) * 2 + 1] = gQ[k].y;
    }
    if (ga_z) {
      ga_z[2 * i] = a_z ? gz1[0] : 0.0;
      ga_z[2 * i + 1] = a_z ? gz1[1] : 0.0;
      gb_z[2 * i] = a_z ? gz2[0] : 0.0;
      gb_z[2 * i + 1] = a_z ? gz2[1] : 0.0;
    }
  }
}
