// simple.hip -- IoU of simple polygons (counter-clockwise, not necessarily
// convex), forward and backward, one wavefront lane per pair, grid-stride.
//
// Sec. III keeps polygons convex and plans arbitrary ones; this is that
// extension, written for the GPU without the convex path's vertex sort.  By
// Green's theorem the area of P n Q is half the integral of x dy - y dx over
// its boundary, which is made of the parts of P's edges inside Q and of Q's
// edges inside P.  Along edge i of P (P_i + t e_i, t in [0, 1]) that integral
// is cross(P_i, P_i+1) times the fraction of the edge inside Q, and that
// fraction needs no sorting: it starts at 1 or 0 (P_i inside Q or not) and
// each crossing at t_k changes the inside length by +-(1 - t_k) (+ where the
// edge enters Q, - where it leaves), a crossing near the edge's start being
// written as +-1 -+ t_k so that short inside parts keep their precision.  Inclusion of P_0 in Q is one
// crossing-number test; every later vertex follows by the parity of the
// crossings on the edge before it.  Moving a vertex moves its two edges: the
// area changes by the edges' outward normals (dy, -dx) weighted by the
// integrals of (1 - t) and of t over their inside parts, which come from the
// same crossings ((1 - t_k)^2 / 2 and (1 - t_k^2) / 2 per crossing).
//
// Signs are the convex path's: certified fp32 orientations with an exact fp64
// fallback, and exact contacts resolved as if Q were moved by (eps, eps^2).
// The forward saves, per pair, the crossing mask (bit 8 i + j: edge i of a
// crosses edge j of b), the entering mask (the same bit when edge i enters b
// there) and the inclusion of each polygon's vertex 0 in the other; the
// backward needs nothing else.
#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

namespace {

template <int K>
constexpr int simple_block() {
  return K == 8 ? 128 : 256;
}

// At K = 8 both kernels are held to 3 waves per SIMD (at most 168 VGPRs):
// left alone the backward takes more and runs 2; held to 4 it spills
// 36 bytes a lane to scratch (HBM traffic) and measured slower.
template <int K>
constexpr int simple_waves() {
  return K == 8 ? 3 : 1;
}

// Row masks of the tie-ruled sign table: bit j of spr[i] when P_i is strictly
// left of Q's edge j, bit j of sqr[i] when Q_j is strictly left of P's edge i.
// Returns true when the lane took the exact fp64 branch.
template <int K, int BLOCK>
__device__ __forceinline__ bool sign_rows(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                          const float (&epx)[K], const float (&epy)[K],
                                          const float (&eqx)[K], const float (&eqy)[K], float E,
                                          float2* __restrict__ s_q, uint32_t (&spr)[K],
                                          uint32_t (&sqr)[K]) {
  constexpr uint32_t KM = (1u << K) - 1u;
  float D = 0.f, omin = __builtin_inff();
#pragma unroll
  for (int i = 0; i < K; ++i) {
    uint32_t wp = 0u, wq = 0u;  // sign bits shifted in at bit 0, j descending: bit j = sign
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
      const float dx = P.x[i] - Q.x[j], dy = P.y[i] - Q.y[j];
      const float op = eqx[j] * dy - eqy[j] * dx;
      const float oq = epy[i] * dx - epx[i] * dy;
      wp = __builtin_amdgcn_alignbit(wp, __float_as_uint(op), 31);
      wq = __builtin_amdgcn_alignbit(wq, __float_as_uint(oq), 31);
      D = fmaxf(D, fmaxf(fabsf(dx), fabsf(dy)));
      const float mo = fminf(fabsf(op), fabsf(oq));
      omin = fminf(omin, (i < n1 && j < n2) ? mo : __builtin_inff());
    }
    spr[i] = ~wp & KM;
    sqr[i] = ~wq & KM;
  }
  const bool exact = !(omin > kCertify * E * D);
  if (exact) {
    // exact signs in fp64; exact zeros take the sign of Q moved by (eps, eps^2)
#pragma unroll
    for (int k = 0; k < K; ++k) s_q[k * BLOCK] = make_float2(Q.x[k], Q.y[k]);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const float pnx = next_of<K, false>(P.x, i, n1), pny = next_of<K, false>(P.y, i, n1);
      const bool tie_p = (P.y[i] != pny) ? (P.y[i] > pny) : (pnx > P.x[i]);
      uint32_t rp = spr[i], rq = sqr[i];
#pragma unroll 1
      for (int j = 0; j < K; ++j) {
        const int jn = j + 1 < n2 ? j + 1 : 0;
        const float2 q = s_q[j * BLOCK], qn = s_q[jn * BLOCK];
        const bool tie_q = (qn.y != q.y) ? (qn.y > q.y) : (q.x > qn.x);
        const double op = orient64(q.x, q.y, qn.x, qn.y, P.x[i], P.y[i]);
        const double oq = orient64(P.x[i], P.y[i], pnx, pny, q.x, q.y);
        const uint32_t bit = 1u << j;
        rp = (rp & ~bit) | ((op > 0.0 || (op == 0.0 && tie_q)) ? bit : 0u);
        rq = (rq & ~bit) | ((oq > 0.0 || (oq == 0.0 && tie_p)) ? bit : 0u);
      }
      spr[i] = rp;
      sqr[i] = rq;
    }
  }
  return exact;
}

// Crossing-number inclusion of P_0 in Q (and of Q_0 in P) from the sign rows
// and exact comparisons, under the same (eps, eps^2) motion of Q: a crossing
// edge hits the ray to +x when the point is on the side of the edge that the
// edge's upward direction leaves on its left.
template <int K>
__device__ __forceinline__ uint32_t vertex0_inclusion(const Poly<K>& P, int n1, const Poly<K>& Q,
                                                      int n2, const uint32_t (&spr)[K],
                                                      const uint32_t (&sqr)[K]) {
  uint32_t in_p = 0u, in_q = 0u;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < n2) {
      const float qny = next_of<K, false>(Q.y, j, n2);
      const bool up0 = Q.y[j] >= P.y[0], up1 = qny >= P.y[0];
      const bool left = (spr[0] >> j) & 1u;
      in_p ^= (up0 != up1 && left == up1) ? 1u : 0u;
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    if (i < n1) {
      const float pny = next_of<K, false>(P.y, i, n1);
      const bool up0 = P.y[i] > Q.y[0], up1 = pny > Q.y[0];
      const bool left = sqr[i] & 1u;
      in_q ^= (up0 != up1 && left == up1) ? 1u : 0u;
    }
  }
  return in_p | (in_q << 1);
}

// Parity of the set bits of a byte.
__device__ __forceinline__ uint32_t parity8(uint32_t v) { return __builtin_popcount(v & 0xffu) & 1u; }

// Per-edge sums over the crossings.  Along P's edge i the inside fraction is
// its start vertex's inclusion plus, per crossing at t with s = +1 where the
// edge enters Q (-1 where it leaves), s (1 - t); the integrals of (1 - t) and
// of t over the inside part add s (1 - t)^2 / 2 and s (1 - t^2) / 2.  Each
// crossing is anchored at its nearer end of the edge: one at t < 1/2 puts s
// into an integer base B (s / 2 into both integrals' bases) and contributes
// -s t, -s t (2 - t) / 2 and -s t^2 / 2 instead, so that a short inside part
// at either end keeps its relative precision (written as 1 - (1 - t) it
// would lose u / t of it).  Per P edge: B, L (the fraction's terms), W1, W2
// (the integrals' terms).  Q's edges take the same sums in their own
// parameter s (the crossing's projection on the edge) with the opposite
// sign (an edge of P entering Q is an edge of Q leaving P there), kept in
// this lane's LDS column: (B', M, V1, V2) per edge of Q.
//
// Each edge of P walks the set bits of its crossing row (a wavefront takes
// as many steps as its busiest lane's row has crossings); the crossed edge of
// Q is read from this lane's LDS column (s_q: Q's vertices).
template <int K, bool GRAD, int BLOCK>
__device__ __forceinline__ void crossing_sums(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                              const float (&epx)[K], const float (&epy)[K],
                                              const uint32_t (&xrow)[K], const uint32_t (&erow)[K],
                                              bool exact, float2* __restrict__ s_q,
                                              float4* __restrict__ s_acc, float (&B)[K],
                                              float (&L)[K], float (&W1)[K], float (&W2)[K],
                                              float (&Bq)[K], float (&M)[K], float (&V1)[K],
                                              float (&V2)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s_q[k * BLOCK] = make_float2(Q.x[k], Q.y[k]);
    s_acc[k * BLOCK] = make_float4(0.f, 0.f, 0.f, 0.f);
    B[k] = 0.f;
    L[k] = 0.f;
    W1[k] = 0.f;
    W2[k] = 0.f;
  }
  // Q's sums: .x base, .y fraction terms, .z / .w the integrals' terms
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int inx = next_idx<K, false>(i, n1);
    uint32_t row = xrow[i];
    const uint32_t er = erow[i];
    while (row) {
      const uint32_t j = (uint32_t)__builtin_ctz(row);
      row &= row - 1u;
      const uint32_t jn = j + 1u < (uint32_t)n2 ? j + 1u : 0u;
      const float2 q = s_q[j * BLOCK], qn = s_q[jn * BLOCK];
      // the sign table's expressions (Q's edge as next_of - vertex)
      const float fx = qn.x - q.x, fy = qn.y - q.y;
      float o0, o1;
      if (!exact) {
        o0 = fx * (P.y[i] - q.y) - fy * (P.x[i] - q.x);
        o1 = fx * (P.y[inx] - q.y) - fy * (P.x[inx] - q.x);
      } else {
        o0 = (float)orient64(q.x, q.y, qn.x, qn.y, P.x[i], P.y[i]);
        o1 = (float)orient64(q.x, q.y, qn.x, qn.y, P.x[inx], P.y[inx]);
      }
      // The crossing point X = P_i + t e_i; its parameter on Q's edge is X's
      // projection onto that edge, not a second independent quotient: where
      // the edges meet at a shallow angle both parameters are uncertain
      // along the edges, and only a shared point keeps the two edges'
      // contributions consistent (an error of X along the boundary then
      // changes the area in proportion to the angle only).  t and 1 - t each
      // come from their own quotient (o0 and -o1 over o0 - o1), s and 1 - s
      // from X's offsets to both ends of Q's edge.
      const float idn = fast_rcp(o0 - o1);
      const float t = fminf(fmaxf(o0 * idn, 0.f), 1.f);
      const float ut = fminf(fmaxf(-o1 * idn, 0.f), 1.f);
      const float rx = fmaf(t, epx[i], P.x[i] - q.x), ry = fmaf(t, epy[i], P.y[i] - q.y);
      const float vx = fmaf(-t, epx[i], qn.x - P.x[i]), vy = fmaf(-t, epy[i], qn.y - P.y[i]);
      const float ifn = fast_rcp(fmaf(fx, fx, fy * fy));
      const float sq = fminf(fmaxf((rx * fx + ry * fy) * ifn, 0.f), 1.f);
      const float us = fminf(fmaxf((vx * fx + vy * fy) * ifn, 0.f), 1.f);
      const float sg = ((er >> j) & 1u) ? 1.f : -1.f;
      const bool near_p = t < 0.5f;  // anchored at the edge's start
      B[i] += near_p ? sg : 0.f;
      float4 a = s_acc[j * BLOCK];
      const bool near_q = sq < 0.5f;
      a.x += near_q ? -sg : 0.f;
      if (GRAD) {
        // the fraction's term is the sum of the integrals' terms (int (1 - t)
        // + int t over the inside part is its length): not kept apart
        W1[i] = fmaf(0.5f * sg, near_p ? -t * (2.f - t) : ut * ut, W1[i]);
        W2[i] = fmaf(0.5f * sg, near_p ? -t * t : ut * (1.f + t), W2[i]);
        a.z = fmaf(-0.5f * sg, near_q ? -sq * (2.f - sq) : us * us, a.z);
        a.w = fmaf(-0.5f * sg, near_q ? -sq * sq : us * (1.f + sq), a.w);
      } else {
        L[i] = fmaf(sg, near_p ? -t : ut, L[i]);
        a.y = fmaf(-sg, near_q ? -sq : us, a.y);
      }
      s_acc[j * BLOCK] = a;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float4 a = s_acc[k * BLOCK];
    Bq[k] = a.x;
    V1[k] = a.z;
    V2[k] = a.w;
    M[k] = GRAD ? a.z + a.w : a.y;
    if (GRAD) L[k] = W1[k] + W2[k];
  }
}

// Edge vectors (padded slots repeat vertex 0, so their edges are zero) and
// the largest edge component.
template <int K>
__device__ __forceinline__ float edges(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                       float (&epx)[K], float (&epy)[K], float (&eqx)[K],
                                       float (&eqy)[K]) {
  float E = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    epx[k] = next_of<K, false>(P.x, k, n1) - P.x[k];
    epy[k] = next_of<K, false>(P.y, k, n1) - P.y[k];
    eqx[k] = next_of<K, false>(Q.x, k, n2) - Q.x[k];
    eqy[k] = next_of<K, false>(Q.y, k, n2) - Q.y[k];
    E = fmaxf(E, fmaxf(fmaxf(fabsf(epx[k]), fabsf(epy[k])), fmaxf(fabsf(eqx[k]), fabsf(eqy[k]))));
  }
  return E;
}

// Inclusion of every vertex: P_i+1 differs from P_i by the parity of the
// crossings on edge i; Q_j+1 from Q_j by that of column j.
template <int K>
__device__ __forceinline__ void vertex_inclusion(uint32_t inside, const uint32_t (&xrow)[K],
                                                 float (&ep)[K], float (&eq)[K]) {
  uint32_t a = inside & 1u, b = (inside >> 1) & 1u;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ep[k] = a ? 1.f : 0.f;
    eq[k] = b ? 1.f : 0.f;
    a ^= parity8(xrow[k]);
    uint32_t col = 0u;
#pragma unroll
    for (int i = 0; i < K; ++i) col ^= (xrow[i] >> k) & 1u;
    b ^= col;
  }
}

// Cross products of consecutive vertices in the frame centred on P_0 (twice
// the signed area of each edge's triangle with P_0), zero on padded edges.
template <int K>
__device__ __forceinline__ void edge_cross(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                           float (&cp)[K], float (&cq)[K]) {
  const float ox = P.x[0], oy = P.y[0];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float ax = P.x[k] - ox, ay = P.y[k] - oy;
    const float bx = next_of<K, false>(P.x, k, n1) - ox, by = next_of<K, false>(P.y, k, n1) - oy;
    cp[k] = k < n1 ? ax * by - ay * bx : 0.f;
    const float cx = Q.x[k] - ox, cy = Q.y[k] - oy;
    const float dx = next_of<K, false>(Q.x, k, n2) - ox, dy = next_of<K, false>(Q.y, k, n2) - oy;
    cq[k] = k < n2 ? cx * dy - cy * dx : 0.f;
  }
}

template <int K>
__global__ __launch_bounds__(simple_block<K>())
__attribute__((amdgpu_waves_per_eu(simple_waves<K>()))) void k_simple_fwd(SimpleFwdArgs args) {
  constexpr int BLOCK = simple_block<K>();
  __shared__ float2 s_q[K * BLOCK];
  __shared__ float4 s_acc[K * BLOCK];
  const int tid = threadIdx.x;
  const int64_t n = args.a.count;
  for (int64_t p = (int64_t)blockIdx.x * BLOCK + tid; p < n; p += (int64_t)gridDim.x * BLOCK) {
    const int n1 = poly_count(args.a.nv, p, args.a.kmax);
    const int n2 = poly_count(args.b.nv, p, args.b.kmax);
    Poly<K> P, Q;
    load_poly<K, false>(args.a.xy, p, args.a.kmax, args.a.vec4, n1, P);
    load_poly<K, false>(args.b.xy, p, args.b.kmax, args.b.vec4, n2, Q);
    float epx[K], epy[K], eqx[K], eqy[K];
    const float E = edges<K>(P, n1, Q, n2, epx, epy, eqx, eqy);
    uint32_t spr[K], sqr[K];
    const bool exact = sign_rows<K, BLOCK>(P, n1, Q, n2, epx, epy, eqx, eqy, E, s_q + tid, spr, sqr);
    // crossings: rows i and i+1 of spr differ at j, bits j and j+1 of sqr[i] differ
    const uint32_t jmask = (1u << n2) - 1u;
    uint32_t xrow[K], erow[K];
    uint64_t xm = 0ull, sm = 0ull;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int inx = next_idx<K, false>(i, n1);
      const uint32_t r = sqr[i];
      const uint32_t rn = (r >> 1) | ((r & 1u) << (n2 - 1));
      xrow[i] = i < n1 ? (spr[i] ^ spr[inx]) & (r ^ rn) & jmask : 0u;
      erow[i] = xrow[i] & ~spr[i];  // P_i right of Q's edge j: the edge enters Q
      xm |= (uint64_t)xrow[i] << (8 * i);
      sm |= (uint64_t)erow[i] << (8 * i);
    }
    const uint32_t inside = vertex0_inclusion<K>(P, n1, Q, n2, spr, sqr);
    float B[K], L[K], W1[K], W2[K], Bq[K], M[K], V1[K], V2[K];
    crossing_sums<K, false, BLOCK>(P, n1, Q, n2, epx, epy, xrow, erow, exact, s_q + tid,
                                   s_acc + tid, B, L, W1, W2, Bq, M, V1, V2);
    float ep[K], eq[K], cp[K], cq[K];
    vertex_inclusion<K>(inside, xrow, ep, eq);
    edge_cross<K>(P, n1, Q, n2, cp, cq);
    float inter = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // inside fractions: the integer part (inclusion and base) plus the terms
      inter = fmaf(cp[k], (ep[k] + B[k]) + L[k], inter);
      inter = fmaf(cq[k], (eq[k] + Bq[k]) + M[k], inter);
      a1 += cp[k];
      a2 += cq[k];
    }
    inter *= 0.5f;
    a1 *= 0.5f;
    a2 *= 0.5f;
    const float u = a1 + a2 - inter;
    args.iou[p] = (inter > 0.f && u > 0.f) ? inter * fast_rcp(u) : 0.f;
    if (args.xmask) {
      args.xmask[p] = xm;
      args.smask[p] = sm;
      args.inside[p] = (uint8_t)inside;
    }
  }
}

template <int K>
__global__ __launch_bounds__(simple_block<K>())
__attribute__((amdgpu_waves_per_eu(simple_waves<K>()))) void k_simple_bwd(SimpleBwdArgs args) {
  constexpr int BLOCK = simple_block<K>();
  __shared__ float2 s_q[K * BLOCK];
  __shared__ float4 s_acc[K * BLOCK];
  const int tid = threadIdx.x;
  const int64_t n = args.a.count;
  for (int64_t p = (int64_t)blockIdx.x * BLOCK + tid; p < n; p += (int64_t)gridDim.x * BLOCK) {
    const int n1 = poly_count(args.a.nv, p, args.a.kmax);
    const int n2 = poly_count(args.b.nv, p, args.b.kmax);
    Poly<K> P, Q;
    load_poly<K, false>(args.a.xy, p, args.a.kmax, args.a.vec4, n1, P);
    load_poly<K, false>(args.b.xy, p, args.b.kmax, args.b.vec4, n2, Q);
    float epx[K], epy[K], eqx[K], eqy[K];
    (void)edges<K>(P, n1, Q, n2, epx, epy, eqx, eqy);
    const uint64_t xm = args.xmask[p], sm = args.smask[p];
    const uint32_t inside = args.inside[p];
    // only the bits of real edge pairs are read, so that a mask that does not
    // fit the pair (invalid saved state) still addresses this lane's slots
    const uint32_t jmask = (1u << n2) - 1u;
    uint32_t xrow[K], erow[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      xrow[i] = i < n1 ? (uint32_t)(xm >> (8 * i)) & jmask : 0u;
      erow[i] = (uint32_t)(sm >> (8 * i)) & jmask;
    }
    float B[K], L[K], W1[K], W2[K], Bq[K], M[K], V1[K], V2[K];
    crossing_sums<K, true, BLOCK>(P, n1, Q, n2, epx, epy, xrow, erow, false, s_q + tid, s_acc + tid,
                                  B, L, W1, W2, Bq, M, V1, V2);
    float ep[K], eq[K], cp[K], cq[K];
    vertex_inclusion<K>(inside, xrow, ep, eq);
    edge_cross<K>(P, n1, Q, n2, cp, cq);
    float inter = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      inter = fmaf(cp[k], (ep[k] + B[k]) + L[k], inter);
      inter = fmaf(cq[k], (eq[k] + Bq[k]) + M[k], inter);
      a1 += cp[k];
      a2 += cq[k];
    }
    inter *= 0.5f;
    a1 *= 0.5f;
    a2 *= 0.5f;
    const float u = a1 + a2 - inter;
    // IoU = I / U: d IoU = (A1 + A2) / U^2 dI - I / U^2 (dA1 + dA2)
    const bool live = inter > 0.f && u > 0.f;
    const float ru = live ? fast_rcp(u) : 0.f;
    const float g = args.grad[p];
    const float cI = g * (a1 + a2) * ru * ru, cA = -g * inter * ru * ru;
    // inside-part weights of each edge: W1 = int (1 - t), W2 = int t over
    // the inside part, each half the integer part plus its terms (the same
    // for Q's edges: V1, V2)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      W1[k] = fmaf(0.5f, ep[k] + B[k], W1[k]);
      W2[k] = fmaf(0.5f, ep[k] + B[k], W2[k]);
      V1[k] = fmaf(0.5f, eq[k] + Bq[k], V1[k]);
      V2[k] = fmaf(0.5f, eq[k] + Bq[k], V2[k]);
    }
    float* oa = args.ga_xy + p * (int64_t)args.a.kmax * 2;
    float* ob = args.gb_xy + p * (int64_t)args.b.kmax * 2;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // the edge arriving at vertex k and the vertex before k
      const int kp = k == 0 ? n1 - 1 : k - 1;
      float w2p = W2[0], npx = epy[0], npy = -epx[0];
      float ppx = P.x[0], ppy = P.y[0];
#pragma unroll
      for (int t = 1; t < K; ++t) {
        w2p = t == kp ? W2[t] : w2p;
        npx = t == kp ? epy[t] : npx;
        npy = t == kp ? -epx[t] : npy;
        ppx = t == kp ? P.x[t] : ppx;
        ppy = t == kp ? P.y[t] : ppy;
      }
      const float pnx = next_of<K, false>(P.x, k, n1), pny = next_of<K, false>(P.y, k, n1);
      const float gx = cI * (epy[k] * W1[k] + npx * w2p) + cA * 0.5f * (pny - ppy);
      const float gy = cI * (-epx[k] * W1[k] + npy * w2p) + cA * 0.5f * (ppx - pnx);
      if (k < args.a.kmax)
        *reinterpret_cast<float2*>(oa + 2 * k) = k < n1 ? make_float2(gx, gy) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int kp = k == 0 ? n2 - 1 : k - 1;
      float v2p = V2[0], npx = eqy[0], npy = -eqx[0];
      float ppx = Q.x[0], ppy = Q.y[0];
#pragma unroll
      for (int t = 1; t < K; ++t) {
        v2p = t == kp ? V2[t] : v2p;
        npx = t == kp ? eqy[t] : npx;
        npy = t == kp ? -eqx[t] : npy;
        ppx = t == kp ? Q.x[t] : ppx;
        ppy = t == kp ? Q.y[t] : ppy;
      }
      const float qnx = next_of<K, false>(Q.x, k, n2), qny = next_of<K, false>(Q.y, k, n2);
      const float gx = cI * (eqy[k] * V1[k] + npx * v2p) + cA * 0.5f * (qny - ppy);
      const float gy = cI * (-eqx[k] * V1[k] + npy * v2p) + cA * 0.5f * (ppx - qnx);
      if (k < args.b.kmax)
        *reinterpret_cast<float2*>(ob + 2 * k) = k < n2 ? make_float2(gx, gy) : make_float2(0.f, 0.f);
    }
  }
}

int64_t grid_for(int64_t n, int block) {
  int64_t blocks = (n + block - 1) / block;
  const int64_t cap = 1 << 20;
  return blocks < 1 ? 1 : (blocks > cap ? cap : blocks);
}

}  // namespace

hipError_t launch_simple_fwd(const SimpleFwdArgs& args, int K, hipStream_t stream) {
  if (K == 4)
    hipLaunchKernelGGL(k_simple_fwd<4>, dim3((unsigned)grid_for(args.a.count, simple_block<4>())),
                       dim3(simple_block<4>()), 0, stream, args);
  else
    hipLaunchKernelGGL(k_simple_fwd<8>, dim3((unsigned)grid_for(args.a.count, simple_block<8>())),
                       dim3(simple_block<8>()), 0, stream, args);
  return hipGetLastError();
}

hipError_t launch_simple_bwd(const SimpleBwdArgs& args, int K, hipStream_t stream) {
  if (K == 4)
    hipLaunchKernelGGL(k_simple_bwd<4>, dim3((unsigned)grid_for(args.a.count, simple_block<4>())),
                       dim3(simple_block<4>()), 0, stream, args);
  else
    hipLaunchKernelGGL(k_simple_bwd<8>, dim3((unsigned)grid_for(args.a.count, simple_block<8>())),
                       dim3(simple_block<8>()), 0, stream, args);
  return hipGetLastError();
}

}  // namespace dgal
