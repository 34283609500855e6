// geom.hpp -- per-pair device geometry for batched convex-polygon IoU on
// gfx950 (one wavefront lane per polygon pair).
//
// Paper: Y. Zhong, "Differentiable Computational Geometry for 2D and 3D machine
// learning", arXiv 2011.11134.  Sec. II-B: IoU = area(P n Q) / (area(P) +
// area(Q) - area(P n Q)); the forward keeps nx and one provenance flag per
// intersection vertex, and the gradient is rebuilt from them.  Sec. II-C:
// results live in fixed-capacity storage.  Sec. III: convex counter-clockwise
// polygons; lines built from two points.
//
// Forward, per pair (P with n1 vertices, Q with n2, capacity CAP = 2K):
//   1. orientation of every vertex against every edge line of the other
//      polygon, in fp32 from the original coordinates, each sign certified by
//      a static error bound; a lane with any uncertain sign recomputes all of
//      them in fp64 (exact for fp32 inputs) with the (eps, eps^2) tie rule;
//   2. inside vertices (all signs positive) and edge crossings (both edges
//      straddle each other's line) are appended, in ascending provenance code,
//      to the lane's column of an LDS buffer (dynamic slot index);
//   3. the points are ordered counter-clockwise by a pseudo-angle about their
//      centroid, measured from the first (smallest-code) point; keys carry the
//      slot index in their low bits, so a min/max network sorts plain words
//      and the points are gathered back from LDS by slot;
//   4. shoelace areas in a frame centred on P's first vertex, then IoU.
// Backward, per pair: the intersection vertices are rebuilt from the codes
// (no orientation test, no sort), the shoelace gradient is routed to the
// polygon vertices by code, crossings through the chain rule of the
// two-line meeting point.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgal {

constexpr uint32_t kCodeQ = 0x10u;
constexpr uint32_t kCodeX = 0x40u;

// 16 * 2^-24: a sign of an fp32 orientation value whose magnitude exceeds
// kCertify * E * D (E: largest edge component, D: largest coordinate spread of
// the pair) is exact.  Derivation: the two differences and two products each
// carry relative error 2^-24, the final (possibly fused) subtraction one more,
// so |error| <= 4 * 2^-24 * (|ex*dy| + |ey*dx|) <= 8 * 2^-24 * E * D; the
// factor 2 on top covers the rounding of E and D themselves.
constexpr float kCertify = 16.0f * 5.9604644775390625e-08f;

template <int K>
struct Poly {
  float x[K], y[K];
};

__device__ __forceinline__ float fast_rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// Vertex count of polygon i, clamped to [3, kmax] so that invalid counts can
// never index outside the K register / LDS slots (their results are
// unspecified, their memory accesses stay in bounds).
__device__ __forceinline__ int poly_count(const uint8_t* nv, int64_t i, int kmax) {
  const int n = nv ? (int)nv[i] : kmax;
  return min(max(n, 3), kmax);
}

// Loads polygon i of a [count][kmax][2] array into K register slots.  Slots at
// or past n hold a copy of vertex 0, so every later computation on them stays
// finite (their results are masked out).
template <int K, bool FIXED>
__device__ __forceinline__ void load_poly(const float* __restrict__ xy, int64_t i, int kmax,
                                          bool vec4, int n, Poly<K>& p) {
  const float* base = xy + i * (int64_t)kmax * 2;
  if (vec4) {  // kmax == K, 16-byte aligned rows
#pragma unroll
    for (int k = 0; k < K; k += 2) {
      float4 v = *reinterpret_cast<const float4*>(base + 2 * k);
      p.x[k] = v.x;
      p.y[k] = v.y;
      p.x[k + 1] = v.z;
      p.y[k + 1] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < kmax) {
        float2 v = *reinterpret_cast<const float2*>(base + 2 * k);
        p.x[k] = v.x;
        p.y[k] = v.y;
      } else {
        p.x[k] = 0.f;
        p.y[k] = 0.f;
      }
    }
  }
  if (!FIXED) {
#pragma unroll
    for (int k = 1; k < K; ++k) {
      p.x[k] = k < n ? p.x[k] : p.x[0];
      p.y[k] = k < n ? p.y[k] : p.y[0];
    }
  }
}

// Next vertex index after static k on a polygon of n vertices.
template <int K, bool FIXED>
__device__ __forceinline__ int next_idx(int k, int n) {
  if (FIXED) return (k + 1) % K;
  return (k + 1 < n) ? k + 1 : 0;
}

template <int K, bool FIXED>
__device__ __forceinline__ float next_of(const float (&v)[K], int k, int n) {
  if (FIXED) return v[(k + 1) % K];
  return (k + 1 < n) ? v[(k + 1) % K] : v[0];
}

// orient(a, b, c) = (b - a) x (c - a) in fp64, in the order of its definition
// and without contraction.  For fp32 inputs every difference is exact (the
// operands' exponents differ by at most 28 for any pair that is not already
// decided by fp32), each product of two differences is exact, and the single
// rounding of the final subtraction keeps the sign, including exact zeros.
__device__ __forceinline__ double orient64(float ax, float ay, float bx, float by, float cx,
                                           float cy) {
#pragma clang fp contract(off)
  double ux = (double)bx - (double)ax, uy = (double)by - (double)ay;
  double vx = (double)cx - (double)ax, vy = (double)cy - (double)ay;
  return ux * vy - uy * vx;
}

// Pseudo-angle of (dx, dy) in [0, 4): monotone in the polar angle in [0, 2pi)
// (one reciprocal instead of an arctangent).
__device__ __forceinline__ float pseudo_angle(float dx, float dy) {
  float ax = fabsf(dx), ay = fabsf(dy);
  float den = ax + ay;
  float r = den > 0.f ? dy * fast_rcp(den) : 0.f;
  return dx >= 0.f ? (dy >= 0.f ? r : 4.f + r) : 2.f - r;
}

// Sorting networks (Batcher odd-even merge) on positions 1..7 and 1..15 of
// the key array; position 0 always holds the smallest-code vertex.
#define DGAL_NET7(X)                                                                       \
  X(0, 1) X(2, 3) X(4, 5) X(0, 2) X(1, 3) X(4, 6) X(1, 2) X(5, 6) X(0, 4) X(1, 5) X(2, 6) \
  X(2, 4) X(3, 5) X(1, 2) X(3, 4) X(5, 6)
#define DGAL_NET15(X)                                                                      \
  X(0, 1) X(2, 3) X(4, 5) X(6, 7) X(8, 9) X(10, 11) X(12, 13) X(0, 2) X(1, 3) X(4, 6)     \
  X(5, 7) X(8, 10) X(9, 11) X(12, 14) X(1, 2) X(5, 6) X(9, 10) X(13, 14) X(0, 4) X(1, 5)  \
  X(2, 6) X(3, 7) X(8, 12) X(9, 13) X(10, 14) X(2, 4) X(3, 5) X(10, 12) X(11, 13) X(1, 2) \
  X(3, 4) X(5, 6) X(9, 10) X(11, 12) X(13, 14) X(0, 8) X(1, 9) X(2, 10) X(3, 11) X(4, 12) \
  X(5, 13) X(6, 14) X(4, 8) X(5, 9) X(6, 10) X(7, 11) X(2, 4) X(3, 5) X(6, 8) X(7, 9)     \
  X(10, 12) X(11, 13) X(1, 2) X(3, 4) X(5, 6) X(7, 8) X(9, 10) X(11, 12) X(13, 14)

template <int CAP>
__device__ __forceinline__ void sort_keys(uint32_t (&key)[CAP]) {
#define DGAL_CSWAP(A, B)                        \
  {                                             \
    uint32_t lo = min(key[1 + A], key[1 + B]);  \
    uint32_t hi = max(key[1 + A], key[1 + B]);  \
    key[1 + A] = lo;                            \
    key[1 + B] = hi;                            \
  }
  if constexpr (CAP == 8) {
    DGAL_NET7(DGAL_CSWAP)
  } else {
    static_assert(CAP == 16, "capacity 8 or 16");
    DGAL_NET15(DGAL_CSWAP)
  }
#undef DGAL_CSWAP
}

// Result of one pair's forward.
template <int K>
struct PairResult {
  float inter, a1, a2;  // areas (intersection, P, Q)
  int m;                // intersection vertex count (clamped to 2K)
  bool overflow;        // more than 2K vertices (invalid input)
  uint32_t codes[K / 2];  // 2K provenance codes, 4 per word, 0xFF padded
};

// Forward of one pair.  s_pt / s_cd address this lane's column of a
// [2K][BLOCK] LDS buffer (element stride BLOCK).
template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ void pair_forward(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                             float2* __restrict__ s_pt,
                                             uint8_t* __restrict__ s_cd, PairResult<K>& res) {
  constexpr int CAP = 2 * K;
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  // ---- edges and the certification scale -------------------------------
  float epx[K], epy[K], eqx[K], eqy[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    epx[k] = next_of<K, FIXED>(P.x, k, n1) - P.x[k];
    epy[k] = next_of<K, FIXED>(P.y, k, n1) - P.y[k];
    eqx[k] = next_of<K, FIXED>(Q.x, k, n2) - Q.x[k];
    eqy[k] = next_of<K, FIXED>(Q.y, k, n2) - Q.y[k];
  }
  // padded slots repeat vertex 0, so their edges are zero or real edges and
  // every min/max below may include them without widening the bound
  float E = 0.f;
  float xmin = P.x[0], xmax = P.x[0], ymin = P.y[0], ymax = P.y[0];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    E = fmaxf(E, fmaxf(fmaxf(fabsf(epx[k]), fabsf(epy[k])), fmaxf(fabsf(eqx[k]), fabsf(eqy[k]))));
    xmin = fminf(xmin, fminf(P.x[k], Q.x[k]));
    xmax = fmaxf(xmax, fmaxf(P.x[k], Q.x[k]));
    ymin = fminf(ymin, fminf(P.y[k], Q.y[k]));
    ymax = fmaxf(ymax, fmaxf(P.y[k], Q.y[k]));
  }
  const float eb = kCertify * E * fmaxf(xmax - xmin, ymax - ymin);

  // ---- 1. orientation table --------------------------------------------
  // sp bit i*K+j: P_i strictly left of Q edge j; sq bit j*K+i: Q_j strictly
  // left of P edge i.  oP[i][j] = orient(Q_j, Q_j+1, P_i).
  using Mask = typename std::conditional<(K * K > 32), uint64_t, uint32_t>::type;
  Mask sp = 0, sq = 0;
  float oP[K][K];
  bool certain = true;
#pragma unroll
  for (int i = 0; i < K; ++i) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const float dx = P.x[i] - Q.x[j], dy = P.y[i] - Q.y[j];
      const float op = eqx[j] * dy - eqy[j] * dx;
      const float oq = epy[i] * dx - epx[i] * dy;
      oP[i][j] = op;
      const bool valid = FIXED || (i < n1 && j < n2);
      certain &= !valid || (fabsf(op) > eb && fabsf(oq) > eb);
      sp |= (Mask)(op > 0.f) << (i * K + j);
      sq |= (Mask)(oq > 0.f) << (j * K + i);
    }
  }
  if (!certain) {
    // exact signs in fp64; exact zeros take the sign of Q moved by (eps, eps^2)
    sp = 0;
    sq = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const float pnx = next_of<K, FIXED>(P.x, i, n1), pny = next_of<K, FIXED>(P.y, i, n1);
      // orient(P_i, P_i1, Q_j + d) = o - e.y*eps + e.x*eps^2
      const bool tie_p = (P.y[i] != pny) ? (P.y[i] > pny) : (pnx > P.x[i]);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float qnx = next_of<K, FIXED>(Q.x, j, n2), qny = next_of<K, FIXED>(Q.y, j, n2);
        // orient(Q_j + d, Q_j1 + d, P_i) = o + f.y*eps - f.x*eps^2
        const bool tie_q = (qny != Q.y[j]) ? (qny > Q.y[j]) : (Q.x[j] > qnx);
        const double op = orient64(Q.x[j], Q.y[j], qnx, qny, P.x[i], P.y[i]);
        const double oq = orient64(P.x[i], P.y[i], pnx, pny, Q.x[j], Q.y[j]);
        const bool bp = op > 0.0 || (op == 0.0 && tie_q);
        const bool bq = oq > 0.0 || (oq == 0.0 && tie_p);
        oP[i][j] = (float)op;
        sp |= (Mask)bp << (i * K + j);
        sq |= (Mask)bq << (j * K + i);
      }
    }
  }

  // ---- 2. inside vertices and crossings, in ascending code -------------
  const uint32_t row_mask = FIXED ? ((1u << K) - 1u) : ((1u << n2) - 1u);
  const uint32_t col_mask = FIXED ? ((1u << K) - 1u) : ((1u << n1) - 1u);
  uint32_t rowd[K], cold[K];  // straddle bits per edge
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t r = (uint32_t)(sp >> (i * K)) & ((1u << K) - 1u);
    const uint32_t rn = (uint32_t)(sp >> (next_idx<K, FIXED>(i, n1) * K)) & ((1u << K) - 1u);
    rowd[i] = r ^ rn;
    const uint32_t c = (uint32_t)(sq >> (i * K)) & ((1u << K) - 1u);
    const uint32_t cn = (uint32_t)(sq >> (next_idx<K, FIXED>(i, n2) * K)) & ((1u << K) - 1u);
    cold[i] = c ^ cn;
  }
  const float ox = P.x[0], oy = P.y[0];  // local frame origin
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t r = (uint32_t)(sp >> (i * K)) & row_mask;
    const bool in = (FIXED || i < n1) && r == row_mask;
    if (in && cnt < CAP) {
      s_pt[cnt * BLOCK] = make_float2(P.x[i] - ox, P.y[i] - oy);
      s_cd[cnt * BLOCK] = (uint8_t)i;
    }
    cnt += in;
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t c = (uint32_t)(sq >> (j * K)) & col_mask;
    const bool in = (FIXED || j < n2) && c == col_mask;
    if (in && cnt < CAP) {
      s_pt[cnt * BLOCK] = make_float2(Q.x[j] - ox, Q.y[j] - oy);
      s_cd[cnt * BLOCK] = (uint8_t)(kCodeQ | j);
    }
    cnt += in;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const bool x = (FIXED || (i < n1 && j < n2)) && ((rowd[i] >> j) & (cold[j] >> i) & 1u);
      if (x) {
        // P edge i meets Q edge j at P_i + t e_i, t = o_i / (o_i - o_i1)
        const float o0 = oP[i][j];
        const float o1 = (FIXED || i + 1 < n1) ? oP[(i + 1) % K][j] : oP[0][j];
        const float den = o0 - o1;
        const float t = den != 0.f ? o0 * fast_rcp(den) : 0.f;
        if (cnt < CAP) {
          s_pt[cnt * BLOCK] = make_float2(fmaf(t, epx[i], P.x[i] - ox), fmaf(t, epy[i], P.y[i] - oy));
          s_cd[cnt * BLOCK] = (uint8_t)(kCodeX | (i << 3) | j);
        }
        ++cnt;
      }
    }
  }
  res.overflow = cnt > CAP;
  const int m = min(cnt, CAP);
  res.m = m;

  // ---- 3. counter-clockwise order --------------------------------------
  float x[CAP], y[CAP];
  float cx = 0.f, cy = 0.f;
#pragma unroll
  for (int k = 0; k < CAP; ++k) {
    float2 v = make_float2(0.f, 0.f);
    if (k < m) v = s_pt[k * BLOCK];
    x[k] = v.x;
    y[k] = v.y;
    cx += v.x;
    cy += v.y;
  }
  const float inv_m = m > 0 ? fast_rcp((float)m) : 0.f;
  cx *= inv_m;
  cy *= inv_m;
  uint32_t key[CAP];
  const float a0 = pseudo_angle(x[0] - cx, y[0] - cy);
  key[0] = 0u;
#pragma unroll
  for (int k = 1; k < CAP; ++k) {
    float r = pseudo_angle(x[k] - cx, y[k] - cy) - a0;
    r = r < 0.f ? r + 4.f : r;
    // r >= 0 or -0: clearing the sign bit makes the word order the float order
    const uint32_t kb = k < m ? (__float_as_uint(r) & 0x7fffffffu) : 0x7f000000u;
    key[k] = (kb & ~(uint32_t)(CAP - 1)) | (uint32_t)k;
  }
  sort_keys<CAP>(key);

  // ---- 4. shoelace about the first vertex ------------------------------
  float acc = 0.f;
  float px_prev = 0.f, py_prev = 0.f;
  uint32_t codes[K / 2];
#pragma unroll
  for (int w = 0; w < K / 2; ++w) codes[w] = 0xffffffffu;
  if (m > 0) codes[0] = 0xffffff00u | (uint32_t)s_cd[0];
#pragma unroll
  for (int r = 1; r < CAP; ++r) {
    if (r < m) {
      const int slot = (int)(key[r] & (uint32_t)(CAP - 1));
      const float2 v = s_pt[slot * BLOCK];
      const float vx = v.x - x[0], vy = v.y - y[0];
      if (r >= 2) acc += px_prev * vy - py_prev * vx;
      px_prev = vx;
      py_prev = vy;
      const uint32_t c = s_cd[slot * BLOCK];
      const int sh = (r & 3) * 8;
      codes[r >> 2] = (codes[r >> 2] & ~(0xffu << sh)) | (c << sh);
    }
  }
  res.inter = m >= 3 ? 0.5f * acc : 0.f;
#pragma unroll
  for (int w = 0; w < K / 2; ++w) res.codes[w] = codes[w];

  // polygon areas in the same frame (P_0 at the origin)
  float s1 = 0.f, s2 = 0.f;
  const float qx0 = Q.x[0] - ox, qy0 = Q.y[0] - oy;
#pragma unroll
  for (int k = 1; k + 1 < K; ++k) {
    if (FIXED || k + 1 < n1) {
      s1 += (P.x[k] - ox) * (P.y[k + 1] - oy) - (P.y[k] - oy) * (P.x[k + 1] - ox);
    }
    if (FIXED || k + 1 < n2) {
      const float ux = Q.x[k] - ox - qx0, uy = Q.y[k] - oy - qy0;
      const float vx = Q.x[k + 1] - ox - qx0, vy = Q.y[k + 1] - oy - qy0;
      s2 += ux * vy - uy * vx;
    }
  }
  res.a1 = 0.5f * s1;
  res.a2 = 0.5f * s2;
}

// IoU from the areas (2D), with the conventions: empty intersection or a
// non-positive union gives 0.
__device__ __forceinline__ float iou_2d(float inter, float a1, float a2, int m) {
  const float u = a1 + a2 - inter;
  return (m > 0 && u > 0.f) ? inter / u : 0.f;
}

// 3D IoU: BEV intersection times z-overlap over the union volume.
__device__ __forceinline__ float iou_3d(float inter, float a1, float a2, int m, float lo1,
                                        float hi1, float lo2, float hi2) {
  const float hz = fmaxf(0.f, fminf(hi1, hi2) - fmaxf(lo1, lo2));
  const float v = inter * hz;
  const float u = a1 * (hi1 - lo1) + a2 * (hi2 - lo2) - v;
  return (m > 0 && u > 0.f) ? v / u : 0.f;
}

// ---------------------------------------------------------------------------
// Backward of one pair from its saved count and codes.
//   s_v: lane column of a [2K][BLOCK] float2 LDS buffer (local vertices)
//   s_g: lane column of a [2K][BLOCK] float2 LDS buffer (gradient accumulators)
// Writes gP[k], gQ[k] for k < K (zero for padded slots) and, in 3D, the
// derivatives with respect to (zlo, zhi) of each polygon.
template <int K, bool FIXED, bool Z3, int BLOCK>
__device__ __forceinline__ void pair_backward(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                              float g, int nx, const uint32_t (&codes)[K / 2],
                                              float lo1, float hi1, float lo2, float hi2,
                                              float2* __restrict__ s_v, float2* __restrict__ s_g,
                                              float2 (&gP)[K], float2 (&gQ)[K], float2& gz1,
                                              float2& gz2) {
  constexpr int CAP = 2 * K;
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  const float ox = P.x[0], oy = P.y[0];
  float lpx[K], lpy[K], lqx[K], lqy[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    lpx[k] = P.x[k] - ox;
    lpy[k] = P.y[k] - oy;
    lqx[k] = Q.x[k] - ox;
    lqy[k] = Q.y[k] - oy;
    s_v[k * BLOCK] = make_float2(lpx[k], lpy[k]);
    s_v[(K + k) * BLOCK] = make_float2(lqx[k], lqy[k]);
  }
  // polygon areas (about vertex 0 of each)
  float s1 = 0.f, s2 = 0.f;
#pragma unroll
  for (int k = 1; k + 1 < K; ++k) {
    if (FIXED || k + 1 < n1) s1 += lpx[k] * lpy[k + 1] - lpy[k] * lpx[k + 1];
    if (FIXED || k + 1 < n2)
      s2 += (lqx[k] - lqx[0]) * (lqy[k + 1] - lqy[0]) - (lqy[k] - lqy[0]) * (lqx[k + 1] - lqx[0]);
  }
  const float a1 = 0.5f * s1, a2 = 0.5f * s2;

  // rebuild the intersection from the codes
  const int m = min(nx, CAP);
  float X[CAP], Y[CAP];
  uint32_t cd[CAP];
#pragma unroll
  for (int r = 0; r < CAP; ++r) {
    cd[r] = (codes[r >> 2] >> ((r & 3) * 8)) & 0xffu;
    float vx = 0.f, vy = 0.f;
    if (r < m) {
      const uint32_t c = cd[r];
      if (c < kCodeQ) {
        const float2 v = s_v[(c & (K - 1)) * BLOCK];
        vx = v.x;
        vy = v.y;
      } else if (c < kCodeX) {
        const float2 v = s_v[(K + (c & (K - 1))) * BLOCK];
        vx = v.x;
        vy = v.y;
      } else {
        const int i = (c >> 3) & (K - 1), j = c & (K - 1);
        const int i1 = (i + 1 < n1) ? i + 1 : 0, j1 = (j + 1 < n2) ? j + 1 : 0;
        const float2 a = s_v[i * BLOCK], b = s_v[i1 * BLOCK];
        const float2 cc = s_v[(K + j) * BLOCK], d = s_v[(K + j1) * BLOCK];
        const float ex = b.x - a.x, ey = b.y - a.y, fx = d.x - cc.x, fy = d.y - cc.y;
        const float wx = cc.x - a.x, wy = cc.y - a.y;
        const float den = ex * fy - ey * fx;
        const float t = den != 0.f ? (wx * fy - wy * fx) / den : 0.f;
        vx = fmaf(t, ex, a.x);
        vy = fmaf(t, ey, a.y);
      }
    }
    X[r] = vx;
    Y[r] = vy;
  }
  float acc = 0.f;
#pragma unroll
  for (int r = 1; r + 1 < CAP; ++r) {
    if (r + 1 < m) acc += (X[r] - X[0]) * (Y[r + 1] - Y[0]) - (Y[r] - Y[0]) * (X[r + 1] - X[0]);
  }
  const float inter = m >= 3 ? 0.5f * acc : 0.f;

  // scalar factors (zero where the IoU is constant: empty, non-positive union)
  float gI = 0.f, gA1 = 0.f, gA2 = 0.f;
  gz1 = make_float2(0.f, 0.f);
  gz2 = make_float2(0.f, 0.f);
  if (!Z3) {
    const float u = a1 + a2 - inter;
    if (m >= 3 && u > 0.f) {
      const float iu2 = 1.f / (u * u);
      gI = g * (a1 + a2) * iu2;
      gA1 = -g * inter * iu2;
      gA2 = gA1;
    }
  } else {
    const float h1 = hi1 - lo1, h2 = hi2 - lo2;
    const float hz = fminf(hi1, hi2) - fmaxf(lo1, lo2);
    const float v = inter * hz, v1 = a1 * h1, v2 = a2 * h2, u = v1 + v2 - v;
    if (m >= 3 && hz > 0.f && u > 0.f) {
      const float iu2 = 1.f / (u * u);
      const float gV = g * (v1 + v2) * iu2;
      const float gV1 = -g * v * iu2;
      gI = gV * hz;
      const float ghz = gV * inter;
      gA1 = gV1 * h1;
      gA2 = gV1 * h2;
      const float gh1 = gV1 * a1, gh2 = gV1 * a2;
      gz1 = make_float2(-gh1, gh1);
      gz2 = make_float2(-gh2, gh2);
      if (hi1 <= hi2) gz1.y += ghz; else gz2.y += ghz;
      if (lo1 >= lo2) gz1.x -= ghz; else gz2.x -= ghz;
    }
  }

  // accumulators start with the polygon-area terms dA/dv = 0.5 (y+ - y-, x- - x+)
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool v1 = FIXED || k < n1, v2 = FIXED || k < n2;
    const int kn1 = next_idx<K, FIXED>(k, n1), kp1 = FIXED ? (k + K - 1) % K : (k == 0 ? n1 - 1 : k - 1);
    const int kn2 = next_idx<K, FIXED>(k, n2), kp2 = FIXED ? (k + K - 1) % K : (k == 0 ? n2 - 1 : k - 1);
    float2 gp = make_float2(0.f, 0.f), gq = make_float2(0.f, 0.f);
    if (v1) {
      const float2 pn = s_v[kn1 * BLOCK], pp = s_v[kp1 * BLOCK];
      gp = make_float2(0.5f * gA1 * (pn.y - pp.y), 0.5f * gA1 * (pp.x - pn.x));
    }
    if (v2) {
      const float2 qn = s_v[(K + kn2) * BLOCK], qp = s_v[(K + kp2) * BLOCK];
      gq = make_float2(0.5f * gA2 * (qn.y - qp.y), 0.5f * gA2 * (qp.x - qn.x));
    }
    s_g[k * BLOCK] = gp;
    s_g[(K + k) * BLOCK] = gq;
  }

  // shoelace gradient of the intersection, edge by edge: the term
  // cross(X_r, X_r+1) gives (y_r+1, -x_r+1) to X_r and (-y_r, x_r) to X_r+1
  float GX[CAP], GY[CAP];
#pragma unroll
  for (int r = 0; r < CAP; ++r) {
    GX[r] = 0.f;
    GY[r] = 0.f;
  }
#pragma unroll
  for (int r = 0; r < CAP; ++r) {
    if (r < m) {
      const bool wrap = (r + 1 >= m);
      const float xn = wrap ? X[0] : X[(r + 1) % CAP];
      const float yn = wrap ? Y[0] : Y[(r + 1) % CAP];
      GX[r] += yn;
      GY[r] -= xn;
      if (r + 1 < CAP) {
        GX[r + 1] -= wrap ? 0.f : Y[r];
        GY[r + 1] += wrap ? 0.f : X[r];
      }
      GX[0] -= wrap ? Y[r] : 0.f;
      GY[0] += wrap ? X[r] : 0.f;
    }
  }
  const float hI = 0.5f * gI;

  // route every vertex's gradient to the polygon vertices it came from
#pragma unroll
  for (int r = 0; r < CAP; ++r) {
    if (r < m && gI != 0.f) {
      const float Gx = hI * GX[r], Gy = hI * GY[r];
      const uint32_t c = cd[r];
      if (c < kCodeX) {
        const int slot = (c < kCodeQ) ? (int)(c & (K - 1)) : K + (int)(c & (K - 1));
        float2 t = s_g[slot * BLOCK];
        t.x += Gx;
        t.y += Gy;
        s_g[slot * BLOCK] = t;
      } else {
        // X = a + t e with t = cross(w, f) / cross(e, f), e = b - a, f = d - c, w = c - a
        const int i = (c >> 3) & (K - 1), j = c & (K - 1);
        const int i1 = (i + 1 < n1) ? i + 1 : 0, j1 = (j + 1 < n2) ? j + 1 : 0;
        const float2 a = s_v[i * BLOCK], b = s_v[i1 * BLOCK];
        const float2 cc = s_v[(K + j) * BLOCK], d = s_v[(K + j1) * BLOCK];
        const float ex = b.x - a.x, ey = b.y - a.y, fx = d.x - cc.x, fy = d.y - cc.y;
        const float wx = cc.x - a.x, wy = cc.y - a.y;
        const float den = ex * fy - ey * fx;
        const float id = den != 0.f ? 1.f / den : 0.f;
        const float t = (wx * fy - wy * fx) * id;
        const float gt = Gx * ex + Gy * ey;
        const float gN = gt * id;       // d/d cross(w, f)
        const float gD = -gt * t * id;  // d/d cross(e, f)
        const float gex = t * Gx + gD * fy, gey = t * Gy - gD * fx;
        const float gfx = -gN * wy - gD * ey, gfy = gN * wx + gD * ex;
        const float gwx = gN * fy, gwy = -gN * fx;
        float2 ta = s_g[i * BLOCK];
        ta.x += Gx - gex - gwx;
        ta.y += Gy - gey - gwy;
        s_g[i * BLOCK] = ta;
        float2 tb = s_g[i1 * BLOCK];
        tb.x += gex;
        tb.y += gey;
        s_g[i1 * BLOCK] = tb;
        float2 tc = s_g[(K + j) * BLOCK];
        tc.x += gwx - gfx;
        tc.y += gwy - gfy;
        s_g[(K + j) * BLOCK] = tc;
        float2 td = s_g[(K + j1) * BLOCK];
        td.x += gfx;
        td.y += gfy;
        s_g[(K + j1) * BLOCK] = td;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    gP[k] = (FIXED || k < n1) ? s_g[k * BLOCK] : make_float2(0.f, 0.f);
    gQ[k] = (FIXED || k < n2) ? s_g[(K + k) * BLOCK] : make_float2(0.f, 0.f);
  }
}

}  // namespace dgal
