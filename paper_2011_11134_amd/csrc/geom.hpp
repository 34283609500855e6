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
//      to the lane's column of an LDS buffer (dynamic slot index), each with
//      the edge the intersection's boundary leaves it on and, per edge, the
//      slot of the next point along it;
//   3. the points are ordered counter-clockwise by walking that boundary from
//      the smallest code (two bit-field reads a step, no angles, no sort);
//      the signs are exact, so the order is the boundary of the pair moved by
//      the tie rule also where points coincide;
//   4. shoelace areas in a frame centred on P's first vertex, then IoU;
//   5. thin pairs (the largest coordinate F of the pair in that frame large
//      against the union: F^2 > kThinUnion * max(A1, A2)) take their areas
//      again in fp64 from the polygons and the (exact) codes (thin_areas64).
// Backward, per pair: the intersection vertices are rebuilt from the codes
// (no orientation test, no sort), the shoelace gradient is routed to the
// polygon vertices by code, crossings through the chain rule of the
// two-line meeting point; thin pairs (and, for elementwise pairs, tiny
// intersections: F^2 > kThinInter * I) take the whole gradient again in fp64
// (pair_backward64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace dgal {

constexpr uint32_t kCodeQ = 0x10u;
constexpr uint32_t kCodeX = 0x40u;

// 16 * 2^-24: a sign of an fp32 orientation value whose magnitude exceeds
// kCertify * E * D (E: largest edge component of the pair, D: largest
// component of the vertex differences P_i - Q_j) is exact.  Derivation: the
// two differences and two products each carry relative error 2^-24, the
// final (possibly fused) subtraction one more, so |error| <= 4 * 2^-24 *
// (|ex*dy| + |ey*dx|) <= 8 * 2^-24 * E * D; the factor 2 on top covers the
// rounding of E, D and of the bound itself.
constexpr float kCertify = 16.0f * 5.9604644775390625e-08f;

// Bounds of the fp64 rebuild.  Rounding in fp32 moves the areas by about
// u F P (u = 2^-24, F the pair's largest coordinate in the frame at P_0, P a
// perimeter, at most about 2 pi F), i.e. the IoU by about u F^2 / U.  Measured
// on thin rotated rectangles (widths 1e-3..1e-2, lengths 1..3): about 4e-8 of
// IoU error per unit of F^2 / U.  The test is taken as soon as the polygons'
// areas are known, against the lower bound max(A1, A2) of the union: lanes
// with F^2 > kThinUnion * max(A1, A2) (so every lane with F^2 / U above 32,
// 1.3e-6 of IoU error) recompute their areas in fp64.  On the benchmark
// workloads F^2 / max(A1, A2) stays below 6 (rectangles), 12 (scenes) and
// 130 (3..8-gons: 4e-4 of the pairs above the bound).
constexpr float kThinUnion = 32.f;
// A gradient's rebuilt vertices are off by about u F against an
// intersection of extent about sqrt(I): relative error about u F / sqrt(I).
// Elementwise pairs with F^2 > kThinInter * I (about 2.5e-4 at the bound with
// the constant a needle-shaped intersection measured) take the gradient in
// fp64.
constexpr float kThinInter = 1048576.f;  // 2^20

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
// finite (their results are masked out).  FIXED callers guarantee kmax == K
// and 16-byte aligned rows, so they always take the vector path.
template <int K, bool FIXED>
__device__ __forceinline__ void load_poly(const float* __restrict__ xy, int64_t i, int kmax,
                                          bool vec4, int n, Poly<K>& p) {
  const float* base = xy + i * (int64_t)kmax * 2;
  if (FIXED || vec4) {  // kmax == K, 16-byte aligned rows
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

// Result of one pair's forward.
template <int K>
struct PairResult {
  bool thin;  // the areas need the fp64 rebuild (thin_areas64)
  float inter, a1, a2;  // areas (intersection, P, Q)
  int m;                // intersection vertex count (clamped to 2K)
  bool overflow;        // more than 2K vertices (invalid input)
  bool exact;           // the signs were recomputed in fp64 (fp32 could not certify them)
  uint32_t codes[K / 2];  // 2K provenance codes, 4 per word, 0xFF padded
};

// Path statistics of a wavefront's live lanes (stats: NULL when off, else
// three device counters: pairs evaluated, pairs whose signs took the fp64
// path, pairs whose areas took the fp64 rebuild), one set of atomic adds per
// wavefront.
__device__ __forceinline__ void count_path(unsigned long long* stats, bool exact, bool thin) {
  if (stats == nullptr) return;  // uniform
  const uint64_t live = __builtin_amdgcn_ballot_w64(true);
  const uint64_t ex = __builtin_amdgcn_ballot_w64(exact);
  const uint64_t th = __builtin_amdgcn_ballot_w64(thin);
  if ((int)(__lane_id()) == __builtin_ctzll(live)) {
    atomicAdd(stats, (unsigned long long)__popcll(live));
    atomicAdd(stats + 1, (unsigned long long)__popcll(ex));
    atomicAdd(stats + 2, (unsigned long long)__popcll(th));
  }
}

// An index the compiler cannot see through, so that a reload from it is not
// merged with an earlier load (which would keep those registers live).
__device__ __forceinline__ int64_t opaque(int64_t i) {
  asm volatile("" : "+v"(i));
  return i;
}

// Waves per SIMD that the LDS of a pair_forward kernel allows at K = 8
// (144 bytes a lane against 160 KiB a CU); the register allocator is held
// to the same count (at most 128 VGPRs, met without spilling; left alone it
// takes more and halves the occupancy).  Kernels at K = 4 are left to the
// allocator.
template <int K>
constexpr int fwd_waves_per_simd() {
  return K == 8 ? 4 : 1;
}

// Forward of one pair.  s_pt / s_cd address this lane's column of
// [2K][BLOCK] LDS buffers (element stride BLOCK): a point, and its code with,
// in the high byte, the edge the intersection's boundary leaves it on.  EMIT: the ordered
// intersection vertices are also returned in ov[0..2K) (absolute frame,
// slots at and past the vertex count set to 0).
template <int K, bool FIXED, int BLOCK, bool EMIT = false>
__device__ __forceinline__ void pair_forward(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                             float2* __restrict__ s_pt,
                                             uint16_t* __restrict__ s_cd, PairResult<K>& res,
                                             float2* ov = nullptr) {
  constexpr int CAP = 2 * K;
  constexpr int NW = (K * K + 31) / 32;  // 32-bit words of a K x K sign table
  constexpr uint32_t KM = (1u << K) - 1u;
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  // ---- edges -------------------------------------------------------------
  // padded slots repeat vertex 0, so their edges are zero or real edges
  float epx[K], epy[K], eqx[K], eqy[K];
  float E = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    epx[k] = next_of<K, FIXED>(P.x, k, n1) - P.x[k];
    epy[k] = next_of<K, FIXED>(P.y, k, n1) - P.y[k];
    eqx[k] = next_of<K, FIXED>(Q.x, k, n2) - Q.x[k];
    eqy[k] = next_of<K, FIXED>(Q.y, k, n2) - Q.y[k];
    E = fmaxf(E, fmaxf(fmaxf(fabsf(epx[k]), fabsf(epy[k])), fmaxf(fabsf(eqx[k]), fabsf(eqy[k]))));
  }

  // ---- 1. orientation table --------------------------------------------
  // oP[i][j] = orient(Q_j, Q_j+1, P_i); oq(i, j) = orient(P_i, P_i+1, Q_j).
  // Their sign bits are shifted, highest table index first, into words whose
  // bit i*K+j is set when the value is negative (or -0); D is the largest
  // component of the vertex differences, omin the smallest magnitude.
  // The 4-slot kernels keep the table for the crossings; the 8-slot ones
  // (64 values) recompute the two values a crossing needs, from registers.
  constexpr bool KEEP_OP = K == 4;
  float oP[KEEP_OP ? K : 1][KEEP_OP ? K : 1];
  uint32_t negp[NW], negq[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    negp[w] = 0u;
    negq[w] = 0u;
  }
  float D = 0.f, omin = __builtin_inff();
#pragma unroll
  for (int i = K - 1; i >= 0; --i) {
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
      const float dx = P.x[i] - Q.x[j], dy = P.y[i] - Q.y[j];
      const float op = eqx[j] * dy - eqy[j] * dx;
      const float oq = epy[i] * dx - epx[i] * dy;
      if constexpr (KEEP_OP) oP[i][j] = op;
      const int w = (i * K + j) >> 5;
      negp[w] = __builtin_amdgcn_alignbit(negp[w], __float_as_uint(op), 31);
      negq[w] = __builtin_amdgcn_alignbit(negq[w], __float_as_uint(oq), 31);
      D = fmaxf(D, fmaxf(fabsf(dx), fabsf(dy)));
      const float mo = fminf(fabsf(op), fabsf(oq));
      omin = fminf(omin, (FIXED || (i < n1 && j < n2)) ? mo : __builtin_inff());
    }
  }
  const bool exact = !(omin > kCertify * E * D);
  res.exact = exact;
  if (exact) {
    // Exact signs in fp64; exact zeros take the sign of Q moved by (eps,
    // eps^2).  Rare, so it is written for few registers rather than speed:
    // Q is staged in this lane's (still unused) LDS column and each row of
    // the table is a runtime loop over Q's edges.
#pragma unroll
    for (int k = 0; k < K; ++k) s_pt[k * BLOCK] = make_float2(Q.x[k], Q.y[k]);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const float pnx = next_of<K, FIXED>(P.x, i, n1), pny = next_of<K, FIXED>(P.y, i, n1);
      // orient(P_i, P_i1, Q_j + d) = o - e.y*eps + e.x*eps^2
      const bool tie_p = (P.y[i] != pny) ? (P.y[i] > pny) : (pnx > P.x[i]);
      const int w = (i * K) >> 5, sh = (i * K) & 31;
#pragma unroll 1
      for (int j = 0; j < K; ++j) {
        const int jn = FIXED ? ((j + 1) & (K - 1)) : (j + 1 < n2 ? j + 1 : 0);
        const float2 q = s_pt[j * BLOCK], qn = s_pt[jn * BLOCK];
        // orient(Q_j + d, Q_j1 + d, P_i) = o + f.y*eps - f.x*eps^2
        const bool tie_q = (qn.y != q.y) ? (qn.y > q.y) : (q.x > qn.x);
        const double op = orient64(q.x, q.y, qn.x, qn.y, P.x[i], P.y[i]);
        const double oq = orient64(P.x[i], P.y[i], pnx, pny, q.x, q.y);
        const bool bp = op > 0.0 || (op == 0.0 && tie_q);
        const bool bq = oq > 0.0 || (oq == 0.0 && tie_p);
        // each bit is replaced in place: the fp32 words stay live on both
        // sides of the branch, so their sign chains are not sunk past it
        // (which would hold all K*K products in registers)
        const uint32_t bit = 1u << (sh + j);
        negp[w] = (negp[w] & ~bit) | (bp ? 0u : bit);
        negq[w] = (negq[w] & ~bit) | (bq ? 0u : bit);
        if constexpr (KEEP_OP) {
          const float o = (float)op;
#pragma unroll
          for (int t = 0; t < K; ++t) oP[i][t] = t == j ? o : oP[i][t];
        }
      }
    }
  }

  // ---- 2. inside vertices and crossings, in ascending code -------------
  // row i of sp: bit j set when P_i is strictly left of Q edge j; row i of
  // sq: bit j set when Q_j is strictly left of P edge i.
  const uint32_t jmask = FIXED ? KM : ((1u << n2) - 1u);
  uint32_t spr[K], sqr[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int w = (i * K) >> 5, sh = (i * K) & 31;
    spr[i] = ~(negp[w] >> sh) & KM;
    sqr[i] = ~(negq[w] >> sh) & KM;
    if (!FIXED && i >= n1) sqr[i] = KM;  // padded P edges constrain nothing
  }
  uint32_t qin = KM;  // bit j: Q_j left of every P edge
#pragma unroll
  for (int i = 0; i < K; ++i) qin &= sqr[i];

  float lpx[K], lpy[K];  // P in the frame centred on P_0
  lpx[0] = 0.f;
  lpy[0] = 0.f;
#pragma unroll
  for (int k = 1; k < K; ++k) {
    lpx[k] = P.x[k] - P.x[0];
    lpy[k] = P.y[k] - P.y[0];
  }
  // polygon areas in the same frame (P_0 at the origin), here so that the
  // polygons' registers are free once the crossings are placed
  {
    float s1 = 0.f, s2 = 0.f;
    const float qx0 = Q.x[0] - P.x[0], qy0 = Q.y[0] - P.y[0];
#pragma unroll
    for (int k = 1; k + 1 < K; ++k) {
      if (FIXED || k + 1 < n1) s1 += lpx[k] * lpy[k + 1] - lpy[k] * lpx[k + 1];
      if (FIXED || k + 1 < n2) {
        const float ux = Q.x[k] - P.x[0] - qx0, uy = Q.y[k] - P.y[0] - qy0;
        const float vx = Q.x[k + 1] - P.x[0] - qx0, vy = Q.y[k + 1] - P.y[0] - qy0;
        s2 += ux * vy - uy * vx;
      }
    }
    res.a1 = 0.5f * s1;
    res.a2 = 0.5f * s2;
  }
  // step 5's test, decided here: F, the pair's largest coordinate in this
  // frame, is bounded by max(|P_k - P_0|, D) (each Q_j - P_0 is one of the
  // differences D bounds), which is at most 2 F
  bool thin_pre;
  {
    float F = D;
#pragma unroll
    for (int k = 1; k < K; ++k) F = fmaxf(F, fmaxf(fabsf(lpx[k]), fabsf(lpy[k])));
    thin_pre = F * F > kThinUnion * fmaxf(res.a1, res.a2);
  }
  // Points go to the lane's LDS column in ascending code (slot 0 holds the
  // smallest).  For the counter-clockwise walk each point also records, in
  // the high byte of its code entry, the edge the boundary leaves it on (P
  // edge i as i, Q edge j as K + j), and each edge records, in its nibble of
  // `nexw`, the slot of the next point on it: the edge's end when that end is
  // inside the other polygon, else the crossing where the edge leaves it.
  // Every nibble is written once for valid input; any mix of slots that
  // invalid input ORs together still names a slot below CAP, so the walk
  // stays in bounds.
  using Nib = typename std::conditional<K == 4, uint32_t, uint64_t>::type;
  Nib nexw = 0;
  int cnt = 0;
  // Appends a point; only invalid input can pass the capacity, and its
  // extra points then overwrite the last slot (the overflow is reported).
  auto put = [&](bool in, float px, float py, uint32_t code, uint32_t leave, uint32_t reach) {
    const int s = min(cnt, CAP - 1);
    if (in) {
      s_pt[s * BLOCK] = make_float2(px, py);
      s_cd[s * BLOCK] = (uint16_t)(code | (leave << 8));
    }
    nexw |= in ? (Nib)s << (4 * reach) : (Nib)0;
    cnt += in;
  };
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t ip = FIXED ? (uint32_t)((i + K - 1) % K) : (uint32_t)(i == 0 ? n1 - 1 : i - 1);
    put((FIXED || i < n1) && (spr[i] & jmask) == jmask, lpx[i], lpy[i], (uint32_t)i, (uint32_t)i,
        ip);
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t jp = FIXED ? (uint32_t)((j + K - 1) % K) : (uint32_t)(j == 0 ? n2 - 1 : j - 1);
    put((FIXED || j < n2) && ((qin >> j) & 1u), Q.x[j] - P.x[0], Q.y[j] - P.y[0], kCodeQ | j,
        (uint32_t)(K + j), (uint32_t)K + jp);
  }
  // A crossing of P edge i with Q edge j where P_i is left of Q edge j's line
  // is where P edge i leaves Q (and Q edge j enters P, so the boundary goes on
  // along Q edge j); otherwise P edge i enters Q there and Q edge j leaves P.
  auto put_x = [&](bool in, float px, float py, int i, int j) {
    const bool p_leaves = (spr[i] >> j) & 1u;
    put(in, px, py, kCodeX | (uint32_t)(i << 3) | (uint32_t)j,
        p_leaves ? (uint32_t)(K + j) : (uint32_t)i, p_leaves ? (uint32_t)i : (uint32_t)(K + j));
  };
#pragma unroll
  for (int i = 0; i < K; ++i) {
    // P edge i straddles the line of Q edge j (rows i and i+1 of sp differ)
    // and Q edge j straddles the line of P edge i (bits j and j+1 of row i of
    // sq differ)
    const int inx = next_idx<K, FIXED>(i, n1);
    const uint32_t r = sqr[i];
    const uint32_t rn = FIXED ? ((r >> 1) | (r << (K - 1))) : ((r >> 1) | ((r & 1u) << (n2 - 1)));
    const uint32_t xm = (spr[i] ^ spr[inx]) & (r ^ rn) & jmask;
    // P edge i meets Q edge j at P_i + t e_i, t = o_i / (o_i - o_i1); the two
    // values have opposite signs (or one is an exact zero that the tie rule
    // signed), so the difference is never zero for coordinates whose
    // products stay normal floats.  Crossings are placed in ascending j.
    if constexpr (KEEP_OP) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if ((FIXED || i < n1) && ((xm >> j) & 1u)) {
          const float o0 = oP[i][j], o1 = oP[inx][j];
          const float t = o0 * fast_rcp(o0 - o1);
          put_x(true, fmaf(t, epx[i], lpx[i]), fmaf(t, epy[i], lpy[i]), i, j);
        }
      }
    } else {
      // Eight slots: the edge walks the set bits of its row (a convex Q is
      // crossed at most twice by an edge, so a wavefront takes at most two
      // steps) and selects Q's edge from registers.  The table's expressions
      // are recomputed from copies of P's vertex that an empty asm makes
      // opaque: otherwise the compiler keeps the K*K table values, or the
      // edge vectors and the local frame, live from the table to here
      // (certified signs survive any difference in rounding between the two
      // evaluations).
      float px = P.x[i], py = P.y[i];
      asm volatile("" : "+v"(px), "+v"(py));
      const float ex = P.x[inx] - px, ey = P.y[inx] - py;
      const float lx = px - P.x[0], ly = py - P.y[0];
      uint32_t row = (FIXED || i < n1) ? xm : 0u;
      while (row) {
        const int j = __builtin_ctz(row);
        row &= row - 1u;
        const int jn = FIXED ? ((j + 1) & (K - 1)) : (j + 1 < n2 ? j + 1 : 0);
        float qx = Q.x[0], qy = Q.y[0], qnx = Q.x[0], qny = Q.y[0];
#pragma unroll
        for (int k = 1; k < K; ++k) {
          qx = k == j ? Q.x[k] : qx;
          qy = k == j ? Q.y[k] : qy;
          qnx = k == jn ? Q.x[k] : qnx;
          qny = k == jn ? Q.y[k] : qny;
        }
        float o0, o1;
        if (!exact) {
          const float fx = qnx - qx, fy = qny - qy;
          o0 = fx * (py - qy) - fy * (px - qx);
          o1 = fx * (P.y[inx] - qy) - fy * (P.x[inx] - qx);
        } else {
          o0 = (float)orient64(qx, qy, qnx, qny, px, py);
          o1 = (float)orient64(qx, qy, qnx, qny, P.x[inx], P.y[inx]);
        }
        const float t = o0 * fast_rcp(o0 - o1);
        put_x(true, fmaf(t, ex, lx), fmaf(t, ey, ly), i, j);
      }
    }
  }
  res.overflow = cnt > CAP;
  const int m = min(cnt, CAP);
  res.m = m;

  // ---- 3 + 4. counter-clockwise walk from slot 0, shoelace about it ----
  // Each step: the edge the current point leaves on, then the slot of the
  // next point on that edge (both masked to their ranges, so that an entry
  // that was never written, read when m = 0, still names a valid slot).  The
  // signs are exact (certified, or fp64 with the tie rule), so the walk is
  // the boundary of the pair moved by the tie rule, where points that
  // coincide still have a definite order.
  const float2 v0 = s_pt[0];
  float acc = 0.f;
  float px_prev = 0.f, py_prev = 0.f;
  uint32_t codes[K / 2];
#pragma unroll
  for (int w = 0; w < K / 2; ++w) codes[w] = 0xffffffffu;
  uint32_t ent = s_cd[0];  // code | leave-edge << 8 of the current point
  if (m > 0) codes[0] = 0xffffff00u | (ent & 0xffu);
  if (EMIT) {
#pragma unroll
    for (int r = 0; r < CAP; ++r) ov[r] = make_float2(0.f, 0.f);
    if (m > 0) ov[0] = make_float2(v0.x + P.x[0], v0.y + P.y[0]);
  }
  uint32_t slot = 0;
#pragma unroll
  for (int r = 1; r < CAP; ++r) {
    if constexpr (K == 4) {
      // every step is taken (the walk only ever names this lane's slots) and
      // the ones at or past m are masked by selects, so that the rolling pair
      // needs no register copies; a dead slot may hold anything and is never
      // added in
      slot = (uint32_t)(nexw >> (4 * ((ent >> 8) & (uint32_t)(CAP - 1)))) & (uint32_t)(CAP - 1);
      ent = s_cd[slot * BLOCK];
      const bool live = r < m;
      const float2 v = s_pt[slot * BLOCK];
      const float vx = v.x - v0.x, vy = v.y - v0.y;
      if (r >= 2) {
        const float term = px_prev * vy - py_prev * vx;
        acc += live ? term : 0.f;
      }
      px_prev = vx;
      py_prev = vy;
      const uint32_t c = live ? (ent & 0xffu) : 0xffu;
      const int sh = (r & 3) * 8;
      codes[r >> 2] = (codes[r >> 2] & ~(0xffu << sh)) | (c << sh);
      if (EMIT) ov[r] = live ? make_float2(v.x + P.x[0], v.y + P.y[0]) : make_float2(0.f, 0.f);
    } else if (r < m) {
      slot = (uint32_t)(nexw >> (4 * ((ent >> 8) & (uint32_t)(CAP - 1)))) & (uint32_t)(CAP - 1);
      ent = s_cd[slot * BLOCK];
      const float2 v = s_pt[slot * BLOCK];
      const float vx = v.x - v0.x, vy = v.y - v0.y;
      if (r >= 2) acc += px_prev * vy - py_prev * vx;
      px_prev = vx;
      py_prev = vy;
      const uint32_t c = ent & 0xffu;
      const int sh = (r & 3) * 8;
      codes[r >> 2] = (codes[r >> 2] & ~(0xffu << sh)) | (c << sh);
      if (EMIT) ov[r] = make_float2(v.x + P.x[0], v.y + P.y[0]);
    }
  }
  res.inter = m >= 3 ? 0.5f * acc : 0.f;
#pragma unroll
  for (int w = 0; w < K / 2; ++w) res.codes[w] = codes[w];
  res.thin = m >= 3 && thin_pre;
}

// IoU from the areas (2D), with the conventions: empty intersection or a
// non-positive union gives 0.  The quotient uses the hardware reciprocal
// (1 ulp), well inside the IoU tolerance.
__device__ __forceinline__ float iou_2d(float inter, float a1, float a2, int m) {
  const float u = a1 + a2 - inter;
  return (m > 0 && u > 0.f) ? inter * fast_rcp(u) : 0.f;
}

// 3D IoU: BEV intersection times z-overlap over the union volume.
__device__ __forceinline__ float iou_3d(float inter, float a1, float a2, int m, float lo1,
                                        float hi1, float lo2, float hi2) {
  const float hz = fmaxf(0.f, fminf(hi1, hi2) - fmaxf(lo1, lo2));
  const float v = inter * hz;
  const float u = a1 * (hi1 - lo1) + a2 * (hi2 - lo2) - v;
  return (m > 0 && u > 0.f) ? v * fast_rcp(u) : 0.f;
}

// IoU of a pair from its areas, 2D, or 3D with z extents [lo, hi] read at
// indices ia / ib.
template <bool Z3>
__device__ __forceinline__ float pair_iou(float inter, float a1, float a2, int m,
                                          const float* zlo_a, const float* zhi_a, int64_t ia,
                                          const float* zlo_b, const float* zhi_b, int64_t ib) {
  if (Z3) return iou_3d(inter, a1, a2, m, zlo_a[ia], zhi_a[ia], zlo_b[ib], zhi_b[ib]);
  return iou_2d(inter, a1, a2, m);
}

// ---------------------------------------------------------------------------
// Backward of one pair from its saved count and codes.
//   s_v: lane column of a [2K][BLOCK] float2 LDS buffer (local vertices)
//   s_g: lane column of a [2K][BLOCK] float2 LDS buffer (gradient accumulators)
//   s_tab: the block's code table (fill_code_table)
// Writes gP[k], gQ[k] for k < K (zero for padded slots) and, in 3D, the
// derivatives with respect to (zlo, zhi) of each polygon.
//
// Every intersection vertex is handled by one code path: its code names the
// LDS slots A, B (an edge) and C, D (the other polygon's edge) with
// X = A + t (B - A), t = cross(C - A, D - C) / cross(B - A, D - C) for a
// crossing; a polygon vertex names its own slot four times, so that every
// difference and t vanish and X = A.
template <int K, bool FIXED>
__device__ __forceinline__ void code_slots(uint32_t c, int n1, int n2, int& ia, int& ib, int& ic,
                                           int& id) {
  const bool cross = c >= kCodeX;
  const int i = (int)((c >> 3) & (K - 1)), j = (int)(c & (K - 1));
  const int own = j + ((c & kCodeQ) ? K : 0);  // vertex slot of a P or Q vertex code
  const int in = FIXED ? ((i + 1) & (K - 1)) : (i + 1 < n1 ? i + 1 : 0);
  const int jn = FIXED ? ((j + 1) & (K - 1)) : (j + 1 < n2 ? j + 1 : 0);
  ia = cross ? i : own;
  ib = cross ? in : own;
  ic = cross ? K + j : own;
  id = cross ? K + jn : own;
}

// Byte offsets, within a lane's column of a [2K][BLOCK] float2 LDS buffer, of
// the slots A, B, C, D that code c names, packed as 16-bit halves:
// x = A | B << 16, y = C | D << 16.  A block fills a 256-entry table of these
// once, so the backward decodes a code with one LDS read.  On fixed-size
// polygons the edge ends wrap at K; otherwise a crossing's B and D are stored
// unwrapped (slot i + 1 and K + j + 1) and wrapped per lane.
template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ uint2 code_offsets(uint32_t c) {
  int ia, ib, ic, id;
  if (FIXED) {
    code_slots<K, true>(c, K, K, ia, ib, ic, id);
  } else {
    code_slots<K, false>(c, K + 1, K + 1, ia, ib, ic, id);  // no wrap below K + 1
  }
  constexpr uint32_t S = BLOCK * sizeof(float2);
  static_assert(2 * K * S < 65536u, "offsets fit 16 bits");
  return make_uint2((uint32_t)ia * S | ((uint32_t)ib * S) << 16,
                    (uint32_t)ic * S | ((uint32_t)id * S) << 16);
}

template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ void fill_code_table(uint2* s_tab) {
  for (int c = threadIdx.x; c < 256; c += blockDim.x)
    s_tab[c] = code_offsets<K, FIXED, BLOCK>((uint32_t)c);
}

// LDS byte offsets of the four slots of code c.  n1S = n1 * S and
// nqS = (K + n2) * S, S the slot stride in bytes, locate the wrap of a
// crossing's edge ends on polygons with fewer than K vertices; offsets are
// clamped to the lane's column, so that codes which do not fit the pair
// (invalid saved state) still address this lane's own slots.
template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ void slot_offsets(uint32_t c, uint32_t n1S, uint32_t nqS,
                                             const uint2* __restrict__ s_tab, uint32_t& oa,
                                             uint32_t& ob, uint32_t& oc, uint32_t& od) {
  const uint2 o = s_tab[c];
  oa = o.x & 0xffffu;
  ob = o.x >> 16;
  oc = o.y & 0xffffu;
  od = o.y >> 16;
  if constexpr (!FIXED) {
    constexpr uint32_t S = BLOCK * sizeof(float2);
    const bool cross = c >= kCodeX;
    ob = (cross && ob == n1S) ? 0u : min(ob, (2 * K - 1) * S);
    od = (cross && od == nqS) ? K * S : min(od, (2 * K - 1) * S);
  }
}

__device__ __forceinline__ float2& at(float2* col, uint32_t off) {
  return *reinterpret_cast<float2*>(reinterpret_cast<char*>(col) + off);
}
__device__ __forceinline__ const float2& at(const float2* col, uint32_t off) {
  return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(col) + off);
}

// Chain rule of one intersection vertex X = A + t (B - A) (see code_slots)
// for dL/dX = G, added into the slots' gradient accumulators: with
// e = B - A, f = D - C, w = C - A,
//   dL/dt = G.e, dL/dcross(w,f) = dL/dt / den, dL/dden = -dL/dt t / den,
//   A gets G - dL/de - dL/dw, B gets dL/de, C gets dL/dw - dL/df, D gets dL/df.
// t and 1/den come from the caller (0 for a polygon vertex, whose slots are
// all A: it adds G to A and zeros to the aliases, which are written first).
__device__ __forceinline__ void route_slot(float Gx, float Gy, float t, float idn, uint32_t oa,
                                           uint32_t ob, uint32_t oc, uint32_t od,
                                           float2* __restrict__ s_v, float2* __restrict__ s_g) {
  const float2 a = at(s_v, oa), b = at(s_v, ob), cc = at(s_v, oc), d = at(s_v, od);
  float2 ta = at(s_g, oa), tb = at(s_g, ob), tc = at(s_g, oc), td = at(s_g, od);
  const float ex = b.x - a.x, ey = b.y - a.y, fx = d.x - cc.x, fy = d.y - cc.y;
  const float wx = cc.x - a.x, wy = cc.y - a.y;
  const float gt = Gx * ex + Gy * ey;
  const float gN = gt * idn;  // d/d cross(w, f)
  const float gD = -gN * t;   // d/d cross(e, f)
  const float gex = t * Gx + gD * fy, gey = t * Gy - gD * fx;
  const float gfx = -gN * wy - gD * ey, gfy = gN * wx + gD * ex;
  const float gwx = gN * fy, gwy = -gN * fx;
  tb.x += gex;
  tb.y += gey;
  tc.x += gwx - gfx;
  tc.y += gwy - gfy;
  td.x += gfx;
  td.y += gfy;
  ta.x += Gx - gex - gwx;
  ta.y += Gy - gey - gwy;
  at(s_g, ob) = tb;
  at(s_g, oc) = tc;
  at(s_g, od) = td;
  at(s_g, oa) = ta;
}

// t and 1/den of the vertex in slots (oa, ob, oc, od); its position is
// A + t (B - A).
__device__ __forceinline__ float2 slot_vertex(uint32_t oa, uint32_t ob, uint32_t oc, uint32_t od,
                                              const float2* __restrict__ s_v, float& t,
                                              float& idn) {
  const float2 a = at(s_v, oa), b = at(s_v, ob), cc = at(s_v, oc), d = at(s_v, od);
  const float ex = b.x - a.x, ey = b.y - a.y, fx = d.x - cc.x, fy = d.y - cc.y;
  const float wx = cc.x - a.x, wy = cc.y - a.y;
  const float den = ex * fy - ey * fx;
  idn = den != 0.f ? fast_rcp(den) : 0.f;
  t = (wx * fy - wy * fx) * idn;
  return make_float2(fmaf(t, ex, a.x), fmaf(t, ey, a.y));
}

// The backward is one pass over the ordered vertices: vertex r + 1 is
// rebuilt while vertex r, whose shoelace gradient needs both neighbours, is
// routed; vertex 0 is routed last.  The routing is linear in the upstream
// gradient, so it accumulates the unscaled shoelace gradient and the IoU's
// factor (which needs the intersection area, known only at the end) scales
// the accumulators when they are read back.
struct SlotGeom {
  uint32_t oa, ob, oc, od;
  float t, idn;
};

template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ float2 rebuild_slot(uint32_t c, uint32_t n1S, uint32_t nqS,
                                               const uint2* __restrict__ s_tab,
                                               const float2* __restrict__ s_v, SlotGeom& sg) {
  slot_offsets<K, FIXED, BLOCK>(c, n1S, nqS, s_tab, sg.oa, sg.ob, sg.oc, sg.od);
  return slot_vertex(sg.oa, sg.ob, sg.oc, sg.od, s_v, sg.t, sg.idn);
}

// `thin` (out): the lane's gradient needs the fp64 rebuild (pair_backward64):
// thin polygons (F^2 > kThinUnion * max(A1, A2)) and, with TINY, tiny
// intersections (F^2 > kThinInter * I).
template <int K, bool FIXED, bool Z3, int BLOCK, bool TINY = false>
__device__ __forceinline__ void pair_backward(const Poly<K>& P, int n1, const Poly<K>& Q, int n2,
                                              float g, int nx, const uint32_t (&codes)[K / 2],
                                              float lo1, float hi1, float lo2, float hi2,
                                              float2* __restrict__ s_v, float2* __restrict__ s_g,
                                              const uint2* __restrict__ s_tab, float2 (&gP)[K],
                                              float2 (&gQ)[K], float2& gz1, float2& gz2,
                                              bool& thin) {
  constexpr int CAP = 2 * K;
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  const float ox = P.x[0], oy = P.y[0];
  float lpx[K], lpy[K], lqx[K], lqy[K];
  float F = 0.f;  // the pair's largest coordinate in the frame at P_0
#pragma unroll
  for (int k = 0; k < K; ++k) {
    lpx[k] = P.x[k] - ox;
    lpy[k] = P.y[k] - oy;
    lqx[k] = Q.x[k] - ox;
    lqy[k] = Q.y[k] - oy;
    F = fmaxf(fmaxf(F, fmaxf(fabsf(lpx[k]), fabsf(lpy[k]))), fmaxf(fabsf(lqx[k]), fabsf(lqy[k])));
    s_v[k * BLOCK] = make_float2(lpx[k], lpy[k]);
    s_v[(K + k) * BLOCK] = make_float2(lqx[k], lqy[k]);
    s_g[k * BLOCK] = make_float2(0.f, 0.f);
    s_g[(K + k) * BLOCK] = make_float2(0.f, 0.f);
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
  const float F2 = F * F;
  const bool thin_pre = F2 > kThinUnion * fmaxf(a1, a2);

  // ---- one pass: rebuild r + 1, route r (padding codes name valid slots;
  // vertices past nx are never used)
  const int m = min(nx, CAP);
  constexpr uint32_t S = BLOCK * sizeof(float2);
  const uint32_t n1S = (uint32_t)n1 * S, nqS = (uint32_t)(K + n2) * S;
  auto code_at = [&](int r) { return (codes[r >> 2] >> ((r & 3) * 8)) & 0xffu; };
  SlotGeom g0, gc;
  const float2 X0 = rebuild_slot<K, FIXED, BLOCK>(code_at(0), n1S, nqS, s_tab, s_v, g0);
  const float2 X1 = rebuild_slot<K, FIXED, BLOCK>(code_at(1), n1S, nqS, s_tab, s_v, gc);
  float2 prev = X0, cur = X1, last = X0;
  float acc = 0.f;  // twice the intersection area, about X0
  if constexpr (K == 4) {
    // Every slot is visited (a wavefront mostly runs to its eighth slot
    // anyway); slots at or past nx are masked by selects, not branches, so
    // that the rolling window needs no copies: a masked slot routes a zero
    // gradient with t = 1/den = 0 (its rebuilt point, from a padding code,
    // may be far off or infinite and is never multiplied in).
#pragma unroll
    for (int r = 1; r < CAP; ++r) {
      const bool live = r < m;
      float2 nxt = X0;
      SlotGeom gn = gc;
      if (r + 1 < CAP) {
        const float2 xr = rebuild_slot<K, FIXED, BLOCK>(code_at(r + 1), n1S, nqS, s_tab, s_v, gn);
        const bool has = r + 1 < m;
        nxt = has ? xr : X0;
        const float term = (cur.x - X0.x) * (nxt.y - X0.y) - (cur.y - X0.y) * (nxt.x - X0.x);
        acc += has ? term : 0.f;
      }
      // d(2I)/dX_r = (y_r+1 - y_r-1, x_r-1 - x_r+1)
      route_slot(live ? nxt.y - prev.y : 0.f, live ? prev.x - nxt.x : 0.f, live ? gc.t : 0.f,
                 live ? gc.idn : 0.f, gc.oa, gc.ob, gc.oc, gc.od, s_v, s_g);
      last = live ? cur : last;
      prev = cur;
      cur = nxt;
      gc = gn;
    }
  } else {
    // sixteen slots, of which a wavefront's polygons use far fewer: stop at
    // the longest (branches, at the price of copies of the rolling window)
#pragma unroll
    for (int r = 1; r < CAP; ++r) {
      if (r < m) {
        float2 nxt = X0;
        SlotGeom gn = gc;
        if (r + 1 < CAP && r + 1 < m) {
          nxt = rebuild_slot<K, FIXED, BLOCK>(code_at(r + 1), n1S, nqS, s_tab, s_v, gn);
          acc += (cur.x - X0.x) * (nxt.y - X0.y) - (cur.y - X0.y) * (nxt.x - X0.x);
        }
        route_slot(nxt.y - prev.y, prev.x - nxt.x, gc.t, gc.idn, gc.oa, gc.ob, gc.oc, gc.od, s_v,
                   s_g);
        last = cur;
        prev = cur;
        cur = nxt;
        gc = gn;
      }
    }
  }
  if (m > 0) route_slot(X1.y - last.y, last.x - X1.x, g0.t, g0.idn, g0.oa, g0.ob, g0.oc, g0.od,
                        s_v, s_g);
  const float inter = m >= 3 ? 0.5f * acc : 0.f;
  thin = m >= 3 && (thin_pre || (TINY && F2 > kThinInter * inter));

  // scalar factors (zero where the IoU is constant: empty, non-positive union)
  float gI = 0.f, gA1 = 0.f, gA2 = 0.f;
  gz1 = make_float2(0.f, 0.f);
  gz2 = make_float2(0.f, 0.f);
  if (!Z3) {
    const float u = a1 + a2 - inter;
    if (m >= 3 && u > 0.f) {
      const float iu = fast_rcp(u);
      const float giu2 = g * iu * iu;
      gI = giu2 * (a1 + a2);
      gA1 = -giu2 * inter;
      gA2 = gA1;
    }
  } else {
    const float h1 = hi1 - lo1, h2 = hi2 - lo2;
    const float hz = fminf(hi1, hi2) - fmaxf(lo1, lo2);
    const float v = inter * hz, v1 = a1 * h1, v2 = a2 * h2, u = v1 + v2 - v;
    if (m >= 3 && hz > 0.f && u > 0.f) {
      const float iu = fast_rcp(u);
      const float giu2 = g * iu * iu;
      const float gV = giu2 * (v1 + v2);
      const float gV1 = -giu2 * v;
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

  // read back: dL/dv = gI / 2 * (routed shoelace terms) + gA * dA/dv, with
  // dA/dv = (y+ - y-, x- - x+) / 2 over the polygon's own neighbours
  const float hI = 0.5f * gI, h1a = 0.5f * gA1, h2a = 0.5f * gA2;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float2 pn, pp, qn, qp;
    if (FIXED) {
      pn = make_float2(lpx[(k + 1) % K], lpy[(k + 1) % K]);
      pp = make_float2(lpx[(k + K - 1) % K], lpy[(k + K - 1) % K]);
      qn = make_float2(lqx[(k + 1) % K], lqy[(k + 1) % K]);
      qp = make_float2(lqx[(k + K - 1) % K], lqy[(k + K - 1) % K]);
    } else {
      const int kn1 = next_idx<K, FIXED>(k, n1), kp1 = k == 0 ? n1 - 1 : k - 1;
      const int kn2 = next_idx<K, FIXED>(k, n2), kp2 = k == 0 ? n2 - 1 : k - 1;
      pn = s_v[kn1 * BLOCK];
      pp = s_v[kp1 * BLOCK];
      qn = s_v[(K + kn2) * BLOCK];
      qp = s_v[(K + kp2) * BLOCK];
    }
    const float2 tp = s_g[k * BLOCK], tq = s_g[(K + k) * BLOCK];
    gP[k] = (FIXED || k < n1) ? make_float2(fmaf(hI, tp.x, h1a * (pn.y - pp.y)),
                                            fmaf(hI, tp.y, h1a * (pp.x - pn.x)))
                              : make_float2(0.f, 0.f);
    gQ[k] = (FIXED || k < n2) ? make_float2(fmaf(hI, tq.x, h2a * (qn.y - qp.y)),
                                            fmaf(hI, tq.y, h2a * (qp.x - qn.x)))
                              : make_float2(0.f, 0.f);
  }
}

// Backward of one pair's intersection polygon: the gradient, with respect to
// both polygons, of sum_r <G[r], X_r> over the nx saved vertices, each
// rebuilt from its code and routed like the IoU backward's (no predicates,
// no sort).  Buffers as in pair_backward.
template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ void pair_vertex_backward(const Poly<K>& P, int n1, const Poly<K>& Q,
                                                     int n2, int nx,
                                                     const uint32_t (&codes)[K / 2],
                                                     const float2 (&G)[2 * K],
                                                     float2* __restrict__ s_v,
                                                     float2* __restrict__ s_g,
                                                     const uint2* __restrict__ s_tab,
                                                     float2 (&gP)[K], float2 (&gQ)[K]) {
  constexpr int CAP = 2 * K;
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  const float ox = P.x[0], oy = P.y[0];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s_v[k * BLOCK] = make_float2(P.x[k] - ox, P.y[k] - oy);
    s_v[(K + k) * BLOCK] = make_float2(Q.x[k] - ox, Q.y[k] - oy);
    s_g[k * BLOCK] = make_float2(0.f, 0.f);
    s_g[(K + k) * BLOCK] = make_float2(0.f, 0.f);
  }
  const int m = min(nx, CAP);
  constexpr uint32_t S = BLOCK * sizeof(float2);
  const uint32_t n1S = (uint32_t)n1 * S, nqS = (uint32_t)(K + n2) * S;
#pragma unroll
  for (int r = 0; r < CAP; ++r) {
    if (r < m) {
      const uint32_t c = (codes[r >> 2] >> ((r & 3) * 8)) & 0xffu;
      uint32_t oa, ob, oc, od;
      slot_offsets<K, FIXED, BLOCK>(c, n1S, nqS, s_tab, oa, ob, oc, od);
      float t, idn;
      (void)slot_vertex(oa, ob, oc, od, s_v, t, idn);
      route_slot(G[r].x, G[r].y, t, idn, oa, ob, oc, od, s_v, s_g);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    gP[k] = (FIXED || k < n1) ? s_g[k * BLOCK] : make_float2(0.f, 0.f);
    gQ[k] = (FIXED || k < n2) ? s_g[(K + k) * BLOCK] : make_float2(0.f, 0.f);
  }
}

// Shoelace area of one polygon (Sec. III) about its first vertex, and its
// gradient dA/dv_k = (y_k+1 - y_k-1, x_k-1 - x_k+1) / 2 (cyclic neighbours;
// padded slots get 0).
template <int K, bool FIXED>
__device__ __forceinline__ float poly_area(const Poly<K>& P, int n) {
  if (FIXED) n = K;
  float s = 0.f;
#pragma unroll
  for (int k = 1; k + 1 < K; ++k) {
    if (FIXED || k + 1 < n) {
      const float ux = P.x[k] - P.x[0], uy = P.y[k] - P.y[0];
      const float vx = P.x[k + 1] - P.x[0], vy = P.y[k + 1] - P.y[0];
      s += ux * vy - uy * vx;
    }
  }
  return 0.5f * s;
}

template <int K, bool FIXED>
__device__ __forceinline__ void poly_area_grad(const Poly<K>& P, int n, float g, float2 (&gv)[K]) {
  if (FIXED) n = K;
  const float h = 0.5f * g;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int kn = FIXED ? (k + 1) % K : (k + 1 < n ? k + 1 : 0);
    const int kp = FIXED ? (k + K - 1) % K : (k == 0 ? n - 1 : k - 1);
    float pnx = P.x[0], pny = P.y[0], ppx = P.x[0], ppy = P.y[0];
#pragma unroll
    for (int t = 0; t < K; ++t) {  // select the neighbours (static when FIXED)
      if (t == kn) {
        pnx = P.x[t];
        pny = P.y[t];
      }
      if (t == kp) {
        ppx = P.x[t];
        ppy = P.y[t];
      }
    }
    gv[k] = (FIXED || k < n) ? make_float2(h * (pny - ppy), h * (ppx - pnx)) : make_float2(0.f, 0.f);
  }
}

// ---------------------------------------------------------------------------
// fp64 rebuild of ill-conditioned pairs (thin polygons, tiny intersections).
// The pair's polygons are staged, as their fp32 values, in the lane's column
// of a [2K][BLOCK] float2 LDS buffer: P in slots 0..K-1, Q in K..2K-1.  Every
// difference of two fp32 values and every product of two such differences is
// exact in fp64, so the rebuilt vertices carry one rounding each; the codes
// (exact on both sides) fix the structure.  Rare lanes: runtime loops, few
// registers.

// The ordered codes as values the compiler cannot trace back to their
// array: the selects of code_of then stay selects between registers (a
// select between two loads from one array would become a load at a dynamic
// index, which puts the array, and the struct around it, in scratch memory).
template <int K>
struct Codes {
  uint32_t w[K / 2];
  __device__ __forceinline__ explicit Codes(const uint32_t (&codes)[K / 2]) {
#pragma unroll
    for (int k = 0; k < K / 2; ++k) {
      w[k] = codes[k];
      asm volatile("" : "+v"(w[k]));
    }
  }
};

// Code r of the ordered list (a dynamic index: shifts of 64-bit words).
template <int K>
__device__ __forceinline__ uint32_t code_of(const Codes<K>& c, int r) {
  const uint64_t lo = (uint64_t)c.w[0] | ((uint64_t)c.w[1] << 32);
  if constexpr (K == 4) {
    return (uint32_t)(lo >> (8 * (r & 7))) & 0xffu;
  } else {
    const uint64_t hi = (uint64_t)c.w[2] | ((uint64_t)c.w[3] << 32);
    return (uint32_t)((r < 8 ? lo : hi) >> (8 * (r & 7))) & 0xffu;
  }
}

// Intersection vertex of code c relative to (ox, oy): a polygon vertex, or
// the crossing X = A + t (B - A), t = cross(C - A, D - C) / cross(B - A,
// D - C), with its slots and t, 1 / den kept for the chain rule.
struct Vert64 {
  double x, y, t, idn;
  int ia, ib, ic, id;
};

template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ Vert64 vertex64(uint32_t c, int n1, int n2,
                                           const float2* __restrict__ col, double ox, double oy) {
  Vert64 v;
  code_slots<K, FIXED>(c, n1, n2, v.ia, v.ib, v.ic, v.id);
  const float2 a = col[v.ia * BLOCK], b = col[v.ib * BLOCK];
  const float2 cc = col[v.ic * BLOCK], d = col[v.id * BLOCK];
  const double ex = (double)b.x - (double)a.x, ey = (double)b.y - (double)a.y;
  const double fx = (double)d.x - (double)cc.x, fy = (double)d.y - (double)cc.y;
  const double wx = (double)cc.x - (double)a.x, wy = (double)cc.y - (double)a.y;
  const double den = ex * fy - ey * fx;
  v.idn = den != 0.0 ? 1.0 / den : 0.0;
  v.t = (wx * fy - wy * fx) * v.idn;
  v.x = ((double)a.x - ox) + v.t * ex;
  v.y = ((double)a.y - oy) + v.t * ey;
  return v;
}

// Area of the polygon in slots 0..n-1 of a column (about its vertex 0).
template <int BLOCK>
__device__ __forceinline__ double area64(const float2* __restrict__ col, int n) {
  const double x0 = col[0].x, y0 = col[0].y;
  double s = 0.0;
  for (int k = 1; k + 1 < n; ++k) {
    const float2 u = col[k * BLOCK], w = col[(k + 1) * BLOCK];
    s += ((double)u.x - x0) * ((double)w.y - y0) - ((double)u.y - y0) * ((double)w.x - x0);
  }
  return 0.5 * s;
}

// Step 5 of the forward: the intersection's and the polygons' areas in fp64,
// each rounded once.
template <int K, bool FIXED, int BLOCK>
__device__ __forceinline__ void thin_areas64(int m, const uint32_t (&codes)[K / 2], int n1, int n2,
                                             const float2* __restrict__ col, float& inter,
                                             float& a1, float& a2) {
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  const Codes<K> cw(codes);
  const double ox = col[0].x, oy = col[0].y;
  double acc = 0.0, x0 = 0.0, y0 = 0.0, xp = 0.0, yp = 0.0;
  for (int r = 0; r < m; ++r) {
    const Vert64 v = vertex64<K, FIXED, BLOCK>(code_of<K>(cw, r), n1, n2, col, ox, oy);
    if (r == 0) {
      x0 = v.x;
      y0 = v.y;
    } else if (r >= 2) {
      acc += (xp - x0) * (v.y - y0) - (yp - y0) * (v.x - x0);
    }
    xp = v.x;
    yp = v.y;
  }
  inter = m >= 3 ? (float)(0.5 * acc) : 0.f;
  a1 = (float)area64<BLOCK>(col, n1);
  a2 = (float)area64<BLOCK>(col + K * BLOCK, n2);
}

// Chain rule of one vertex for d(2I)/dX = (Gx, Gy), as route_slot, in fp64,
// added into the column's fp32 accumulators (each receives a few terms
// computed in fp64; their sum's rounding is relative to the gradient).
template <int BLOCK>
__device__ __forceinline__ void route64(double Gx, double Gy, const Vert64& v,
                                        const float2* __restrict__ col, float2* __restrict__ acc) {
  auto add = [&](int s, double x, double y) {
    float2 t = acc[s * BLOCK];
    t.x = (float)((double)t.x + x);
    t.y = (float)((double)t.y + y);
    acc[s * BLOCK] = t;
  };
  if (v.ia == v.ib) {  // a polygon vertex: its own slot takes the gradient
    add(v.ia, Gx, Gy);
    return;
  }
  const float2 a = col[v.ia * BLOCK], b = col[v.ib * BLOCK];
  const float2 cc = col[v.ic * BLOCK], d = col[v.id * BLOCK];
  const double ex = (double)b.x - (double)a.x, ey = (double)b.y - (double)a.y;
  const double fx = (double)d.x - (double)cc.x, fy = (double)d.y - (double)cc.y;
  const double wx = (double)cc.x - (double)a.x, wy = (double)cc.y - (double)a.y;
  const double gt = Gx * ex + Gy * ey;
  const double gN = gt * v.idn;
  const double gD = -gN * v.t;
  const double gex = v.t * Gx + gD * fy, gey = v.t * Gy - gD * fx;
  const double gfx = -gN * wy - gD * ey, gfy = gN * wx + gD * ex;
  const double gwx = gN * fy, gwy = -gN * fx;
  add(v.ib, gex, gey);
  add(v.ic, gwx - gfx, gwy - gfy);
  add(v.id, gfx, gfy);
  add(v.ia, Gx - gex - gwx, Gy - gey - gwy);
}

// The backward of pair_backward, in fp64 (polygons staged in s_v as above;
// s_g is overwritten): the same outputs, for the lanes it flags `thin`.
template <int K, bool FIXED, bool Z3, int BLOCK>
__device__ __forceinline__ void pair_backward64(int n1, int n2, float g, int nx,
                                                const uint32_t (&codes)[K / 2], float lo1,
                                                float hi1, float lo2, float hi2,
                                                const float2* __restrict__ s_v,
                                                float2* __restrict__ s_g, float2 (&gP)[K],
                                                float2 (&gQ)[K], float2& gz1, float2& gz2) {
  constexpr int CAP = 2 * K;
  if (FIXED) {
    n1 = K;
    n2 = K;
  }
  const int m = min(nx, CAP);
  const Codes<K> cw(codes);
#pragma unroll
  for (int k = 0; k < CAP; ++k) s_g[k * BLOCK] = make_float2(0.f, 0.f);
  const double ox = s_v[0].x, oy = s_v[0].y;
  // one pass with a rolling window: d(2I)/dX_r = (y_r+1 - y_r-1, x_r-1 - x_r+1)
  double acc = 0.0;
  if (m >= 3) {
    const Vert64 first = vertex64<K, FIXED, BLOCK>(code_of<K>(cw, 0), n1, n2, s_v, ox, oy);
    const Vert64 last = vertex64<K, FIXED, BLOCK>(code_of<K>(cw, m - 1), n1, n2, s_v, ox, oy);
    double px = last.x, py = last.y;
    Vert64 cur = first;
    for (int r = 0; r < m; ++r) {
      const Vert64 nxt =
          r + 1 < m ? vertex64<K, FIXED, BLOCK>(code_of<K>(cw, r + 1), n1, n2, s_v, ox, oy)
                    : first;
      route64<BLOCK>(nxt.y - py, px - nxt.x, cur, s_v, s_g);
      acc += (cur.x - first.x) * (nxt.y - first.y) - (cur.y - first.y) * (nxt.x - first.x);
      px = cur.x;
      py = cur.y;
      cur = nxt;
    }
  }
  const double inter = m >= 3 ? 0.5 * acc : 0.0;
  const double a1 = area64<BLOCK>(s_v, n1), a2 = area64<BLOCK>(s_v + K * BLOCK, n2);

  // scalar factors, as in pair_backward
  double gI = 0.0, gA1 = 0.0, gA2 = 0.0;
  double z1x = 0.0, z1y = 0.0, z2x = 0.0, z2y = 0.0;
  if (!Z3) {
    const double u = a1 + a2 - inter;
    if (m >= 3 && u > 0.0) {
      const double giu2 = (double)g / (u * u);
      gI = giu2 * (a1 + a2);
      gA1 = -giu2 * inter;
      gA2 = gA1;
    }
  } else {
    const double h1 = (double)hi1 - lo1, h2 = (double)hi2 - lo2;
    const double hz = (double)fminf(hi1, hi2) - (double)fmaxf(lo1, lo2);
    const double v = inter * hz, v1 = a1 * h1, v2 = a2 * h2, u = v1 + v2 - v;
    if (m >= 3 && hz > 0.0 && u > 0.0) {
      const double giu2 = (double)g / (u * u);
      const double gV = giu2 * (v1 + v2), gV1 = -giu2 * v;
      gI = gV * hz;
      const double ghz = gV * inter;
      gA1 = gV1 * h1;
      gA2 = gV1 * h2;
      const double gh1 = gV1 * a1, gh2 = gV1 * a2;
      z1x = -gh1;
      z1y = gh1;
      z2x = -gh2;
      z2y = gh2;
      if (hi1 <= hi2) z1y += ghz; else z2y += ghz;
      if (lo1 >= lo2) z1x -= ghz; else z2x -= ghz;
    }
  }
  gz1 = make_float2((float)z1x, (float)z1y);
  gz2 = make_float2((float)z2x, (float)z2y);

  // read back: dL/dv = gI / 2 * (routed terms) + gA / 2 * (y+ - y-, x- - x+)
  const double hI = 0.5 * gI, h1a = 0.5 * gA1, h2a = 0.5 * gA2;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int kn1 = next_idx<K, FIXED>(k, n1), kp1 = k == 0 ? n1 - 1 : k - 1;
    const int kn2 = next_idx<K, FIXED>(k, n2), kp2 = k == 0 ? n2 - 1 : k - 1;
    const float2 pn = s_v[kn1 * BLOCK], pp = s_v[kp1 * BLOCK];
    const float2 qn = s_v[(K + kn2) * BLOCK], qp = s_v[(K + kp2) * BLOCK];
    const float2 tp = s_g[k * BLOCK], tq = s_g[(K + k) * BLOCK];
    gP[k] = (FIXED || k < n1)
                ? make_float2((float)(hI * tp.x + h1a * ((double)pn.y - (double)pp.y)),
                              (float)(hI * tp.y + h1a * ((double)pp.x - (double)pn.x)))
                : make_float2(0.f, 0.f);
    gQ[k] = (FIXED || k < n2)
                ? make_float2((float)(hI * tq.x + h2a * ((double)qn.y - (double)qp.y)),
                              (float)(hI * tq.y + h2a * ((double)qp.x - (double)qn.x)))
                : make_float2(0.f, 0.f);
  }
}

// Stages a pair's polygons (fp32 values) into a lane column for the fp64
// rebuild: P in slots 0..K-1, Q in K..2K-1.
template <int K, int BLOCK>
__device__ __forceinline__ void stage_pair(float2* __restrict__ col, const Poly<K>& P,
                                           const Poly<K>& Q) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    col[k * BLOCK] = make_float2(P.x[k], P.y[k]);
    col[(K + k) * BLOCK] = make_float2(Q.x[k], Q.y[k]);
  }
}

}  // namespace dgal
