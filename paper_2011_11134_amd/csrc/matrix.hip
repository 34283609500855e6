// matrix.hip -- IoU matrices (one block a.count x b.count, or ragged segments
// such as per-scene self-pairs of 3D boxes, Sec. IV-A case study at scale) and
// their backward from the compact list of non-empty pairs.
//
// Forward schedule: the output is cut into TILE x TILE tiles; a persistent
// grid walks the tile space of all segments (a prefix sum of tiles per
// segment, computed on the device so the call is graph-capturable).  For one
// tile a workgroup stages the TILE row boxes and TILE column boxes in LDS with
// a bounding circle each, culls every pair whose circles (or z-extents) are
// apart, compacts the survivors into an LDS list and runs the exact pair
// forward on them with all lanes busy; the finished tile leaves LDS as
// coalesced row segments.
#include <type_traits>

#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

constexpr int kTile = 64;          // rows and columns per tile
constexpr int kMatBlock = 256;     // threads per workgroup
constexpr int kMaxSeg = DGAL_MAX_SEGMENTS;

struct MatArgs {
  PolyArgs a, b;
  const int64_t* a_off;  // NULL => one segment
  const int64_t* b_off;
  const int64_t* out_off;
  const int64_t* tile_prefix;  // [nseg+1] (segmented) from k_seg_prep
  int nseg;
  int64_t single_tiles;  // tile count of the single segment
  int self_pairs;
  float* iou;
  int64_t out_size;
  // saved list (pair_id == nullptr => forward only)
  int64_t* pair_id;
  uint8_t* s_nx;
  uint8_t* s_flags;
  int64_t capacity;
  int64_t* count;
  int cap;
  int* err;
};

struct Segment {
  int64_t a0, b0, na, nb, out0;
  bool ok;
};

__device__ __forceinline__ Segment load_segment(const MatArgs& m, int s) {
  Segment g;
  if (m.a_off == nullptr) {
    g.a0 = 0;
    g.b0 = 0;
    g.na = m.a.count;
    g.nb = m.b.count;
    g.out0 = 0;
    g.ok = true;
    return g;
  }
  const int64_t a0 = m.a_off[s], a1 = m.a_off[s + 1], b0 = m.b_off[s], b1 = m.b_off[s + 1];
  const int64_t o0 = m.out_off[s];
  g.a0 = a0;
  g.b0 = b0;
  g.na = a1 - a0;
  g.nb = b1 - b0;
  g.out0 = o0;
  g.ok = a0 >= 0 && a1 >= a0 && a1 <= m.a.count && b0 >= 0 && b1 >= b0 && b1 <= m.b.count &&
         o0 >= 0 && o0 <= m.out_size && g.na * g.nb <= m.out_size - o0 &&
         (!m.self_pairs || (a0 == b0 && a1 == b1));
  if (s > 0) {  // blocks are laid out in segment order without overlap
    const int64_t pna = m.a_off[s] - m.a_off[s - 1], pnb = m.b_off[s] - m.b_off[s - 1];
    g.ok = g.ok && o0 >= m.out_off[s - 1] + pna * pnb;
  }
  return g;
}

// Tile prefix over segments (one workgroup): tile_prefix[s] = tiles of
// segments < s.  Rejected segments get no tiles and raise kErrSegment.
__global__ __launch_bounds__(256) void k_seg_prep(MatArgs m, int64_t* tile_prefix) {
  __shared__ int64_t part[256];
  const int tid = threadIdx.x;
  const int per = (m.nseg + 255) / 256;
  const int s0 = tid * per, s1 = min(m.nseg, s0 + per);
  int64_t sum = 0;
  for (int s = s0; s < s1; ++s) {
    const Segment g = load_segment(m, s);
    if (!g.ok) {
      atomicOr(m.err, kErrSegment);
      continue;
    }
    sum += ((g.na + kTile - 1) / kTile) * ((g.nb + kTile - 1) / kTile);
  }
  part[tid] = sum;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive scan
    const int64_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t run = tid > 0 ? part[tid - 1] : 0;
  if (tid == 0) tile_prefix[0] = 0;
  for (int s = s0; s < s1; ++s) {
    const Segment g = load_segment(m, s);
    if (g.ok) run += ((g.na + kTile - 1) / kTile) * ((g.nb + kTile - 1) / kTile);
    tile_prefix[s + 1] = run;
  }
}

// Staged box: vertices (local K slots), count, bounding circle, z-extent.
template <int K>
struct BoxLds {
  float x[K][kTile];
  float y[K][kTile];
  float cx[kTile], cy[kTile], r[kTile];
  float lo[kTile], hi[kTile];
  uint8_t n[kTile];
};

template <int K, bool FIXED, bool Z3>
__device__ __forceinline__ void stage_box(const PolyArgs& p, int64_t idx, bool valid, int t,
                                          BoxLds<K>& s) {
  Poly<K> P;
  int n = K;
  if (valid) {
    n = FIXED ? K : poly_count(p.nv, idx, p.kmax);
    load_poly<K, FIXED>(p.xy, idx, p.kmax, p.vec4, n, P);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      P.x[k] = 0.f;
      P.y[k] = 0.f;
    }
  }
  float cx = 0.f, cy = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cx += P.x[k];
    cy += P.y[k];
    s.x[k][t] = P.x[k];
    s.y[k][t] = P.y[k];
  }
  // padded slots repeat vertex 0, so the mean over K slots is inside the hull
  cx *= 1.0f / K;
  cy *= 1.0f / K;
  float r2 = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float dx = P.x[k] - cx, dy = P.y[k] - cy;
    r2 = fmaxf(r2, dx * dx + dy * dy);
  }
  s.cx[t] = cx;
  s.cy[t] = cy;
  // inflated by 1e-5 relative: covers the rounding of the centre, the
  // distances and the square root, so the circle contains the polygon
  s.r[t] = valid ? sqrtf(r2) * 1.00001f + 1e-30f : -1.f;
  s.n[t] = (uint8_t)n;
  if (Z3) {
    s.lo[t] = valid ? p.zlo[idx] : 0.f;
    s.hi[t] = valid ? p.zhi[idx] : 0.f;
  }
}

template <int K, bool FIXED, bool Z3>
__global__ __launch_bounds__(kMatBlock) void k_matrix_fwd(MatArgs m) {
  constexpr int CAP = 2 * K;
  __shared__ BoxLds<K> sa, sb;
  __shared__ float s_out[kTile][kTile + 1];
  __shared__ uint16_t s_surv[kTile * kTile];
  __shared__ int s_nsurv;
  __shared__ float2 s_pt[CAP * kMatBlock];
  __shared__ uint8_t s_cd[CAP * kMatBlock];
  const int tid = threadIdx.x;
  const bool segmented = m.a_off != nullptr;
  const int64_t total = segmented ? m.tile_prefix[m.nseg] : m.single_tiles;

  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    // locate the tile's segment
    int s = 0;
    int64_t lt = t;
    if (segmented) {
      int lo = 0, hi = m.nseg - 1;  // last s with prefix[s] <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m.tile_prefix[mid] <= t) lo = mid; else hi = mid - 1;
      }
      s = lo;
      lt = t - m.tile_prefix[s];
    }
    const Segment g = load_segment(m, s);
    if (!g.ok) continue;  // unreachable: rejected segments own no tiles
    const int64_t tcols = (g.nb + kTile - 1) / kTile;
    const int64_t r0 = (lt / tcols) * kTile, c0 = (lt % tcols) * kTile;
    const int nr = (int)min((int64_t)kTile, g.na - r0), nc = (int)min((int64_t)kTile, g.nb - c0);

    __syncthreads();  // previous tile done with LDS
    if (tid < kTile) {
      stage_box<K, FIXED, Z3>(m.a, g.a0 + r0 + tid, tid < nr, tid, sa);
    } else if (tid < 2 * kTile) {
      stage_box<K, FIXED, Z3>(m.b, g.b0 + c0 + (tid - kTile), tid - kTile < nc, tid - kTile, sb);
    }
    if (tid == 0) s_nsurv = 0;
    __syncthreads();

    // cull: 16 pairs per thread, rows tid/16*... (row-major over the tile)
#pragma unroll 4
    for (int q = tid; q < kTile * kTile; q += kMatBlock) {
      const int r = q / kTile, c = q % kTile;
      float v = 0.f;
      bool surv = false;
      if (r < nr && c < nc) {
        const float dx = sa.cx[r] - sb.cx[c], dy = sa.cy[r] - sb.cy[c];
        const float rr = sa.r[r] + sb.r[c];
        surv = dx * dx + dy * dy <= rr * rr * 1.00001f;
        if (Z3) surv &= fminf(sa.hi[r], sb.hi[c]) > fmaxf(sa.lo[r], sb.lo[c]);
        if (m.self_pairs && g.a0 + r0 + r == g.b0 + c0 + c) {
          surv = false;
          v = 1.f;
        }
      }
      s_out[r][c] = v;
      if (surv) {
        const int slot = atomicAdd(&s_nsurv, 1);
        s_surv[slot] = (uint16_t)q;
      }
    }
    __syncthreads();

    // exact forward on the survivors, all lanes busy
    const int ns = s_nsurv;
    for (int k = tid; k < ns; k += kMatBlock) {
      const int q = s_surv[k];
      const int r = q / kTile, c = q % kTile;
      Poly<K> P, Q;
#pragma unroll
      for (int v = 0; v < K; ++v) {
        P.x[v] = sa.x[v][r];
        P.y[v] = sa.y[v][r];
        Q.x[v] = sb.x[v][c];
        Q.y[v] = sb.y[v][c];
      }
      const int n1 = sa.n[r], n2 = sb.n[c];
      PairResult<K> res;
      pair_forward<K, FIXED, kMatBlock>(P, n1, Q, n2, s_pt + tid, s_cd + tid, res);
      float v;
      if (Z3) {
        v = iou_3d(res.inter, res.a1, res.a2, res.m, sa.lo[r], sa.hi[r], sb.lo[c], sb.hi[c]);
      } else {
        v = iou_2d(res.inter, res.a1, res.a2, res.m);
      }
      s_out[r][c] = v;
      if (res.overflow) atomicOr(m.err, kErrCapacity);
      if (m.pair_id != nullptr && res.m > 0) {
        const unsigned long long e = atomicAdd(reinterpret_cast<unsigned long long*>(m.count), 1ull);
        if ((int64_t)e < m.capacity) {
          m.pair_id[e] = g.out0 + (r0 + r) * g.nb + (c0 + c);
          m.s_nx[e] = (uint8_t)res.m;
          uint8_t* row = m.s_flags + (int64_t)e * m.cap;
#pragma unroll
          for (int b = 0; b < CAP; ++b)
            if (b < m.cap) row[b] = (uint8_t)(res.codes[b >> 2] >> ((b & 3) * 8));
        } else {
          atomicOr(m.err, kErrCapacity);
        }
      }
    }
    __syncthreads();

    // write the tile: each row segment is contiguous in the output
    float* base = m.iou + g.out0 + r0 * g.nb + c0;
    for (int q = tid; q < kTile * kTile; q += kMatBlock) {
      const int r = q / kTile, c = q % kTile;
      if (r < nr && c < nc) base[(int64_t)r * g.nb + c] = s_out[r][c];
    }
  }
}

// Zero-fills n floats (gradient outputs before atomic accumulation).
__global__ void k_fill_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// Resets the saved-list counter (a kernel, not a memset, so that graph
// replays see the reset).
__global__ void k_reset_count(int64_t* count) { *count = 0; }

struct MatBwdArgs {
  PolyArgs a, b;
  const int64_t* a_off;
  const int64_t* b_off;
  const int64_t* out_off;
  int nseg;
  int self_pairs;
  const float* grad;
  int64_t out_size;  // elements of grad
  const int64_t* pair_id;
  const uint8_t* s_nx;
  const uint8_t* s_flags;
  int64_t capacity;
  const int64_t* count;
  int cap;
  float* ga_xy;
  float* gb_xy;  // == ga_xy when self_pairs
  float* ga_z;
  float* gb_z;
};

template <int K, bool FIXED, bool Z3>
__global__ __launch_bounds__(128) void k_matrix_bwd(MatBwdArgs m) {
  constexpr int BLOCK = 128;
  constexpr int CAP = 2 * K;
  __shared__ float2 s_v[CAP * BLOCK];
  __shared__ float2 s_g[CAP * BLOCK];
  const int tid = threadIdx.x;
  int64_t n = *m.count;
  n = n < m.capacity ? n : m.capacity;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + tid; e < n; e += (int64_t)gridDim.x * BLOCK) {
    const int64_t pid = m.pair_id[e];
    if (pid < 0 || pid >= m.out_size) continue;  // not written by a forward on these shapes
    int64_t a0 = 0, b0 = 0, nb = m.b.count, local = pid;
    if (m.a_off != nullptr) {
      int lo = 0, hi = m.nseg - 1;  // last s with out_off[s] <= pid and a non-empty block
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m.out_off[mid] <= pid) lo = mid; else hi = mid - 1;
      }
      // empty segments share their out_off with the next one: step back to
      // the last segment whose block holds pid
      int s = lo;
      while (s > 0 && (m.b_off[s + 1] - m.b_off[s]) * (m.a_off[s + 1] - m.a_off[s]) == 0) --s;
      a0 = m.a_off[s];
      b0 = m.b_off[s];
      nb = m.b_off[s + 1] - b0;
      local = pid - m.out_off[s];
    }
    if (nb <= 0) continue;
    const int64_t ia = a0 + local / nb, ib = b0 + local % nb;
    if (ia < 0 || ia >= m.a.count || ib < 0 || ib >= m.b.count) continue;
    const int n1 = FIXED ? K : poly_count(m.a.nv, ia, m.a.kmax);
    const int n2 = FIXED ? K : poly_count(m.b.nv, ib, m.b.kmax);
    Poly<K> P, Q;
    load_poly<K, FIXED>(m.a.xy, ia, m.a.kmax, m.a.vec4, n1, P);
    load_poly<K, FIXED>(m.b.xy, ib, m.b.kmax, m.b.vec4, n2, Q);
    uint32_t codes[K / 2];
#pragma unroll
    for (int w = 0; w < K / 2; ++w) codes[w] = 0xffffffffu;
    const uint8_t* row = m.s_flags + e * (int64_t)m.cap;
#pragma unroll
    for (int k = 0; k < CAP; ++k) {
      if (k < m.cap) {
        const uint32_t c = row[k];
        codes[k >> 2] = (codes[k >> 2] & ~(0xffu << ((k & 3) * 8))) | (c << ((k & 3) * 8));
      }
    }
    float lo1 = 0.f, hi1 = 0.f, lo2 = 0.f, hi2 = 0.f;
    if (Z3) {
      lo1 = m.a.zlo[ia];
      hi1 = m.a.zhi[ia];
      lo2 = m.b.zlo[ib];
      hi2 = m.b.zhi[ib];
    }
    float2 gP[K], gQ[K], gz1, gz2;
    pair_backward<K, FIXED, Z3, BLOCK>(P, n1, Q, n2, m.grad[pid], (int)m.s_nx[e], codes, lo1, hi1,
                                       lo2, hi2, s_v + tid, s_g + tid, gP, gQ, gz1, gz2);
    float* oa = m.ga_xy + ia * (int64_t)m.a.kmax * 2;
    float* ob = m.gb_xy + ib * (int64_t)m.b.kmax * 2;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < n1 && k < m.a.kmax) {
        unsafeAtomicAdd(oa + 2 * k, gP[k].x);
        unsafeAtomicAdd(oa + 2 * k + 1, gP[k].y);
      }
      if (k < n2 && k < m.b.kmax) {
        unsafeAtomicAdd(ob + 2 * k, gQ[k].x);
        unsafeAtomicAdd(ob + 2 * k + 1, gQ[k].y);
      }
    }
    if (Z3) {
      unsafeAtomicAdd(m.ga_z + 2 * ia, gz1.x);
      unsafeAtomicAdd(m.ga_z + 2 * ia + 1, gz1.y);
      unsafeAtomicAdd(m.gb_z + 2 * ib, gz2.x);
      unsafeAtomicAdd(m.gb_z + 2 * ib + 1, gz2.y);
    }
  }
}

namespace {

template <int K, bool FIXED, bool Z3>
void launch_fwd(const MatArgs& m, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_matrix_fwd<K, FIXED, Z3>), dim3(grid), dim3(kMatBlock), 0, s, m);
}

template <int K, bool FIXED, bool Z3>
void launch_bwd(const MatBwdArgs& m, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_matrix_bwd<K, FIXED, Z3>), dim3(grid), dim3(128), 0, s, m);
}

}  // namespace

int matrix_forward(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                   const int64_t* b_off, const int64_t* out_off, int nseg, int self_pairs,
                   float* iou, int64_t out_size, const dgal_saved* saved, hipStream_t stream) {
  if (!valid_polys(a) || !valid_polys(b)) return DGAL_EINVAL;
  if ((a.zlo == nullptr) != (b.zlo == nullptr)) return DGAL_EINVAL;
  const bool segmented = a_off != nullptr;
  if (segmented != (b_off != nullptr) || segmented != (out_off != nullptr)) return DGAL_EINVAL;
  if (segmented && (nseg < 1 || nseg > kMaxSeg)) return DGAL_EINVAL;
  if (self_pairs && !same_polys(a, b)) return DGAL_EINVAL;
  if (out_size < 0) return DGAL_EINVAL;
  if (!segmented && (a.count > 0 && b.count > 0) && out_size / (a.count > 0 ? a.count : 1) < b.count)
    return DGAL_EINVAL;
  if (out_size > 0 && (iou == nullptr || !aligned(iou, 4))) return DGAL_EINVAL;
  if (saved != nullptr) {
    if (saved->pair_id == nullptr || saved->nx == nullptr || saved->xflags == nullptr ||
        saved->count == nullptr || saved->capacity < 0)
      return DGAL_EINVAL;
  }
  if (a.count == 0 && b.count == 0 && !segmented) return DGAL_OK;
  DeviceGuard dg(ctx.device);
  if (!dg.ok) return DGAL_EHIP;
  const int K = (a.kmax <= 4 && b.kmax <= 4) ? 4 : 8;
  MatArgs m;
  m.a = poly_args(a, K);
  m.b = poly_args(b, K);
  m.a_off = a_off;
  m.b_off = b_off;
  m.out_off = out_off;
  m.nseg = segmented ? nseg : 1;
  m.self_pairs = self_pairs;
  m.iou = iou;
  m.out_size = out_size;
  m.pair_id = saved ? saved->pair_id : nullptr;
  m.s_nx = saved ? saved->nx : nullptr;
  m.s_flags = saved ? saved->xflags : nullptr;
  m.capacity = saved ? saved->capacity : 0;
  m.count = saved ? saved->count : nullptr;
  m.cap = a.kmax + b.kmax;
  m.err = ctx.err;
  m.single_tiles = segmented ? 0 : ((a.count + kTile - 1) / kTile) * ((b.count + kTile - 1) / kTile);
  m.tile_prefix = nullptr;
  if (saved) hipLaunchKernelGGL(k_reset_count, dim3(1), dim3(1), 0, stream, saved->count);
  if (segmented) {
    m.tile_prefix = ctx.prefix;
    hipLaunchKernelGGL(k_seg_prep, dim3(1), dim3(256), 0, stream, m, ctx.prefix);
  }
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K;
  const bool z3 = a.zlo != nullptr;
  int grid = ctx.cus * 4;
  if (!segmented && m.single_tiles < grid) grid = (int)(m.single_tiles > 0 ? m.single_tiles : 1);
  if (K == 4) {
    if (fixed) {
      z3 ? launch_fwd<4, true, true>(m, grid, stream) : launch_fwd<4, true, false>(m, grid, stream);
    } else {
      z3 ? launch_fwd<4, false, true>(m, grid, stream) : launch_fwd<4, false, false>(m, grid, stream);
    }
  } else {
    if (fixed) {
      z3 ? launch_fwd<8, true, true>(m, grid, stream) : launch_fwd<8, true, false>(m, grid, stream);
    } else {
      z3 ? launch_fwd<8, false, true>(m, grid, stream) : launch_fwd<8, false, false>(m, grid, stream);
    }
  }
  return hipGetLastError() == hipSuccess ? DGAL_OK : DGAL_EHIP;
}

int matrix_backward(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                    const int64_t* b_off, const int64_t* out_off, int nseg, int self_pairs,
                    const float* grad_iou, int64_t out_size, const dgal_saved* saved,
                    float* grad_a_xy, float* grad_b_xy, float* grad_a_z, float* grad_b_z,
                    hipStream_t stream) {
  if (!valid_polys(a) || !valid_polys(b) || out_size < 0) return DGAL_EINVAL;
  const bool z3 = a.zlo != nullptr;
  if ((a.zlo == nullptr) != (b.zlo == nullptr)) return DGAL_EINVAL;
  const bool segmented = a_off != nullptr;
  if (segmented != (b_off != nullptr) || segmented != (out_off != nullptr)) return DGAL_EINVAL;
  if (segmented && (nseg < 1 || nseg > kMaxSeg)) return DGAL_EINVAL;
  if (self_pairs && !same_polys(a, b)) return DGAL_EINVAL;
  if (saved == nullptr || saved->pair_id == nullptr || saved->nx == nullptr ||
      saved->xflags == nullptr || saved->count == nullptr || saved->capacity < 0)
    return DGAL_EINVAL;
  if (grad_iou == nullptr || grad_a_xy == nullptr) return DGAL_EINVAL;
  if (self_pairs ? (grad_b_xy != nullptr || grad_b_z != nullptr) : (grad_b_xy == nullptr))
    return DGAL_EINVAL;
  if (z3 != (grad_a_z != nullptr)) return DGAL_EINVAL;
  if (!self_pairs && z3 != (grad_b_z != nullptr)) return DGAL_EINVAL;
  DeviceGuard dg(ctx.device);
  if (!dg.ok) return DGAL_EHIP;
  const int K = (a.kmax <= 4 && b.kmax <= 4) ? 4 : 8;
  float* gbx = self_pairs ? grad_a_xy : grad_b_xy;
  float* gbz = self_pairs ? grad_a_z : grad_b_z;
  const int zb = 256;
  auto zero = [&](float* p, int64_t n) {
    if (p != nullptr && n > 0) {
      int64_t blocks = (n + zb - 1) / zb;
      hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(blocks > 4096 ? 4096 : blocks)), dim3(zb), 0,
                         stream, p, n);
    }
  };
  zero(grad_a_xy, a.count * a.kmax * 2);
  if (!self_pairs) zero(grad_b_xy, b.count * b.kmax * 2);
  if (z3) {
    zero(grad_a_z, a.count * 2);
    if (!self_pairs) zero(grad_b_z, b.count * 2);
  }
  MatBwdArgs m;
  m.a = poly_args(a, K);
  m.b = poly_args(b, K);
  m.a_off = a_off;
  m.b_off = b_off;
  m.out_off = out_off;
  m.nseg = segmented ? nseg : 1;
  m.self_pairs = self_pairs;
  m.grad = grad_iou;
  m.out_size = out_size;
  m.pair_id = saved->pair_id;
  m.s_nx = saved->nx;
  m.s_flags = saved->xflags;
  m.capacity = saved->capacity;
  m.count = saved->count;
  m.cap = a.kmax + b.kmax;
  m.ga_xy = grad_a_xy;
  m.gb_xy = gbx;
  m.ga_z = grad_a_z;
  m.gb_z = gbz;
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K;
  const int grid = ctx.cus * 4;
  if (K == 4) {
    if (fixed) {
      z3 ? launch_bwd<4, true, true>(m, grid, stream) : launch_bwd<4, true, false>(m, grid, stream);
    } else {
      z3 ? launch_bwd<4, false, true>(m, grid, stream) : launch_bwd<4, false, false>(m, grid, stream);
    }
  } else {
    if (fixed) {
      z3 ? launch_bwd<8, true, true>(m, grid, stream) : launch_bwd<8, true, false>(m, grid, stream);
    } else {
      z3 ? launch_bwd<8, false, true>(m, grid, stream) : launch_bwd<8, false, false>(m, grid, stream);
    }
  }
  return hipGetLastError() == hipSuccess ? DGAL_OK : DGAL_EHIP;
}

}  // namespace dgal
